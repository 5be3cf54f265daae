"""GPU parity of the O(N) phi^4 path (lat_on_* through the C ABI) with the
FP64 CPU oracle on the same seeded inputs.

Both sides run the same multi-hit Metropolis chain with the same uniforms;
an accept decision could differ only where the acceptance uniform lies
within rounding of exp(-dS) (probability ~1e-16 per hit), so FP64 fields
agree to 1e-12 (max abs over all sites and components) and the accepted-hit
counts agree exactly.  FP32 storage rounds the field after every update:
values agree to 1e-5 except at the rare sites where a decision flipped
(at most 1% of the sites here, typically none)."""
import ctypes

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1310_7087_amd")

TOL64 = 1e-12

# (N, dims, kappa, lambda, h, delta, start, nhit)
CASES = [
    (4, (8, 8, 8, 8), 0.3, 1.0, 0.0, 1.0, O.HOT, 100),
    (1, (6, 4, 10, 2), 0.2, 0.5, 0.1, 1.5, O.COLD, 20),
    (2, (4, 6, 8, 4), -0.1, 0.0, -0.3, 0.8, O.HOT, 10),
    (3, (2, 2, 2, 2), 0.25, 2.0, 0.4, 1.2, O.HOT, 7),
    (4, (10, 2, 4, 6), 0.31, 0.7, 0.05, 0.9, O.COLD, 50),
]


def pair(n, dims, kappa, lam, h, delta, start, nhit, rng=O.RNG_PHILOX, seed=3, storage=0, rng_const=0.5,
         lattice_id=0, block_size=0):
    g = P.ONField(n, dims, kappa, lam, h, delta, storage=storage, rng=rng, rng_const=rng_const, seed=seed,
                  nhit=nhit, lattice_id=lattice_id, start=start, block_size=block_size)
    o = O.ONField(n, dims, kappa, lam, h, delta, rng=rng, rng_const=rng_const, seed=seed, nhit=nhit,
                  lattice_id=lattice_id, start=start)
    return g, o


@pytest.mark.parametrize("case", CASES)
def test_start_and_sweeps_match_oracle(case):
    g, o = pair(*case)
    assert np.array_equal(g.get_field(), o.get_field())  # starts are exact in FP64
    for k in (1, 2):
        g.sweep(k)
        o.sweep(k)
        assert np.abs(g.get_field() - o.get_field()).max() <= TOL64, case
        assert g.acceptance() == o.acceptance()
        assert np.abs(g.measure() - o.measure()).max() <= TOL64
    g.close()


@pytest.mark.parametrize("rng", [O.RNG_RANLUX, O.RNG_MRG32K3A])
@pytest.mark.parametrize("n", [1, 4])
def test_sequential_streams_match_oracle(n, rng):
    g, o = pair(n, (8, 4, 4, 6), 0.28, 0.9, 0.1, 1.1, O.HOT, 30, rng=rng, seed=77)
    assert np.array_equal(g.get_field(), o.get_field())
    g.sweep(2)
    o.sweep(2)
    assert np.abs(g.get_field() - o.get_field()).max() <= TOL64
    assert g.acceptance() == o.acceptance()
    g.close()


def test_constant_generator_walk():
    """The hand-derived walk of the oracle's pins: every site ends at
    (0, -1, -1, -1) after four accepted hits."""
    g = P.ONField(4, (4, 4, 2, 2), 0.0, 0.0, 0.0, 0.5, rng=P.RNG_CONST, rng_const=0.25, nhit=10, start=P.COLD)
    g.sweep(1)
    assert np.array_equal(g.get_field(), np.tile([0.0, -1.0, -1.0, -1.0], (64, 1)))
    assert g.acceptance() == 0.4
    g.close()


@pytest.mark.parametrize("block", [64, 128])
def test_work_group_size_does_not_change_results(block):
    a = P.ONField(4, (6, 4, 10, 2), 0.3, 1.0, 0.2, 1.0, seed=5, nhit=40)
    b = P.ONField(4, (6, 4, 10, 2), 0.3, 1.0, 0.2, 1.0, seed=5, nhit=40, block_size=block)
    a.sweep(3)
    b.sweep(3)
    assert np.array_equal(a.get_field(), b.get_field())
    assert a.acceptance() == b.acceptance()
    a.close()
    b.close()


def test_run_series_equals_stepwise_measurements():
    a = P.ONField(2, (8, 8, 4, 4), 0.2, 0.3, 0.1, 1.2, seed=9, nhit=10)
    b = P.ONField(2, (8, 8, 4, 4), 0.2, 0.3, 0.1, 1.2, seed=9, nhit=10)
    series = a.run(12, 3)
    want = []
    for _ in range(4):
        b.sweep(3)
        want.append(b.measure())
    assert series.shape == (4, 7)
    assert np.array_equal(series, np.array(want))
    assert a.info()["sweeps"] == 12
    a.close()
    b.close()


def test_longer_chain_matches_oracle():
    g, o = pair(4, (8, 8, 8, 8), 0.3, 1.0, 0.0, 1.0, O.HOT, 100, seed=21)
    g.sweep(20)
    o.sweep(20)
    assert np.abs(g.get_field() - o.get_field()).max() <= TOL64
    g.close()


def test_f32_storage_close_to_oracle():
    g, o = pair(4, (8, 8, 8, 8), 0.3, 1.0, 0.0, 1.0, O.HOT, 100, storage=P.F32, seed=4)
    assert np.array_equal(g.get_field(), o.get_field())  # the hot start is exact in FP32
    g.sweep(1)
    o.sweep(1)
    d = np.abs(g.get_field() - o.get_field()).max(axis=1)
    assert (d > 1e-5).mean() <= 0.01
    assert np.median(d) < 1e-6
    m = g.measure() - o.measure()
    assert np.abs(m).max() < 1e-4
    g.close()


def test_set_and_get_field_round_trip():
    g = P.ONField(3, (4, 4, 4, 2), 0.1, 0.2, seed=2, nhit=5)
    phi = np.random.default_rng(0).standard_normal((g.V, 3))
    g.set_field(phi)
    assert np.array_equal(g.get_field(), phi)
    o = O.ONField(3, (4, 4, 4, 2), 0.1, 0.2, seed=2, nhit=5)
    o.set_field(phi)
    g.sweep(2)
    o.sweep(2)
    assert np.abs(g.get_field() - o.get_field()).max() <= TOL64
    g.close()


def test_time_seed_is_reported():
    g = P.ONField(1, (2, 2, 2, 2), 0.1, 0.1, seed=0, nhit=1)
    assert g.info()["seed"] != 0
    g.close()


def test_full_size_o4_32():
    """An O(4) lattice of the paper's Table 1 (32^4, NHIT = 100): one sweep
    from the hot start, every site against the oracle."""
    g, o = pair(4, (32, 32, 32, 32), 0.3, 1.0, 0.0, 1.0, O.HOT, 100, seed=13)
    g.sweep(1)
    o.sweep(1)
    assert np.abs(g.get_field() - o.get_field()).max() <= TOL64
    assert g.acceptance() == o.acceptance()
    assert np.abs(g.measure() - o.measure()).max() <= TOL64
    g.close()


@pytest.mark.parametrize("rng", [P.RNG_PHILOX, P.RNG_RANLUX, P.RNG_MRG32K3A])
def test_checkpoint_continues_the_chain(tmp_path, rng):
    """N sweeps straight equal N/2 + save + load + N/2, bit for bit."""
    a = P.ONField(4, (6, 4, 8, 2), 0.3, 1.0, 0.1, 0.55, rng=rng, seed=8, nhit=25)
    b = P.ONField(4, (6, 4, 8, 2), 0.3, 1.0, 0.1, 0.55, rng=rng, seed=8, nhit=25)
    a.sweep(4)
    b.sweep(2)
    path = tmp_path / "o4.ckpt"
    b.save(path)
    b.close()
    c = P.ONField.load(path)
    assert c.info()["sweeps"] == 2 and c.dims == (6, 4, 8, 2)
    c.sweep(2)
    assert np.array_equal(a.get_field(), c.get_field())
    assert a.acceptance() == c.acceptance()
    a.close()
    c.close()


def test_checkpoint_rejects_a_damaged_file(tmp_path):
    f = P.ONField(2, (4, 4, 2, 2), 0.2, 0.5, seed=1, nhit=3)
    path = tmp_path / "o2.ckpt"
    f.save(path)
    data = bytearray(path.read_bytes())
    data[200] ^= 1
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(bytes(data))
    with pytest.raises(P.LatError) as e:
        P.ONField.load(bad)
    assert e.value.code == P.ECORRUPT
    f.close()


def _binned(x, nbins=20):
    x = np.asarray(x)
    b = x[: len(x) // nbins * nbins].reshape(nbins, -1).mean(axis=1)
    return b.mean(), b.std(ddof=1) / np.sqrt(nbins)


@pytest.mark.parametrize("storage,rng", [(0, O.RNG_PHILOX), (1, O.RNG_RANLUX)])
def test_long_run_matches_exact_one_site_density(storage, rng):
    """kappa = 0 on the GPU itself: the chain samples the one-site density,
    whose moments come from quadrature (independent of both implementations)."""
    from test_oracle_on import one_site_moments
    f = P.ONField(4, (8, 8, 8, 8), 0.0, 0.5, 0.3, 1.4, storage=storage, rng=rng, seed=19, nhit=6)
    f.sweep(50)
    s = f.run(2000, 1)
    p2, q, m0 = one_site_moments(4, 0.5, 0.3)
    for col, want in ((0, p2), (2, q), (3, m0)):
        got, err = _binned(s[:, col])
        assert abs(got - want) < 4.5 * err + 2e-4, (col, got, want, err)
    f.close()


def test_long_run_matches_free_field_propagator():
    """lambda = 0 on the GPU: <phi^2>, the link product and <phi_0> of the
    free lattice field, exactly known on the finite lattice."""
    from test_oracle_on import free_field
    dims = (8, 4, 6, 4)
    f = P.ONField(2, dims, 0.1, 0.0, 0.2, 1.3, seed=5, nhit=8)
    f.sweep(200)
    s = f.run(4000, 1)
    phi2, link, m = free_field(dims, 2, 0.1, 0.2)
    for col, want in ((0, phi2), (1, link), (3, m)):
        got, err = _binned(s[:, col])
        assert abs(got - want) < 4.5 * err + 2e-4, (col, got, want, err)
    f.close()


def test_acceptance_before_a_sweep_is_a_state_error():
    f = P.ONField(1, (2, 2, 2, 2), 0.1, 0.1, seed=1, nhit=2)
    with pytest.raises(P.LatError) as e:
        f.acceptance()
    assert e.value.code == P.ESTATE
    f.sweep(1)
    assert 0.0 <= f.acceptance() <= 1.0
    f.close()


def test_f32_storage_rounds_set_values():
    f = P.ONField(2, (4, 2, 2, 2), 0.1, 0.1, storage=P.F32, seed=1, nhit=2)
    phi = np.random.default_rng(1).standard_normal((f.V, 2))
    f.set_field(phi)
    assert np.array_equal(f.get_field(), phi.astype(np.float32).astype(np.float64))
    f.close()


def test_wrong_buffer_sizes_are_rejected():
    f = P.ONField(3, (2, 2, 2, 2), 0.1, 0.1, seed=1, nhit=2)
    buf = np.zeros(f.V * 2)
    ptr = buf.ctypes.data_as(ctypes.c_void_p)
    assert P.lib.lat_on_set_field(f._h, ptr, buf.size) == P.EINVAL
    assert P.lib.lat_on_get_field(f._h, ptr, buf.size) == P.EINVAL
    assert P.lib.lat_on_get_field(f._h, None, f.V * 3) == P.EINVAL
    f.close()


def test_mrg_cold_start_and_states_match_oracle():
    g, o = pair(3, (6, 4, 2, 4), 0.2, 0.4, 0.0, 0.9, O.COLD, 12, rng=O.RNG_MRG32K3A, seed=123)
    g.sweep(3)
    o.sweep(3)
    assert np.abs(g.get_field() - o.get_field()).max() <= TOL64
    assert g.acceptance() == o.acceptance()
    g.close()
