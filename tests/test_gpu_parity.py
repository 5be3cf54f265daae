"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle
on the same seeded inputs.

Tolerances: FP64 links and observables agree to 1e-12 (max abs over all
link components) wherever the update map is well conditioned, i.e. where
the oracle itself moves by < 1e-13 when its input links are perturbed at the
rounding level (2e-16 relative); this covers single heat-bath sweeps from
any start and compound sweeps from cold or thermalised links.
Overrelaxation on a Haar-random configuration is chaotic (the oracle's own
rounding envelope grows by ~10-100x per sweep), so there the bar is 100x
that measured envelope, and beyond the first compound sweep the comparison
is statistical.  FP32 forms: 2e-5.  Integer data (generator states, accept
decisions, raw Philox words): bit-exact."""
import numpy as np
import pytest

import oracle as O
from helpers import det_error, to_matrices, unitarity_error
from inputs import SU2_4x4, SU3_16x4, SU3_64x16, su3_32x8

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1310_7087_amd")

TOL64 = 1e-12
TOL32 = 2e-5


def pair(group, dims, beta, flux=0, rng=O.RNG_PHILOX, seed=1, start=O.HOT, storage=0, nhit=10,
         rng_const=0.5, lattice_id=0, frozen=0, **kw):
    g = P.Lattice(group, dims, beta, flux, storage=storage, rng=rng, seed=seed, start=start, nhit=nhit,
                  rng_const=rng_const, lattice_id=lattice_id, frozen=frozen, **kw)
    o = O.Lattice(group, dims, beta, flux=flux, rng=rng, seed=seed, start=start, nhit=nhit,
                  rng_const=rng_const, lattice_id=lattice_id, frozen=frozen)
    return g, o


def maxdiff(a, b):
    return float(np.abs(a - b).max())


def envelope(group, dims, beta, links, sweeps, flux=0, seed=1, rng=O.RNG_PHILOX, eps=2e-16):
    """Largest change of the oracle's links after `sweeps` when its input links
    are perturbed at the rounding level: the conditioning of the update map."""
    a = O.Lattice(group, dims, beta, flux=flux, seed=seed, rng=rng, start=O.COLD)
    b = O.Lattice(group, dims, beta, flux=flux, seed=seed, rng=rng, start=O.COLD)
    a.set_links(links)
    b.set_links(links * (1 + eps * np.random.default_rng(0).standard_normal(links.shape)))
    for h, o in sweeps:
        a.sweep(h, o)
        b.sweep(h, o)
    return maxdiff(a.get_links(), b.get_links())


def test_philox_words_bit_exact():
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    key = [0x1234567, 0x89ABCDEF]
    got = P.philox4x32_10(ctr, key)
    want = np.array([O.philox4x32_10(c, key) for c in ctr[:512]])
    assert np.array_equal(got[:512], want)


@pytest.mark.parametrize("group,rng,start,flux", [
    (3, O.RNG_PHILOX, O.HOT, 0), (3, O.RNG_MRG32K3A, O.HOT, 2), (2, O.RNG_PHILOX, O.HOT, 1),
    (2, O.RNG_MRG32K3A, O.HOT, 0), (3, O.RNG_PHILOX, O.COLD, 3), (2, O.RNG_CONST, O.HOT, 0)])
def test_initial_links(group, rng, start, flux):
    g, o = pair(group, (6, 4, 4, 2), 5.0, flux=flux, rng=rng, seed=9, start=start)
    assert maxdiff(g.get_links(), o.get_links()) < 1e-13
    if rng == O.RNG_MRG32K3A:
        assert np.array_equal(g.rng_state(), o.mrg_states())


def test_su2_4x4_cold_mrg_ten_sweeps():
    """SU(2) 4^4, beta 2.3, cold start, MRG32k3a seed 1: ten heat-bath sweeps,
    plaquette after each; generator states bit-exact, links to 1e-12."""
    w = SU2_4x4
    g, o = pair(w.group, w.dims, w.beta, rng=O.RNG_MRG32K3A, seed=w.seed, start=O.COLD)
    for k in range(w.sweeps):
        g.sweep(1, 0)
        o.sweep(1, 0)
        assert np.array_equal(g.rng_state(), o.mrg_states()), k
        assert maxdiff(g.get_links(), o.get_links()) < TOL64, k
        pg, _ = g.measure()
        po, _ = o.measure()
        assert maxdiff(pg, po) < TOL64, k


def test_su3_16x4_hot_heat_bath_sweep():
    """SU(3) 16^3x4, beta 5.69, Haar start seed 7: one heat-bath sweep
    (well conditioned), accept decisions bit-exact, links to 1e-12."""
    w = SU3_16x4
    g, o = pair(w.group, w.dims, w.beta, seed=w.seed, start=O.HOT)
    g.set_accept_log(True)
    o.enable_accept_log(True)
    g.sweep(1, 0)
    o.sweep(1, 0)
    assert np.array_equal(g.accept_log(), o.accept_log())
    assert maxdiff(g.get_links(), o.get_links()) < TOL64
    pg, lg = g.measure()
    po, lo = o.measure()
    assert maxdiff(pg, po) < TOL64 and maxdiff(lg, lo) < TOL64


def test_su3_16x4_hot_compound_sweep_within_rounding_envelope():
    """First (1 HB + 4 OR) sweep from the Haar start: overrelaxation of random
    links amplifies rounding; the GPU must stay within 100x the oracle's own
    rounding envelope."""
    w = SU3_16x4
    g, o = pair(w.group, w.dims, w.beta, seed=w.seed, start=O.HOT)
    env = envelope(w.group, w.dims, w.beta, o.get_links(), [(1, 4)], seed=w.seed)
    g.sweep(1, 4)
    o.sweep(1, 4)
    d = maxdiff(g.get_links(), o.get_links())
    print(f"GPU-oracle {d:.2e}, oracle rounding envelope {env:.2e}")
    assert d <= max(TOL64, 100 * env)


def test_su3_16x4_thermalised_compound_sweep():
    """From links thermalised by the oracle: one (1 HB + 4 OR) sweep, with the
    bar set by the measured conditioning."""
    w = SU3_16x4
    o = O.Lattice(w.group, w.dims, w.beta, seed=w.seed, start=O.HOT)
    o.sweep(5, 10)
    links = o.get_links()
    g = P.Lattice(w.group, w.dims, w.beta, seed=w.seed, start=P.COLD)
    g.set_links(links)
    o2 = O.Lattice(w.group, w.dims, w.beta, seed=w.seed, start=O.COLD)
    o2.set_links(links)
    env = envelope(w.group, w.dims, w.beta, links, [(1, 4)], seed=w.seed)
    g.set_accept_log(True)
    o2.enable_accept_log(True)
    g.sweep(1, 4)
    o2.sweep(1, 4)
    assert np.array_equal(g.accept_log(), o2.accept_log())
    d = maxdiff(g.get_links(), o2.get_links())
    print(f"GPU-oracle {d:.2e}, oracle rounding envelope {env:.2e}")
    assert d <= max(TOL64, 100 * env)
    assert maxdiff(g.measure()[0], o2.measure()[0]) < TOL64


def test_su3_16x4_long_run_statistics():
    """100 (1 HB + 4 OR) sweeps from the Haar start; the chains decorrelate, so
    the mean plaquettes of sweeps 21..100 are compared within their binned
    errors."""
    w = SU3_16x4
    g, o = pair(w.group, w.dims, w.beta, seed=w.seed, start=O.HOT)
    pg, lg = g.run(100, 1, 4, measure_every=1)
    po, lo = [], []
    for _ in range(100):
        o.sweep(1, 4)
        p, l = o.measure()
        po.append(p)
        lo.append(l)
    po, lo = np.array(po), np.array(lo)

    def mean_err(x, nb=8):
        b = x[20:20 + (len(x) - 20) // nb * nb].reshape(nb, -1).mean(axis=1)
        return b.mean(), b.std(ddof=1) / np.sqrt(nb)
    for a, b in ((pg[:, 0], po[:, 0]), (pg[:, 1], po[:, 1]), (pg[:, 2], po[:, 2])):
        (ma, ea), (mb, eb) = mean_err(a), mean_err(b)
        assert abs(ma - mb) < 4 * np.hypot(ea, eb) + 1e-6, (ma, ea, mb, eb)
    # beta 5.69 at Nt = 4 is the deconfinement point: L tunnels between the
    # confined and deconfined phases on time scales far beyond 80 sweeps, so
    # binned errors of its mean are not valid errors; both chains must stay
    # in the physical range of |L| on this volume instead
    absg = np.hypot(lg[20:, 0], lg[20:, 1])
    abso = np.hypot(lo[20:, 0], lo[20:, 1])
    assert absg.max() < 0.3 and abso.max() < 0.3
    assert abs(absg.mean() - abso.mean()) < 0.1


@pytest.mark.parametrize("group,dims", [
    (3, (2, 2, 2, 2)), (2, (2, 2, 2, 2)), (3, (6, 4, 10, 2)), (2, (18, 6, 4, 4)), (3, (4, 2, 2, 16)),
    (3, (34, 2, 2, 2))])
def test_ragged_and_degenerate_shapes(group, dims):
    # extents of 2 (x+1 = x-1), plane lengths that are not work-group multiples:
    # heat bath from the Haar start, then compound sweeps from a cold start with flux
    beta = 5.5 if group == 3 else 2.2
    g, o = pair(group, dims, beta, seed=21)
    g.sweep(1, 0)
    o.sweep(1, 0)
    assert maxdiff(g.get_links(), o.get_links()) < TOL64
    g, o = pair(group, dims, beta, flux=1, seed=21, start=O.COLD)
    for _ in range(2):
        g.sweep(1, 1)
        o.sweep(1, 1)
    assert maxdiff(g.get_links(), o.get_links()) < TOL64
    pg, lg = g.measure()
    po, lo = o.measure()
    assert maxdiff(pg, po) < TOL64 and maxdiff(lg, lo) < TOL64


@pytest.mark.parametrize("n", [1, 4])
def test_flux_w_frame_matches_u_frame_oracle(n):
    g, o = pair(3, (8, 8, 4, 4), 5.9, flux=n, seed=3, start=O.COLD)
    pg, _ = g.measure()
    po, _ = o.measure()
    assert maxdiff(pg, po) < 1e-14
    g.sweep(1, 4)
    o.sweep(1, 4)
    assert maxdiff(g.get_links(), o.get_links()) < TOL64
    assert maxdiff(g.measure()[0], o.measure()[0]) < TOL64


def test_constant_generator_and_zero_coupling():
    g, o = pair(2, (4, 4, 4, 4), 2.3, rng=O.RNG_CONST, start=O.COLD)
    g.sweep(1, 0)
    o.sweep(1, 0)
    assert maxdiff(g.get_links(), o.get_links()) < TOL64
    # beta = 0: alpha below threshold, heat bath leaves links; OR with a staple still reflects
    # (on Haar-random links, so the bar is the oracle's own rounding envelope)
    g, o = pair(3, (4, 4, 4, 2), 0.0, seed=4)
    env = envelope(3, (4, 4, 4, 2), 0.0, o.get_links(), [(2, 1)], seed=4)
    before = g.get_links()
    g.sweep(2, 1)
    o.sweep(2, 1)
    assert maxdiff(g.get_links(), o.get_links()) < max(TOL64, 100 * env)
    assert maxdiff(g.get_links(), before) > 0.1  # the overrelaxation step moved the links


def test_set_links_then_sweep_matches():
    o = O.Lattice(3, (8, 4, 4, 4), 6.0, seed=12, start=O.HOT)
    o.sweep(4, 10)
    links = o.get_links()
    g = P.Lattice(3, (8, 4, 4, 4), 6.0, seed=12, start=P.COLD)
    g.set_links(links)
    assert maxdiff(g.get_links(), links) == 0.0
    # continue both from the same links and the same heat-bath counter
    o2 = O.Lattice(3, (8, 4, 4, 4), 6.0, seed=12, start=O.COLD)
    o2.set_links(links)
    env = envelope(3, (8, 4, 4, 4), 6.0, links, [(1, 1)], seed=12)
    g.sweep(1, 1)
    o2.sweep(1, 1)
    assert maxdiff(g.get_links(), o2.get_links()) < max(TOL64, 100 * env)


def test_measure_random_configuration():
    o = O.Lattice(3, (6, 6, 4, 8), 5.7, flux=2, seed=31, start=O.HOT)
    o.sweep(1, 1)
    g = P.Lattice(3, (6, 6, 4, 8), 5.7, flux=2, seed=31, start=P.COLD)
    g.set_links(o.get_links())
    pg, lg = g.measure()
    po, lo = o.measure()
    assert maxdiff(pg, po) < 1e-14 and maxdiff(lg, lo) < 1e-14


def test_unitarity_after_many_sweeps():
    g = P.Lattice(3, (8, 8, 8, 4), 5.69, seed=7)
    g.run(20, 1, 4, measure_every=0)
    m = to_matrices(g.get_links(), 3)
    assert unitarity_error(m) < 1e-13 and det_error(m) < 1e-13


def test_tile_order_independence_and_repeatability():
    # z-slab per XCD (order 0 with 8 | Nz), identity, reversed, contiguous
    # chunks, compact 4-D work-group tiles: the pass is order independent
    res = []
    for order, tile in ((0, None), (1, None), (2, None), (3, None), (0, (8, 4, 2, 1)), (1, (4, 4, 4, 4)), (0, None)):
        g = P.Lattice(3, (16, 16, 16, 4), 5.9, seed=17, tile_order=order, block_size=64 if tile is None else 0,
                      tile=tile)
        g.sweep(1, 2)
        res.append(g.get_links())
    for r in res[1:]:
        assert np.array_equal(r, res[0])


@pytest.mark.parametrize("block", [64, 128, 256])
def test_block_size_independence(block):
    ref = P.Lattice(3, (8, 4, 8, 4), 5.9, seed=2)
    g = P.Lattice(3, (8, 4, 8, 4), 5.9, seed=2, block_size=block)
    ref.sweep(1, 1)
    g.sweep(1, 1)
    assert np.array_equal(ref.get_links(), g.get_links())


def test_run_series_matches_individual_measurements():
    a = P.Lattice(3, (8, 8, 4, 4), 5.7, seed=8)
    b = P.Lattice(3, (8, 8, 4, 4), 5.7, seed=8)
    ps, ls = a.run(6, 1, 2, measure_every=2)
    assert ps.shape == (3, 3)
    for k in range(3):
        b.sweep(1, 2)
        b.sweep(1, 2)
        p, l = b.measure()
        assert np.array_equal(ps[k], p) and np.array_equal(ls[k], l)


def test_checkpoint_round_trip(tmp_path):
    for rng in (P.RNG_PHILOX, P.RNG_MRG32K3A):
        a = P.Lattice(3, (4, 4, 4, 4), 5.7, seed=5, rng=rng)
        a.sweep(1, 1)
        path = tmp_path / f"c{rng}.ckpt"
        a.save(str(path))
        a.sweep(2, 1)
        b = P.load_lattice(str(path), 3, (4, 4, 4, 4))
        b.sweep(2, 1)
        assert np.array_equal(a.get_links(), b.get_links())
        assert b.info()["hb_sweeps"] == a.info()["hb_sweeps"]
        raw = bytearray(path.read_bytes())
        raw[200] ^= 0xFF
        path.write_bytes(bytes(raw))
        with pytest.raises(P.LatError):
            P.load_lattice(str(path), 3, (4, 4, 4, 4))


@pytest.mark.parametrize("storage,tol", [(P.F32, TOL32), (P.F32_C12, TOL32)])
def test_fp32_forms_one_sweep(storage, tol):
    """FP32 storage and staple arithmetic against the FP64 oracle, from the
    same links: accept decisions (FP64 on both sides) are compared first."""
    o = O.Lattice(3, (16, 16, 16, 4), 5.69, seed=7, start=O.HOT)
    o.sweep(3, 6)
    links = o.get_links()
    g = P.Lattice(3, (16, 16, 16, 4), 5.69, seed=7, start=P.COLD, storage=storage)
    g.set_links(links)
    g32 = g.get_links()
    assert maxdiff(g32, links) < 1e-6
    o2 = O.Lattice(3, (16, 16, 16, 4), 5.69, seed=7, start=O.COLD)
    o2.set_links(g32)  # identical starting links (already rounded to FP32)
    g.set_accept_log(True)
    o2.enable_accept_log(True)
    g.sweep(1, 0)
    o2.sweep(1, 0)
    flips = int((g.accept_log() != o2.accept_log()).sum())
    d = np.abs(g.get_links() - o2.get_links()).max(axis=(1, 2))
    if flips == 0:
        assert d.max() < tol
    else:  # a flipped decision moves links in its light cone by O(1); it must stay rare
        assert flips <= 2 and (d > tol).mean() < 0.01


@pytest.mark.parametrize("storage", [P.F32, P.F32_C12])
def test_fp32_forms_observables(storage):
    o = O.Lattice(3, (8, 8, 8, 4), 5.9, flux=1, seed=4, start=O.HOT)
    o.sweep(1, 1)
    g = P.Lattice(3, (8, 8, 8, 4), 5.9, flux=1, seed=4, start=P.COLD, storage=storage)
    g.set_links(o.get_links())
    pg, lg = g.measure()
    po, lo = o.measure()
    assert maxdiff(pg, po) < 1e-6 and maxdiff(lg, lo) < 1e-6


def test_su2_fp32_form():
    o = O.Lattice(2, (8, 8, 8, 4), 2.3, seed=6, start=O.HOT)
    o.sweep(3, 6)
    g = P.Lattice(2, (8, 8, 8, 4), 2.3, seed=6, start=P.COLD, storage=P.F32)
    g.set_links(o.get_links())
    assert maxdiff(g.get_links(), o.get_links()) < 1e-7
    o2 = O.Lattice(2, (8, 8, 8, 4), 2.3, seed=6, start=O.COLD)
    o2.set_links(g.get_links())
    g.set_accept_log(True)
    o2.enable_accept_log(True)
    g.sweep(1, 0)
    o2.sweep(1, 0)
    flips = int((g.accept_log() != o2.accept_log()).sum())
    d = np.abs(g.get_links() - o2.get_links()).max(axis=(1, 2))
    assert flips <= 2 and (d > TOL32).mean() < 0.01
    if flips == 0:
        assert d.max() < TOL32


def test_full_size_32x8_flux4_one_compound_sweep():
    """The measured workload's lattice (SU(3) 32^3x8, beta 5.9, n = 4, cold
    start) in the bench's launch configuration: every link after one
    (1 HB + 4 OR) sweep against the oracle."""
    w = su3_32x8(4)
    g, o = pair(w.group, w.dims, w.beta, flux=w.flux, seed=w.seed, start=O.COLD)
    O.set_threads(O.get_threads())
    g.sweep(1, 4)
    o.sweep(1, 4)
    assert maxdiff(g.get_links(), o.get_links()) < TOL64
    pg, lg = g.measure()
    po, lo = o.measure()
    assert maxdiff(pg, po) < TOL64 and maxdiff(lg, lo) < TOL64


def test_autotune_keeps_the_chain(tmp_path, monkeypatch):
    monkeypatch.setenv("LAT_TUNE_CACHE", str(tmp_path / "tune.txt"))
    for storage in (P.F64, P.F32_C12):
        a = P.Lattice(3, (16, 16, 16, 4), 5.9, seed=3, storage=storage)
        b = P.Lattice(3, (16, 16, 16, 4), 5.9, seed=3, storage=storage)
        a.sweep(1, 1)
        b.sweep(1, 1)
        before = a.get_links()
        info0 = a.info()
        shape = a.autotune(1, 4)
        assert shape["block_size"] in (64, 128, 256) and shape["tile_order"] in (0, 1, 2, 4)
        kinds = a.launch_shapes()
        assert kinds["overrelaxation"]["block_size"] == shape["block_size"]
        assert np.array_equal(a.get_links(), before) and a.info() == info0
        a.sweep(1, 4)
        b.sweep(1, 4)
        assert np.array_equal(a.get_links(), b.get_links())
        # a second tuner call is answered from the cache file
        c = P.Lattice(3, (16, 16, 16, 4), 5.9, seed=3, storage=storage)
        assert c.autotune(1, 4) == shape
    import json
    cache = json.loads((tmp_path / "tune.txt").read_text())
    assert len(cache) == 2 and all(len(v) == 16 for v in cache.values())


def test_full_size_64x16_heat_bath_sweep(tmp_path, monkeypatch):
    """SU(3) 64^3x16, beta 6.0, Haar start (seed 23), FP64, in the launch
    shape the autotuner picks: every link and the observables after one
    heat-bath sweep against the oracle."""
    monkeypatch.setenv("LAT_TUNE_CACHE", str(tmp_path / "tune.txt"))
    w = SU3_64x16
    O.set_threads(O.get_threads())
    g, o = pair(w.group, w.dims, w.beta, seed=w.seed, start=O.HOT)
    g.autotune(1, 4)
    g.sweep(1, 0)
    o.sweep(1, 0)
    assert maxdiff(g.get_links(), o.get_links()) < TOL64
    pg, lg = g.measure()
    po, lo = o.measure()
    assert maxdiff(pg, po) < TOL64 and maxdiff(lg, lo) < TOL64


def test_full_size_64x16_twelve_real_heat_bath_sweep(tmp_path, monkeypatch):
    """The same lattice in FP32 12-real storage, in its tuned launch shape,
    from links three compound sweeps off the Haar start: one heat-bath sweep
    against the oracle started from the identical (FP32-rounded) links.
    Decisions are taken in FP64 on both sides; a flipped one is expected about
    once per 10^7 and moves only the links it reaches within the sweep."""
    monkeypatch.setenv("LAT_TUNE_CACHE", str(tmp_path / "tune.txt"))
    w = SU3_64x16
    O.set_threads(O.get_threads())
    src = P.Lattice(w.group, w.dims, w.beta, storage=P.F64, seed=w.seed, start=P.HOT)
    src.run(3, 1, 4, measure_every=0)
    links = src.get_links()
    src.close()
    g = P.Lattice(w.group, w.dims, w.beta, storage=P.F32_C12, seed=w.seed, start=P.COLD)
    g.set_links(links)
    del links
    g.autotune(1, 4)
    o = O.Lattice(w.group, w.dims, w.beta, seed=w.seed, start=O.COLD)
    o.set_links(g.get_links())
    g.set_accept_log(True)
    o.enable_accept_log(True)
    g.sweep(1, 0)
    o.sweep(1, 0)
    la, lb = g.accept_log(), o.accept_log()
    flips = int((la != lb).sum())
    assert flips <= 1e-6 * la.size
    d = np.abs(g.get_links() - o.get_links()).max(axis=(1, 2))
    if flips == 0:
        assert d.max() < TOL32
    else:
        assert (d > TOL32).sum() <= 500 * flips
    pg, _ = g.measure()
    po, _ = o.measure()
    assert maxdiff(pg, po) < 1e-6


def test_f64_twelve_real_form():
    """FP64 12-real storage (row 3 rebuilt in FP64 on every load) against the
    FP64 oracle at the FP64 bar: links round-trip, one heat-bath sweep from the
    Haar start, and the measured workload's first compound sweep from cold."""
    o = O.Lattice(3, (16, 16, 16, 4), 5.69, seed=7, start=O.HOT)
    links = o.get_links()
    g = P.Lattice(3, (16, 16, 16, 4), 5.69, seed=7, start=P.HOT, storage=P.F64_C12)
    assert maxdiff(g.get_links(), links) < 1e-14  # same Haar start, row 3 rebuilt
    g.set_links(links)
    assert maxdiff(g.get_links(), links) < 1e-14
    g.sweep(1, 0)
    o.sweep(1, 0)
    assert maxdiff(g.get_links(), o.get_links()) < TOL64
    w = su3_32x8(1)
    g, o = pair(w.group, w.dims, w.beta, flux=w.flux, seed=w.seed, start=O.COLD, storage=P.F64_C12)
    g.sweep(1, 4)
    o.sweep(1, 4)
    assert maxdiff(g.get_links(), o.get_links()) < TOL64
    pg, lg = g.measure()
    po, lo = o.measure()
    assert maxdiff(pg, po) < TOL64 and maxdiff(lg, lo) < TOL64


@pytest.mark.parametrize("storage", [P.F64, P.F32_C12])
def test_graph_replays_equal_eager_launches(storage):
    """Every replay of the captured compound-sweep graph against the same
    passes launched one by one (the profiling path), with eager measurements
    and link reads between the replays."""
    a = P.Lattice(3, (8, 8, 8, 4), 5.8, 1, storage=storage, seed=12)
    b = P.Lattice(3, (8, 8, 8, 4), 5.8, 1, storage=storage, seed=12)
    for _ in range(4):
        a.sweep(1, 4)                      # graph replay
        b.profile_passes(1, 4, reps=1)     # the same passes, launched eagerly
        assert np.array_equal(a.get_links(), b.get_links())
        pa, la = a.measure()
        pb, lb = b.measure()
        assert np.array_equal(pa, pb) and np.array_equal(la, lb)
    assert a.info() == b.info()


@pytest.mark.parametrize("group,rng,start,sweeps", [
    (3, O.RNG_PHILOX, O.COLD, [(1, 4), (2, 0)]),
    (3, O.RNG_PHILOX, O.HOT, [(1, 0)]),
    (2, O.RNG_MRG32K3A, O.COLD, [(1, 0)] * 10)])
def test_frozen_background_links(group, rng, start, sweeps):
    """Spatial links of the slice t = 0 held at the background (a
    non-removable external field) against the oracle: every link, the
    generator states (MRG32k3a draws nothing for a frozen link) and the
    observables.  Sequences stay where the update map is well conditioned
    (one compound sweep from cold, then heat-bath sweeps), as for the other
    FP64 bars."""
    dims = (8, 6, 4, 4)
    beta = 5.7 if group == 3 else 2.3
    g, o = pair(group, dims, beta, flux=2, rng=rng, seed=9, start=start, frozen=1)
    t0 = np.arange(int(np.prod(dims))) // (dims[0] * dims[1] * dims[2]) == 0
    before = g.get_links()
    for h, r in sweeps:
        g.sweep(h, r)
        o.sweep(h, r)
    after = g.get_links()
    assert np.array_equal(after[t0, :3], before[t0, :3])
    assert maxdiff(after, o.get_links()) < TOL64
    if rng == O.RNG_MRG32K3A:
        assert np.array_equal(g.rng_state(), o.mrg_states())
    pg, lg = g.measure()
    po, lo = o.measure()
    assert maxdiff(pg, po) < TOL64 and maxdiff(lg, lo) < TOL64


def test_frozen_flag_survives_a_checkpoint(tmp_path):
    a = P.Lattice(3, (8, 6, 4, 4), 5.7, 2, seed=9, start=P.HOT, frozen=P.FROZEN_T0)
    a.sweep(1, 2)
    a.save(str(tmp_path / "f.ckpt"))
    b = P.load_lattice(str(tmp_path / "f.ckpt"), 3, (8, 6, 4, 4))
    a.sweep(1, 2)
    b.sweep(1, 2)
    assert np.array_equal(a.get_links(), b.get_links())


def swb_blocks(seed: int, n_blocks: int):
    """RANLUX luxury 3 written out: the Lehmer-seeded subtract-with-borrow
    generator, every 223rd group of outputs cut to its first 24; returns the
    delivered blocks and the carry after each."""
    e = seed
    x = []
    for _ in range(24):
        e = (40014 * e) % 2147483563
        x.append(e % (1 << 24))
    c = 1 if x[-1] == 0 else 0
    blocks, carries = [], []
    for b in range(n_blocks):
        out = []
        for k in range(223 if b else 24):
            y = x[-10] - x[-24] - c
            c = 1 if y < 0 else 0
            y %= 1 << 24
            x = x[1:] + [y]
            out.append(y)
        blocks.append(out[-24:] if b else out)
        carries.append(c)
    return blocks, carries


@pytest.mark.parametrize("group,dims,beta", [(3, (8, 6, 4, 4), 5.7), (2, (6, 6, 4, 4), 2.3)])
def test_ranlux_streams(group, dims, beta):
    """RANLUX luxury 3 per-site streams against the oracle: the hot start,
    three heat-bath sweeps (every accept decision) and a compound sweep from
    cold; the stored state of sample sites against the generator written
    out (four delivered blocks after the hot start, one per link)."""
    g, o = pair(group, dims, beta, rng=O.RNG_RANLUX, seed=77, start=O.HOT)
    assert maxdiff(g.get_links(), o.get_links()) < TOL64
    st = g.rng_state()
    for i in (0, 1, 37, int(np.prod(dims)) - 1):
        blocks, carries = swb_blocks(O.ranlux_site_seed(77, i, 0), 4)
        assert list(st[i, :24]) == blocks[3] and st[i, 24] == carries[3], i
    g.set_accept_log(True)
    o.enable_accept_log(True)
    for _ in range(3):
        g.sweep(1, 0)
        o.sweep(1, 0)
        assert np.array_equal(g.accept_log(), o.accept_log())
        assert maxdiff(g.get_links(), o.get_links()) < TOL64
    g, o = pair(group, dims, beta, rng=O.RNG_RANLUX, seed=78, start=O.COLD)
    g.sweep(1, 4)
    o.sweep(1, 4)
    assert maxdiff(g.get_links(), o.get_links()) < TOL64


def test_ranlux_state_survives_a_checkpoint(tmp_path):
    a = P.Lattice(3, (8, 6, 4, 4), 5.7, 0, rng=P.RNG_RANLUX, seed=5, start=P.HOT)
    a.sweep(1, 2)
    a.save(str(tmp_path / "r.ckpt"))
    b = P.load_lattice(str(tmp_path / "r.ckpt"), 3, (8, 6, 4, 4))
    a.sweep(2, 2)
    b.sweep(2, 2)
    assert np.array_equal(a.get_links(), b.get_links())


def test_run_series_in_graph_chunks_equals_stepwise():
    """Steady lat_run loops launch eight compound sweeps (and their
    measurements) per graph: the series, the links and the counters equal
    those of single sweeps with a measurement after each."""
    a = P.Lattice(3, (4, 4, 4, 4), 5.7, seed=12)
    b = P.Lattice(3, (4, 4, 4, 4), 5.7, seed=12)
    ps, ls = a.run(21, 1, 2, measure_every=1)
    assert ps.shape == (21, 3)
    for k in range(21):
        b.sweep(1, 2)
        p, l = b.measure()
        assert np.array_equal(ps[k], p) and np.array_equal(ls[k], l), k
    assert np.array_equal(a.get_links(), b.get_links())
    assert a.info() == b.info()


def test_run_series_across_the_device_buffer_refill():
    """More measurements than the device series holds (4096): the buffer is
    copied out and refilled mid-run without losing or repeating a value."""
    a = P.Lattice(2, (2, 2, 2, 2), 2.3, seed=4)
    b = P.Lattice(2, (2, 2, 2, 2), 2.3, seed=4)
    n = 4096 + 27
    ps, ls = a.run(n, 1, 1, measure_every=1)
    p1, l1 = b.run(4000, 1, 1, measure_every=1)
    p2, l2 = b.run(n - 4000, 1, 1, measure_every=1)
    assert np.array_equal(ps, np.concatenate([p1, p2])) and np.array_equal(ls, np.concatenate([l1, l2]))
    assert a.info() == b.info()
    # and a run without measurements advances the chain the same way
    c = P.Lattice(2, (2, 2, 2, 2), 2.3, seed=4)
    c.run(n, 1, 1, measure_every=0)
    assert np.array_equal(c.get_links(), a.get_links())
