"""GPU tests of the persistent batch launch: every member of a batch of
uneven lattices is bit-identical to the same lattice run alone (the batch
result is defined as the per-lattice result), for any launch shape; and a
member matches the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
from inputs import batch_workloads

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1310_7087_amd")


def descs_of(ws):
    return [dict(group=w.group, dims=w.dims, beta=w.beta, flux=w.flux, seed=w.seed, start=w.start,
                 lattice_id=w.lattice_id) for w in ws]


def small_batch():
    # mixed groups, uneven sizes, one flux member, shapes with ragged tiles
    return [dict(group=3, dims=(8, 8, 8, 4), beta=5.7, seed=11, lattice_id=0),
            dict(group=2, dims=(10, 10, 10, 4), beta=2.3, seed=11, lattice_id=1),
            dict(group=3, dims=(6, 4, 10, 2), beta=5.9, seed=11, lattice_id=2, flux=2),
            dict(group=2, dims=(2, 2, 2, 2), beta=2.2, seed=11, lattice_id=3),
            dict(group=3, dims=(12, 12, 12, 6), beta=6.0, seed=11, lattice_id=4)]


@pytest.mark.parametrize("storage", [P.F32, P.F64, P.F32_C12, P.F64_C12])
@pytest.mark.parametrize("shape", [(0, 256, 1, 0), (0, 64, 1, 0), (0, 128, 3, 0), (2, 128, 1, 0), (2, 64, 2, 0)])
def test_members_equal_single_runs(storage, shape):
    descs = small_batch()
    b = P.Batch(descs, storage=storage, rng=P.RNG_PHILOX)
    b.configure(*shape)
    pb, lb = b.run(3, 1, 4)
    for i, d in enumerate(descs):
        st = storage
        if d["group"] == 2 and storage in (P.F32_C12, P.F64_C12):  # SU(2) members keep all 4 reals
            st = P.F32 if storage == P.F32_C12 else P.F64
        single = P.Lattice(d["group"], d["dims"], d["beta"], d.get("flux", 0), storage=st,
                           rng=P.RNG_PHILOX, seed=d["seed"], lattice_id=d["lattice_id"], start=P.HOT)
        for _ in range(3):
            single.sweep(1, 4)
        assert np.array_equal(b.get_links(i), single.get_links()), (i, d)
        p, l = single.measure()
        assert np.array_equal(pb[i], p) and np.array_equal(lb[i], l)


def test_batch_member_matches_oracle():
    """FP64 batch, every member (the flux member and the 12^3x6 one
    included): one heat-bath sweep from the Haar start against the oracle."""
    descs = small_batch()
    b = P.Batch(descs, storage=P.F64, rng=P.RNG_PHILOX)
    b.run(1, 1, 0)
    for i, d in enumerate(descs):
        o = O.Lattice(d["group"], d["dims"], d["beta"], flux=d.get("flux", 0), seed=d["seed"],
                      lattice_id=d["lattice_id"], start=O.HOT)
        o.sweep(1, 0)
        assert np.abs(b.get_links(i) - o.get_links()).max() < 1e-12, i


def test_batch_compound_sweep_matches_oracle_from_thermalised_links():
    """FP64 batch from thermalised links (ten compound sweeps of each member
    run alone; single-lattice FP64 parity is tested elsewhere): one
    (1 HB + 4 OR) compound sweep of every member against the oracle at the
    FP64 bar, links and observables."""
    descs = small_batch()
    starts = []
    for d in descs:
        g = P.Lattice(d["group"], d["dims"], d["beta"], d.get("flux", 0), storage=P.F64, rng=P.RNG_PHILOX,
                      seed=d["seed"] + 100, lattice_id=d["lattice_id"], start=P.COLD)
        g.run(10, 1, 4, measure_every=0)
        starts.append(g.get_links())
        g.close()
    b = P.Batch(descs, storage=P.F64, rng=P.RNG_PHILOX)
    for i, l in enumerate(starts):
        b.set_links(i, l)
    pb, lb = b.run(1, 1, 4)
    for i, d in enumerate(descs):
        o = O.Lattice(d["group"], d["dims"], d["beta"], flux=d.get("flux", 0), seed=d["seed"],
                      lattice_id=d["lattice_id"], start=O.COLD)
        o.set_links(starts[i])
        o.sweep(1, 4)
        assert np.abs(b.get_links(i) - o.get_links()).max() < 1e-12, i
        po, lo = o.measure()
        assert np.abs(pb[i] - po).max() < 1e-12 and np.abs(lb[i] - lo).max() < 1e-12, i
    b.close()


def test_scan_workload_runs_and_repeats():
    """The 64-lattice beta scan (8^3x4 .. 24^3x6, SU(2)/SU(3)), two sweeps,
    bit-identical when repeated with another launch shape."""
    ws = batch_workloads(64, seed=11)
    d = descs_of(ws)
    a = P.Batch(d, storage=P.F32)
    pa, _ = a.run(2, 1, 4)
    b = P.Batch(d, storage=P.F32)
    b.configure(0, 128, 2, 0)
    pb, _ = b.run(2, 1, 4)
    assert np.array_equal(pa, pb)
    assert np.all(pa[:, 0] > 0.2) and np.all(pa[:, 0] < 0.8)


@pytest.mark.skip(reason="persistent batch form disabled: its run did not finish within the test's time "
                         "limit on MI355X (cross-XCD dependency polling); cause not yet shown")
@pytest.mark.parametrize("shape", [(1, 256, 1, 0), (1, 128, 2, 37)])
def test_persistent_form_equals_per_pass_form(shape):
    descs = small_batch()
    a = P.Batch(descs, storage=P.F32)
    pa, la = a.run(2, 1, 4)
    b = P.Batch(descs, storage=P.F32)
    b.configure(*shape)
    pb, lb = b.run(2, 1, 4)
    for i in range(len(descs)):
        assert np.array_equal(a.get_links(i), b.get_links(i)), i
    assert np.array_equal(pa, pb) and np.array_equal(la, lb)


def test_persistent_form_is_refused():
    b = P.Batch(small_batch()[:2], storage=P.F32)
    with pytest.raises(P.LatError) as e:
        b.configure(1, 256, 1, 0)
    assert e.value.code == P.EUNSUPPORTED


def test_batch_autotune_keeps_members():
    descs = small_batch()
    a = P.Batch(descs, storage=P.F32)
    b = P.Batch(descs, storage=P.F32)
    a.run(1, 1, 1)
    b.run(1, 1, 1)
    before = [a.get_links(i) for i in range(len(descs))]
    shape = a.autotune(1, 4)
    assert shape["block_size"] in (64, 128, 256) and shape["sites_per_thread"] in (1, 2, 4)
    for i in range(len(descs)):
        assert np.array_equal(a.get_links(i), before[i])
    pa, _ = a.run(2, 1, 4)
    pb, _ = b.run(2, 1, 4)
    assert np.array_equal(pa, pb)
    for i in range(len(descs)):
        assert np.array_equal(a.get_links(i), b.get_links(i))
