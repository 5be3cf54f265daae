"""FP32 storage forms against the FP64 oracle, overrelaxation included.

Each case starts the HIP path (FP32 18-real, FP32 12-real, SU(2) FP32) and
the oracle from the identical links (thermalised, then rounded to the
storage form by the library) and the identical random numbers, runs one
sweep, and compares every link.  Heat-bath accept decisions are taken in
FP64 on both sides; a decision that FP32 rounding of the staple flipped
moves its link by O(1), and with it every link that the rest of the sweep
computes from it: those links (the decision's light cone, lightcone.py)
are excluded, all others are held to the bar.

Bars.  One sweep, heat bath or overrelaxation (every link updated once):
2e-5 per link.  A compound (1 HB + 4 OR) sweep updates each link five
times, and overrelaxation amplifies input errors: the oracle's own links
move, after one compound sweep of thermalised links, by up to 6e-5 (SU(3)
16^3x4, beta 5.69; 5e-5 at 32^3x8, beta 5.9) when only its input is
perturbed by a single FP32 rounding (2^-24 relative), so no FP32
computation of that sweep can meet 2e-5 on every link.  There every link
is held to 10 times the largest such sensitivity measured on the same
links (the FP32 path rounds many times per update where the probe rounds
once), and the observables to 2e-6 (1e-6 after a single sweep).
"""
import numpy as np
import pytest

import oracle as O
from lightcone import downstream, flipped_updates

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1310_7087_amd")

TOL32 = 2e-5
_THERM = {}


def thermalised(group, dims, beta, flux, seed):
    """Links after ten (1 HB + 4 OR) sweeps of the FP64 HIP path from a cold
    start (FP64 parity with the oracle is tested elsewhere)."""
    key = (group, dims, beta, flux, seed)
    if key not in _THERM:
        g = P.Lattice(group, dims, beta, flux, storage=P.F64, seed=seed, start=P.COLD)
        g.run(10, 1, 4, measure_every=0)
        _THERM[key] = g.get_links()
        g.close()
    return _THERM[key]


def sensitivity(group, dims, beta, flux, seed, links, sweep, samples=2):
    """Per-link change [V, 4] of the oracle's result when its input links are
    perturbed by one FP32 rounding (relative 2^-24, random sign and size)."""
    ref = O.Lattice(group, dims, beta, flux=flux, seed=seed, start=O.COLD)
    ref.set_links(links)
    ref.sweep(*sweep)
    base = ref.get_links()
    env = np.zeros(base.shape[:2])
    rng = np.random.default_rng(1)
    for _ in range(samples):
        o = O.Lattice(group, dims, beta, flux=flux, seed=seed, start=O.COLD)
        o.set_links(links * (1 + 2.0 ** -24 * rng.uniform(-1, 1, links.shape)))
        o.sweep(*sweep)
        env = np.maximum(env, np.abs(o.get_links() - base).max(axis=2))
    return env


def compare(group, dims, beta, flux, storage, sweep, seed=3):
    """Runs `sweep` on both sides from the same rounded links; returns the
    per-link difference [V, 4], the light cone of flipped decisions, the
    number of flips and both sides' observables."""
    links = thermalised(group, dims, beta, flux, seed)
    g = P.Lattice(group, dims, beta, flux, storage=storage, seed=seed, start=P.COLD)
    g.set_links(links)
    start = g.get_links()  # rounded to the storage form (12-real: row 3 rebuilt)
    o = O.Lattice(group, dims, beta, flux=flux, seed=seed, start=O.COLD)
    o.set_links(start)
    n_hb, n_or = sweep
    if n_hb:
        g.set_accept_log(True)
        o.enable_accept_log(True)
    g.sweep(n_hb, n_or)
    o.sweep(n_hb, n_or)
    V = int(np.prod(dims))
    flips = None
    nflip = 0
    if n_hb:
        flips = flipped_updates(g.accept_log(), o.accept_log(), n_hb, V)
        nflip = int(flips.sum())
    cone = downstream(dims, n_hb, n_or, flips=flips)
    d = np.abs(g.get_links() - o.get_links()).max(axis=2)
    obs = (np.concatenate(g.measure()), np.concatenate(o.measure()))
    g.close()
    return d, cone, nflip, obs, start


def report(tag, d, cone, nflip, obs, env=None):
    ok = ~cone
    msg = (f"{tag}: flips {nflip}, cone {int(cone.sum())} links; outside: max {d[ok].max():.2e}, "
           f"q99.9 {np.quantile(d[ok], 0.999):.2e}, >2e-5: {int((d[ok] > TOL32).sum())}; "
           f"observables (P, P_s, P_t, Re L, Im L) diff {np.abs(obs[0] - obs[1]).max():.1e}")
    if env is not None:
        msg += (f"; oracle FP32-rounding sensitivity max {env.max():.2e}, q99.9 {np.quantile(env, 0.999):.2e}; "
                f"max diff / max sensitivity {d[ok].max() / env.max():.2f}")
    print(msg, flush=True)


FORMS = [(3, (16, 16, 16, 4), 5.69, 0, "F32"), (3, (16, 16, 16, 4), 5.69, 0, "F32_C12"),
         (2, (8, 8, 8, 4), 2.3, 0, "F32"), (3, (8, 8, 8, 4), 5.9, 1, "F32_C12")]


@pytest.mark.parametrize("group,dims,beta,flux,form", FORMS)
@pytest.mark.parametrize("sweep", [(0, 1), (1, 0)])
def test_fp32_single_sweep(group, dims, beta, flux, form, sweep):
    storage = getattr(P, form)
    print(f"FP32 single sweep {sweep}: SU({group}) {dims} beta {beta} flux {flux} {form}", flush=True)
    d, cone, nflip, obs, _ = compare(group, dims, beta, flux, storage, sweep)
    report(f"{form} {sweep}", d, cone, nflip, obs)
    assert d[~cone].max() < TOL32
    assert np.abs(obs[0] - obs[1]).max() < 1e-6
    assert cone.mean() < 0.05


@pytest.mark.parametrize("group,dims,beta,flux,form", FORMS[:3])
def test_fp32_compound_sweep(group, dims, beta, flux, form):
    storage = getattr(P, form)
    print(f"FP32 compound sweep (1, 4): SU({group}) {dims} beta {beta} {form}", flush=True)
    d, cone, nflip, obs, start = compare(group, dims, beta, flux, storage, (1, 4))
    env = sensitivity(group, dims, beta, flux, 3, start, (1, 4))
    report(f"{form} (1, 4)", d, cone, nflip, obs, env)
    ok = ~cone
    assert d[ok].max() <= max(TOL32, 10 * env.max())
    assert np.abs(obs[0] - obs[1]).max() < 2e-6


@pytest.mark.parametrize("form", ["F32_C12", "F32"])
def test_fp32_bench_lattice(form):
    """The measured workload's lattice, SU(3) 32^3x8, beta 5.9, n = 4, from
    thermalised links: one overrelaxation sweep, one heat-bath sweep and
    one compound sweep against the oracle."""
    storage = getattr(P, form)
    O.set_threads(O.get_threads())
    for sweep in [(0, 1), (1, 0), (1, 4)]:
        print(f"FP32 32^3x8 {form} sweep {sweep}", flush=True)
        d, cone, nflip, obs, start = compare(3, (32, 32, 32, 8), 5.9, 4, storage, sweep)
        ok = ~cone
        if sweep == (1, 4):
            env = sensitivity(3, (32, 32, 32, 8), 5.9, 4, 3, start, sweep, samples=1)
            report(f"32^3x8 {form} {sweep}", d, cone, nflip, obs, env)
            assert d[ok].max() <= max(TOL32, 10 * env.max())
        else:
            report(f"32^3x8 {form} {sweep}", d, cone, nflip, obs)
            assert d[ok].max() < TOL32
        assert np.abs(obs[0] - obs[1]).max() < (1e-6 if sweep != (1, 4) else 2e-6)
        # a flipped heat-bath decision reaches further through four more sweeps
        assert cone.mean() < (0.05 if sweep != (1, 4) else 0.5)


def test_fp32_batch_members():
    """FP32 batch (one launch per pass over all members) from thermalised
    links: every member's links after one overrelaxation sweep and after a
    compound sweep against the oracle; decisions flipped by FP32 rounding
    are read from the same member run alone with the accept log (the batch
    is bit-identical to single runs)."""
    descs = [dict(group=3, dims=(8, 8, 8, 4), beta=5.7, seed=11, lattice_id=0),
             dict(group=2, dims=(10, 10, 10, 4), beta=2.3, seed=11, lattice_id=1),
             dict(group=3, dims=(6, 4, 10, 2), beta=5.9, seed=11, lattice_id=2),
             dict(group=3, dims=(12, 12, 12, 6), beta=6.0, seed=11, lattice_id=3)]
    starts = [thermalised(d["group"], d["dims"], d["beta"], 0, 5) for d in descs]
    for sweep in [(0, 1), (1, 4)]:
        b = P.Batch(descs, storage=P.F32, rng=P.RNG_PHILOX)
        for i, l in enumerate(starts):
            b.set_links(i, l)
        rounded = [b.get_links(i) for i in range(len(descs))]
        b.run(1, *sweep)
        for i, d in enumerate(descs):
            single = P.Lattice(d["group"], d["dims"], d["beta"], storage=P.F32, seed=d["seed"],
                               lattice_id=d["lattice_id"], start=P.COLD)
            single.set_links(rounded[i])
            o = O.Lattice(d["group"], d["dims"], d["beta"], seed=d["seed"], lattice_id=d["lattice_id"],
                          start=O.COLD)
            o.set_links(rounded[i])
            if sweep[0]:
                single.set_accept_log(True)
                o.enable_accept_log(True)
            single.sweep(*sweep)
            o.sweep(*sweep)
            got = b.get_links(i)
            assert np.array_equal(got, single.get_links())
            V = int(np.prod(d["dims"]))
            flips = flipped_updates(single.accept_log(), o.accept_log(), sweep[0], V) if sweep[0] else None
            cone = downstream(d["dims"], sweep[0], sweep[1], flips=flips)
            dd = np.abs(got - o.get_links()).max(axis=2)
            report(f"batch member {i} {sweep}", dd, cone, 0 if flips is None else int(flips.sum()),
                   (np.concatenate(single.measure()), np.concatenate(o.measure())))
            if sweep == (0, 1):
                assert dd[~cone].max() < TOL32
            else:
                env = sensitivity(d["group"], d["dims"], d["beta"], 0, d["seed"], rounded[i], sweep)
                assert dd[~cone].max() <= max(TOL32, 10 * env.max())
            single.close()
        b.close()
