#!/usr/bin/env python3
"""Throughput of the checkerboard SU(3) Wilson-action sweep on one MI355X.

A step is one working sweep of the whole hot path on SU(3) 32^3 x 8
(beta 5.9, one flux quantum of the lambda_3 background, cold start): one
compound sweep (1 heat-bath + 4 overrelaxation sweeps, reunitarisation
fused into the last) followed by the plaquette and Polyakov-loop
measurement.  The metric is link updates per second,
steps * (1 + 4) * 4 V / time, with the lattice resident in HBM; the plain
FP64 18-real form gives the headline value.  Each form first picks its
launch shape with the library's autotuner (the lattice state is restored).

Also reported: the FP32, 12-real FP32 and 12-real FP64 storage forms
(speed-up over FP64), the precision of the FP32 forms against FP64 for every
observable (paired runs that share start and random numbers), the roofline
of the dominant pass kernel (event-timed in this run), SU(3) 64^3 x 16 (the
case that does not fit the last-level cache), the 64-lattice batch in FP32
against the same lattices run one by one in FP64, RANLUX-driven working
sweeps on the lattice shapes of the paper's Table 1 (SU(3) 32^4, SU(2)
44^4), the O(4) model's pass, and the FP64 CPU oracle timed on a bounded
sample of the headline workload on the host cores.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
for p in (ROOT, os.path.join(ROOT, "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
DIMS = (32, 32, 32, 8)
BETA = 5.9
FLUX = 1
N_HB, N_OR = 1, 4
REPEATS = 5
BYTES_PER_LINK = {"f64": 144, "f32": 72, "f32c12": 48, "f64c12": 96}
KERNEL_SOURCES = ["paper_1310_7087_amd/csrc/lat_kernels.hip", "paper_1310_7087_amd/csrc/lat_dev.hpp",
                  "paper_1310_7087_amd/csrc/lat_types.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v


def binned(x, nbins=10):
    """Mean and binned standard error of a series (last nbins*k entries)."""
    import numpy as np
    x = np.asarray(x, dtype=float)
    n = len(x) // nbins * nbins
    if n < 2 * nbins:
        return float(np.mean(x)), float("nan")
    b = x[len(x) - n:].reshape(nbins, -1).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / np.sqrt(nbins))


def observables(plaq, poly):
    """Mean and binned error of P, P_s, P_t, Re L and |L| over a series."""
    import numpy as np
    series = {"P": plaq[:, 0], "P_s": plaq[:, 1], "P_t": plaq[:, 2], "ReL": poly[:, 0],
              "absL": np.hypot(poly[:, 0], poly[:, 1])}
    return {k: dict(zip(("mean", "err"), binned(v))) for k, v in series.items()}


def storage_of(P, form):
    return {"f64": P.F64, "f32": P.F32, "f32c12": P.F32_C12, "f64c12": P.F64_C12}[form]


def run_form(P, form: str, steps: int, warmup: int):
    import torch
    V = volume(DIMS)
    lat = P.Lattice(3, DIMS, BETA, FLUX, storage=storage_of(P, form), rng=P.RNG_PHILOX, seed=3, start=P.COLD)
    log(f"[{form}] warmup {warmup} steps")
    early, _ = lat.run(warmup, N_HB, N_OR, measure_every=1)
    # launch shape tuned on the warmed-up links (the state is restored)
    lat.autotune(N_HB, N_OR)
    shape = lat.launch_shapes()
    log(f"[{form}] launch shapes {shape}")
    lat.run(1, N_HB, N_OR, measure_every=1)  # graph capture of the tuned shape
    torch.cuda.synchronize()
    log(f"[{form}] timing {steps} steps in {REPEATS} repeats")
    series, times = [], []
    for k in range(REPEATS):
        n = steps // REPEATS + (1 if k < steps % REPEATS else 0)
        t0 = time.perf_counter()
        series.append(lat.run(n, N_HB, N_OR, measure_every=1))  # queued on the device, synchronises
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0, n))
    import numpy as np
    plaq = np.concatenate([x[0] for x in series])
    poly = np.concatenate([x[1] for x in series])
    dt = sum(t for t, _ in times)
    per_repeat = sorted(n * (N_HB + N_OR) * 4 * volume(DIMS) / t for t, n in times)
    updates = steps * (N_HB + N_OR) * 4 * V
    # event-timed passes of the same kernels on the same stream
    t_hb, t_or = lat.profile_passes(N_HB, N_OR, reps=5)
    b = BYTES_PER_LINK[form]
    pass_bytes = 4.5 * V * b  # reads all 4V links, writes the V/2 updated ones
    obs = observables(plaq, poly)
    res = {
        "link_updates_per_s": updates / dt,
        "median_of_repeats": per_repeat[len(per_repeat) // 2],
        "repeat_range": [per_repeat[0], per_repeat[-1]],
        "ms_per_step": 1e3 * dt / steps,
        "launch_shape": shape,
        "early_plaquettes": [float(x) for x in early[:10, 0]],
        "observables": obs,
        "plaquette_last": [float(x) for x in plaq[-1]],
        "polyakov_last": [float(poly[-1][0]), float(poly[-1][1])],
        "hb_pass_us": 1e3 * t_hb,
        "or_pass_us": 1e3 * t_or,
        "hb_pass_GBs": pass_bytes / (t_hb * 1e-3) / 1e9,
        "or_pass_GBs": pass_bytes / (t_or * 1e-3) / 1e9,
        "algorithmic_GBs": updates * 9 * b / dt / 1e9,
        "pass_bytes": pass_bytes,
    }
    res["hbm_fraction"] = res["algorithmic_GBs"] / HBM_PEAK_GBS
    lat.close()
    return res


def run_flux_observables(P, forms, steps: int = 1000, warmup: int = 50, fluxes=(0, 4)):
    """The headline lattice at the other flux quanta of the workload (n = 0
    and 4; n = 1 is the timed run): P, P_s, P_t, Re L and |L| with binned
    errors per storage form, from the cold start, `warmup` compound sweeps
    discarded.  The background is a change of variables of the Haar measure,
    so the equilibrium values do not depend on n."""
    import numpy as np
    out = {}
    for n in fluxes:
        row = {}
        for form in forms:
            lat = P.Lattice(3, DIMS, BETA, n, storage=storage_of(P, form), rng=P.RNG_PHILOX, seed=3, start=P.COLD)
            lat.run(warmup, N_HB, N_OR, measure_every=0)
            lat.autotune(N_HB, N_OR)
            plaq, poly = lat.run(steps, N_HB, N_OR, measure_every=1)
            lat.close()
            row[form] = observables(plaq, poly)
        out[f"flux_{n}"] = row
        log(f"[flux {n}] <P> " + ", ".join(f"{f} {row[f]['P']['mean']:.6f}({row[f]['P']['err'] * 1e6:.0f}e-6)"
                                           for f in forms))
    return out


def paired(x, y, nbins=50):
    """Mean and binned error of the per-sweep difference x - y of two series
    of the same length."""
    import numpy as np
    return binned(np.asarray(x) - np.asarray(y), nbins)


def precision_leg(P, steps: int, therm: int = 200, forms=("f32c12", "f32", "f64c12"), seeds=(3,)):
    """FP32 storage forms against FP64 on the headline lattice.  Within a
    replica every form starts from the same cold links and draws the same
    random numbers, so the chains are coupled and the per-sweep difference of
    each observable (P, P_s, P_t, Re L, |L|) has a smaller variance than two
    independent chains would give; its mean over `steps` measured compound
    sweeps, after `therm` discarded ones, with a binned error (50 bins),
    bounds the FP32 form's systematic error.  Replicas (one per seed) are
    independent; their differences are combined as an inverse-variance
    weighted mean, and the chi^2 of the replicas about it checks the binned
    errors.  The independent-chain error is reported beside the paired one.
    The FP64 12-real form, which rounds like the reference, is the control:
    its difference shows what the decorrelation of coupled chains alone
    gives."""
    import numpy as np
    out = {"steps": steps, "thermalisation": therm, "bins": 50, "bound": 1e-5, "seeds": list(seeds)}
    keys = ("P", "P_s", "P_t", "ReL", "absL")
    reps = []
    for seed in seeds:
        series = {}
        for form in ("f64",) + tuple(forms):
            t0 = time.perf_counter()
            lat = P.Lattice(3, DIMS, BETA, FLUX, storage=storage_of(P, form), rng=P.RNG_PHILOX, seed=seed,
                            start=P.COLD)
            plaq, poly = lat.run(therm + steps, N_HB, N_OR, measure_every=1)
            lat.close()
            series[form] = {"P": plaq[therm:, 0], "P_s": plaq[therm:, 1], "P_t": plaq[therm:, 2],
                            "ReL": poly[therm:, 0], "absL": np.hypot(poly[therm:, 0], poly[therm:, 1])}
            log(f"[precision] seed {seed} {form}: {therm + steps} compound sweeps in "
                f"{time.perf_counter() - t0:.1f} s")
        ref = series["f64"]
        rep = {"seed": seed, "f64_means": {k: dict(zip(("mean", "err"), binned(v, 50))) for k, v in ref.items()}}
        for form in forms:
            rows = {}
            for k in keys:
                v = series[form][k]
                d, e = paired(v, ref[k])
                rows[k] = {"delta": d, "err": e,
                           "independent_chain_err": math.hypot(binned(v, 50)[1], binned(ref[k], 50)[1])}
            rep[form] = rows
            log(f"[precision] seed {seed} {form} - f64: <P> {rows['P']['delta']:.2e} +- {rows['P']['err']:.1e} "
                f"(independent chains: +- {rows['P']['independent_chain_err']:.1e})")
        reps.append(rep)
    out["replicas"] = reps
    for form in forms:
        comb = {}
        for k in keys:
            d = np.array([r[form][k]["delta"] for r in reps])
            e = np.array([r[form][k]["err"] for r in reps])
            w = 1.0 / e ** 2
            m = float(np.sum(w * d) / np.sum(w))
            comb[k] = {"delta": m, "err": float(np.sqrt(1.0 / np.sum(w))),
                       "chi2_per_dof": float(np.sum(w * (d - m) ** 2) / (len(d) - 1)) if len(d) > 1 else None}
        dp = comb["P"]
        comb["P_within_bound"] = bool(abs(dp["delta"]) + 2 * dp["err"] <= out["bound"])
        out[form] = comb
        log(f"[precision] {form} - f64 over {len(seeds)} replica(s): <P> {dp['delta']:.2e} +- {dp['err']:.1e}")
    return out


def precision_large(P, steps: int, therm: int = 200, seed: int = 23, forms=("f32c12",)):
    """FP32 12-real (and any other `forms`, e.g. the FP64 12-real control)
    against FP64 on SU(3) 64^3 x 16 (beta 6.0, Haar start): chains coupled
    to the FP64 one (same start, same random numbers), `therm` compound
    sweeps discarded, the paired per-sweep difference of each observable
    over `steps` measured ones with a binned error (20 bins)."""
    import numpy as np
    dims = (64, 64, 64, 16)
    series = {}
    for form in ("f64",) + tuple(forms):
        t0 = time.perf_counter()
        lat = P.Lattice(3, dims, 6.0, 0, storage=storage_of(P, form), rng=P.RNG_PHILOX, seed=seed, start=P.HOT)
        plaq, poly = lat.run(therm + steps, N_HB, N_OR, measure_every=1)
        lat.close()
        series[form] = {"P": plaq[therm:, 0], "P_s": plaq[therm:, 1], "P_t": plaq[therm:, 2],
                        "ReL": poly[therm:, 0], "absL": np.hypot(poly[therm:, 0], poly[therm:, 1])}
        log(f"[precision 64^3x16] {form}: {therm + steps} compound sweeps in {time.perf_counter() - t0:.1f} s")
    out = {"lattice": list(dims), "beta": 6.0, "start": "hot", "seed": seed, "steps": steps,
           "thermalisation": therm, "bins": 20, "bound": 1e-5,
           "f64_means": {k: dict(zip(("mean", "err"), binned(v, 20))) for k, v in series["f64"].items()}}
    for form in forms:
        rows = {}
        for k, v in series[form].items():
            d, e = paired(v, series["f64"][k], 20)
            rows[k] = {"delta": d, "err": e,
                       "independent_chain_err": math.hypot(binned(v, 20)[1], binned(series["f64"][k], 20)[1])}
        rows["P_within_bound"] = bool(abs(rows["P"]["delta"]) + 2 * rows["P"]["err"] <= 1e-5)
        out[form] = rows
        log(f"[precision 64^3x16] {form} - f64: <P> {rows['P']['delta']:.2e} +- {rows['P']['err']:.1e}, "
            f"|L| {rows['absL']['delta']:.2e} +- {rows['absL']['err']:.1e}")
    return out


def run_large(P, sweeps: int = 40):
    """SU(3) 64^3 x 16, beta 6.0, Haar start (seed 23): FP64 18-real against
    FP32 12-real on the lattice that does not fit the 256 MB last-level cache."""
    dims = (64, 64, 64, 16)
    V = volume(dims)
    out = {}
    for form in ("f64", "f32c12"):
        lat = P.Lattice(3, dims, 6.0, 0, storage=storage_of(P, form), rng=P.RNG_PHILOX, seed=23, start=P.HOT)
        lat.run(5, N_HB, N_OR, measure_every=0)
        lat.autotune(N_HB, N_OR)
        shape = lat.launch_shapes()
        lat.run(1, N_HB, N_OR, measure_every=1)  # graph capture
        t0 = time.perf_counter()
        plaq, _ = lat.run(sweeps, N_HB, N_OR, measure_every=1)
        dt = time.perf_counter() - t0
        t_hb, t_or = lat.profile_passes(N_HB, N_OR, reps=2)
        b = BYTES_PER_LINK[form]
        r = {"launch_shape": shape, "link_updates_per_s": sweeps * 5 * 4 * V / dt,
             "ms_per_step": 1e3 * dt / sweeps, "algorithmic_GBs": sweeps * 5 * 4 * V * 9 * b / dt / 1e9,
             "or_pass_us": 1e3 * t_or, "hb_pass_us": 1e3 * t_hb,
             "or_pass_hbm_fraction": 4.5 * V * b / (t_or * 1e-3) / 1e9 / HBM_PEAK_GBS,
             "plaquette_tail": [float(x) for x in plaq[-3:, 0]]}
        r["hbm_fraction"] = r["algorithmic_GBs"] / HBM_PEAK_GBS
        r["plaquette_mean_last_half"], r["plaquette_err_last_half"] = binned(plaq[sweeps // 2:, 0], 5)
        out[form] = r
        lat.close()
        log(f"[64^3x16 {form}] {r['link_updates_per_s']:.3e} link updates/s")
    out["speedup_f32c12_vs_f64"] = out["f32c12"]["link_updates_per_s"] / out["f64"]["link_updates_per_s"]
    out["delta_plaquette_f32c12_minus_f64"] = (out["f32c12"]["plaquette_mean_last_half"]
                                              - out["f64"]["plaquette_mean_last_half"])
    out["config"] = {"lattice": list(dims), "beta": 6.0, "start": "hot", "seed": 23,
                     "sweeps_before_timing": 6, "sweeps": sweeps, "n_hb": N_HB, "n_or": N_OR}
    return out


def run_batch(P, sweeps: int = 10, precision_sweeps: int = 1000):
    """64 independent lattices (SU(2)/SU(3), 8^3x4 .. 24^3x6, coupling scan):
    the FP32 batch launch (18-real, and 12-real for the SU(3) members)
    against the same lattices run one by one in FP64 (the plain form) and
    against the FP64 batch."""
    from inputs import batch_workloads
    ws = batch_workloads(64, seed=11)
    descs = [dict(group=w.group, dims=w.dims, beta=w.beta, flux=w.flux, seed=w.seed, start=w.start,
                  lattice_id=w.lattice_id) for w in ws]
    links = sum(4 * volume(w.dims) for w in ws)
    rates, shapes = {}, {}
    for name, storage in (("f32_batched", P.F32), ("f32c12_batched", P.F32_C12), ("f64_batched", P.F64)):
        bt = P.Batch(descs, storage=storage)
        bt.run(20, N_HB, N_OR, measure=False)
        shapes[name] = bt.autotune(N_HB, N_OR)
        bt.run(sweeps, N_HB, N_OR, measure=False)  # captures the graph timed below
        t0 = time.perf_counter()
        bt.run(sweeps, N_HB, N_OR, measure=False)
        rates[name] = sweeps * 5 * links / (time.perf_counter() - t0)
        bt.close()
    singles = [P.Lattice(d["group"], d["dims"], d["beta"], 0, storage=P.F64, rng=P.RNG_PHILOX,
                         seed=d["seed"], lattice_id=d["lattice_id"], start=d["start"]) for d in descs]
    for s in singles:
        s.run(2, N_HB, N_OR, measure_every=0)
    t0 = time.perf_counter()
    for s in singles:
        s.run(sweeps, N_HB, N_OR, measure_every=0)
    rates["f64_one_by_one"] = sweeps * 5 * links / (time.perf_counter() - t0)
    for s in singles:
        s.close()
    log(f"[batch] F32 batched {rates['f32_batched']:.3e}, F32 12-real batched {rates['f32c12_batched']:.3e}, "
        f"F64 batched {rates['f64_batched']:.3e}, "
        f"F64 one by one {rates['f64_one_by_one']:.3e} link updates/s")
    # algorithmic bytes: 9 b per link update (4.5 V b per pass), b by group and storage
    # SU(2) members of the 12-real batch keep FP32 quaternions
    bpl = {("f32", 3): 72, ("f32", 2): 16, ("f32c12", 3): 48, ("f32c12", 2): 16, ("f64", 3): 144, ("f64", 2): 32}
    frac = {}
    for name in ("f32_batched", "f32c12_batched", "f64_batched"):
        form = name[:-len("_batched")]
        per_update = sum(4 * volume(w.dims) * 9 * bpl[(form, w.group)] for w in ws) / links
        frac[name] = {"algorithmic_GBs": rates[name] * per_update / 1e9,
                      "hbm_fraction": rates[name] * per_update / 1e9 / HBM_PEAK_GBS}
    out = {"lattices": len(ws), "total_links": links, "sweeps": sweeps, "launch_shapes": shapes,
           "roofline": frac,
           "f32_batched_link_updates_per_s": rates["f32_batched"],
           "f32c12_batched_link_updates_per_s": rates["f32c12_batched"],
           "speedup_f32c12": rates["f32c12_batched"] / rates["f64_one_by_one"],
           "f64_batched_link_updates_per_s": rates["f64_batched"],
           "f64_one_by_one_link_updates_per_s": rates["f64_one_by_one"],
           "speedup": rates["f32_batched"] / rates["f64_one_by_one"]}
    if precision_sweeps > 0:
        out["precision"] = batch_precision(P, descs, precision_sweeps)
    return out


def batch_precision(P, descs, n, therm=100, seeds=(None,)):
    """Every member of the batch, FP32 batch against FP64 batch: the same
    Haar starts and random numbers, `n` compound sweeps, the first `therm`
    discarded.  Each member's per-sweep difference of P, P_s, P_t and |L|
    gives a paired mean and binned error; the members' differences (of every
    replica: one per seed, which replaces the members' own seeds) are
    combined as an inverse-variance weighted mean, with the chi^2 per member
    about it.  Re L is not compared: the small members tunnel between centre
    sectors, so two decorrelated chains sit in different sectors for long
    stretches and the paired difference of Re L has no usable binned error;
    |L| does not depend on the sector."""
    import numpy as np
    keys = ("P", "P_s", "P_t", "absL")
    nbins = 20 if n - therm >= 2000 else 10
    deltas = {k: [] for k in keys}
    errs = {k: [] for k in keys}
    for seed in seeds:
        ds = descs if seed is None else [dict(d, seed=seed) for d in descs]
        series = {}
        for name, storage in (("f32", P.F32), ("f64", P.F64)):
            t0 = time.perf_counter()
            bt = P.Batch(ds, storage=storage)
            bt.autotune(N_HB, N_OR)
            obs = np.empty((n, len(ds), 4))
            for k in range(n):
                p, l = bt.run(1, N_HB, N_OR, measure=True)
                obs[k, :, :3] = p[:, :3]
                obs[k, :, 3] = np.hypot(l[:, 0], l[:, 1])
            bt.close()
            series[name] = obs[therm:]
            log(f"[batch precision] seed {seed}: {name} {n} compound sweeps in {time.perf_counter() - t0:.1f} s")
        for j, key in enumerate(keys):
            for i in range(len(ds)):
                d, e = paired(series["f32"][:, i, j], series["f64"][:, i, j], nbins)
                deltas[key].append(d)
                errs[key].append(e)
    out = {"sweeps": n, "thermalisation": therm, "bins": nbins, "bound": 1e-5,
           "member_seeds": [s for s in seeds if s is not None] or "workload"}
    for key in keys:
        delta, err = np.array(deltas[key]), np.array(errs[key])
        w = 1.0 / err ** 2
        dw = float(np.sum(w * delta) / np.sum(w))
        out[key] = {"delta": dw, "err": float(np.sqrt(1.0 / np.sum(w))),
                    "chi2_per_member": float(np.mean(((delta - dw) / err) ** 2)),
                    "max_abs_member_delta": float(np.max(np.abs(delta)))}
    dp = out["P"]
    # a run too short to resolve 1e-5 does not decide the bound
    out["P_within_bound"] = (bool(abs(dp["delta"]) + 2 * dp["err"] <= 1e-5) if dp["err"] <= 3e-6 else None)
    log(f"[batch] weighted <P> difference FP32 - FP64 {dp['delta']:.2e} +- {dp['err']:.1e}")
    return out


def copy_bandwidth(torch, mib: int = 2048, reps: int = 5) -> float:
    """Read + write GB/s of a plain device-to-device copy of `mib` MiB (the
    practical HBM ceiling beside the 8 TB/s peak), timed with events."""
    src = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2.0 * src.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# Working sweeps (one heat-bath sweep with NHIT = 10 and reunitarisation,
# plus the measurement; Haar start) on the lattice shapes of the paper's
# Table 1, with RANLUX luxury-level-3 streams (the paper's generator) and
# Philox beside them.
TABLE1_SHAPES = [{"group": 3, "dims": (32, 32, 32, 32), "beta": 6.0},
                 {"group": 2, "dims": (44, 44, 44, 44), "beta": 2.3}]


def run_ranlux_workloads(P, sweeps: int = 20):
    out = []
    for w in TABLE1_SHAPES:
        V = volume(w["dims"])
        row = {"group": w["group"], "lattice": list(w["dims"]), "beta": w["beta"]}
        for form, storage in (("f64", P.F64), ("f32", P.F32)):
            rates = {}
            for gen, rng in (("ranlux", P.RNG_RANLUX), ("philox", P.RNG_PHILOX)):
                lat = P.Lattice(w["group"], w["dims"], w["beta"], 0, storage=storage, rng=rng, seed=5,
                                start=P.HOT)
                lat.run(3, 1, 0, measure_every=1)  # includes the graph capture
                t0 = time.perf_counter()
                lat.run(sweeps, 1, 0, measure_every=1)
                rates[gen] = sweeps * 4 * V / (time.perf_counter() - t0)
                lat.close()
            row[form] = {"link_updates_per_s": rates["ranlux"], "philox_link_updates_per_s": rates["philox"]}
        log(f"[RANLUX working sweeps] SU({w['group']}) {w['dims']}: F64 {row['f64']['link_updates_per_s']:.3e}, "
            f"F32 {row['f32']['link_updates_per_s']:.3e} link updates/s")
        out.append(row)
    return out


# O(4) phi^4 model, the paper's other Table 1 workload: lattice, the
# paper's NHIT = 100 Metropolis hits per site, and a benchmark point in the
# model's coupling space (the paper gives none; delta gives about the 50%
# acceptance the paper mentions).
O4_KAPPA, O4_LAMBDA, O4_DELTA, O4_NHIT = 0.3, 1.0, 0.55, 100
O4_SIZES = (16, 32, 72)
O4_SOURCES = ["paper_1310_7087_amd/csrc/lat_on.hip", "paper_1310_7087_amd/csrc/lat_dev.hpp",
              "paper_1310_7087_amd/csrc/lat_types.hpp"]
# one wave64 VALU instruction per compute unit and cycle (4 SIMDs of 16
# lanes, 4 cycles per wave64 instruction), 256 CUs at 2.4 GHz
VALU_WAVE_INSTR_PEAK = 256 * 2.4e9


def o4_valu_per_hit():
    """VALU wave-instructions per Metropolis hit of the O(4) pass kernel from
    the committed rocprofv3 counters, if the kernel sources are unchanged."""
    path = os.path.join(ROOT, "profiles", "pmc_o4.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    h = hashlib.sha256()
    for f in O4_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if data.get("kernel_hash") != h.hexdigest()[:16]:
        return None
    return data.get("valu_wave_instructions_per_hit")


def run_o4(P, sweeps: int = 10, sizes=O4_SIZES):
    """The O(4) model on L^4 lattices: working sweeps (sweep + measurement)
    with RANLUX (the paper's generator) and Philox, FP64 and FP32 storage."""
    out = []
    for L in sizes:
        dims = (L,) * 4
        V = volume(dims)
        row = {"lattice": list(dims), "kappa": O4_KAPPA, "lambda": O4_LAMBDA, "delta": O4_DELTA, "nhit": O4_NHIT}
        for form, st in (("f64", P.F64), ("f32", P.F32)):
            for gen, rng in (("ranlux", P.RNG_RANLUX), ("philox", P.RNG_PHILOX)):
                f = P.ONField(4, dims, O4_KAPPA, O4_LAMBDA, 0.0, O4_DELTA, storage=st, rng=rng, seed=5,
                              nhit=O4_NHIT)
                f.run(2, 1)
                t0 = time.perf_counter()
                f.run(sweeps, 1)
                dt = (time.perf_counter() - t0) / sweeps
                row[f"{form}_{gen}"] = {"seconds_per_working_sweep": dt, "site_updates_per_s": V / dt,
                                        "hits_per_s": V * O4_NHIT / dt, "acceptance": f.acceptance()}
                f.close()
        log(f"[O(4) {L}^4] F64 RANLUX {row['f64_ranlux']['seconds_per_working_sweep'] * 1e3:.2f} ms, "
            f"Philox {row['f64_philox']['seconds_per_working_sweep'] * 1e3:.2f} ms per working sweep")
        out.append(row)
    # the pass kernel's VALU issue rate at 32^4 (FP64, Philox)
    f = P.ONField(4, (32,) * 4, O4_KAPPA, O4_LAMBDA, 0.0, O4_DELTA, storage=P.F64, rng=P.RNG_PHILOX, seed=5,
                  nhit=O4_NHIT)
    f.sweep(2)
    ms = f.profile(20)
    f.close()
    hits = volume((32,) * 4) // 2 * O4_NHIT
    per_hit = o4_valu_per_hit()
    roof = {"bound": "alu", "kernel": "on_pass<f64, N=4, philox>", "avg_launch_us": ms * 1e3,
            "hits_per_launch": hits, "hits_per_s": hits / (ms * 1e-3), "unit": "VALU wave-instructions/s",
            "peak": VALU_WAVE_INSTR_PEAK, "valu_wave_instructions_per_hit": per_hit,
            "achieved": None, "frac": None}
    if per_hit:
        roof["achieved"] = hits * per_hit / (ms * 1e-3)
        roof["frac"] = roof["achieved"] / VALU_WAVE_INSTR_PEAK
    return {"lattices": out, "o4_32_pass_roofline": roof}


def cpu_baseline(steps: int):
    import oracle as O
    cores = len(os.sched_getaffinity(0))
    O.set_threads(cores)
    V = volume(DIMS)
    ref = O.Lattice(3, DIMS, BETA, flux=FLUX, rng=O.RNG_PHILOX, seed=3, start=O.COLD)
    t0 = time.perf_counter()
    for _ in range(steps):
        ref.sweep(N_HB, N_OR)
        ref.measure()
    dt = time.perf_counter() - t0
    # one thread on an eighth of the volume (about the same time per update)
    O.set_threads(1)
    small = (16, 16, 16, 8)
    ref1 = O.Lattice(3, small, BETA, flux=FLUX, rng=O.RNG_PHILOX, seed=3, start=O.COLD)
    t0 = time.perf_counter()
    ref1.sweep(N_HB, N_OR)
    dt1 = time.perf_counter() - t0
    O.set_threads(cores)
    return {"value": steps * (N_HB + N_OR) * 4 * V / dt, "unit": "link updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{steps} step(s) (1 HB + 4 OR compound sweep + plaquette/Polyakov) of the same "
                      f"SU(3) 32^3x8 lattice from the cold start, FP64, {cores} OpenMP threads",
            "seconds": dt, "cpu_model": cpu_model(),
            "single_thread_value": (N_HB + N_OR) * 4 * volume(small) / dt1,
            "single_thread_sample": "one (1 HB + 4 OR) compound sweep of SU(3) 16^3x8 from the cold start, 1 thread"}


def traffic_for(kernel: str, form: str):
    """Bytes per launch between the L2 caches and the memory fabric (reads
    plus writes; they are served by HBM or by the last-level cache in front
    of it) from the committed rocprofv3 PMC summary, valid only while the
    kernel sources are unchanged since it was taken."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            data = json.load(fh)
    except ValueError:
        return None
    if data.get("kernel_hash") != kernel_hash():
        return None
    entry = data.get("kernels", {}).get(f"{form}:{kernel}")
    return None if entry is None else entry.get("fabric_bytes_per_launch")


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--forms", default="f64,f32,f32c12,f64c12",
                    help="storage forms to time; the first is the headline value")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the 64^3x16 and batch measurements")
    ap.add_argument("--precision-sweeps", type=int, default=1000,
                    help="compound sweeps of the batch precision comparison (0 skips it)")
    ap.add_argument("--precision-steps", type=int, default=20000,
                    help="measured compound sweeps per form of the paired FP32-vs-FP64 precision leg "
                         "(0 skips it)")
    ap.add_argument("--precision-forms", default="f32c12,f32",
                    help="storage forms compared with FP64 in the precision leg")
    ap.add_argument("--batch-precision-seeds", default="",
                    help="member seeds of independent replicas of the batch precision comparison "
                         "(default: the workload's own seeds, one replica)")
    ap.add_argument("--precision-large-steps", type=int, default=0,
                    help="measured compound sweeps of the FP32 12-real vs FP64 comparison on 64^3x16 "
                         "(0 skips it)")
    ap.add_argument("--precision-large-forms", default="f32c12",
                    help="forms compared with FP64 on 64^3x16 (f64c12 adds the FP64 12-real control)")
    ap.add_argument("--precision-large-seed", type=int, default=23, help="seed of the 64^3x16 pair")
    ap.add_argument("--precision-seeds", default="3,4,5",
                    help="seeds of the independent replicas of the precision leg")
    ap.add_argument("--precision-only", action="store_true",
                    help="only run the precision leg and print its JSON line")
    ap.add_argument("--cpu-steps", type=int, default=8,
                    help="steps of the CPU oracle in the bounded baseline sample (about 1 s each on 16 cores)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (a known-size kernel that "
                         "calibrates the profiler's HBM byte counters)")
    ap.add_argument("--o4-only", action="store_true",
                    help="only run the O(4) model's lattices and print their JSON line")
    ap.add_argument("--o4-sizes", default="16,32,72", help="O(4) lattice extents L (L^4) to run")
    ap.add_argument("--batch-only", action="store_true",
                    help="only run the 64-lattice batch leg, without its precision sweeps (after the "
                         "--copy-mib calibration copy), and print its JSON line")
    ap.add_argument("--large-only", action="store_true",
                    help="only run the SU(3) 64^3x16 leg (after the --copy-mib calibration copy) and print "
                         "its JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the lattice is resident on a single MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        return 2
    if "LAT_TUNE_CACHE" not in os.environ:
        # launch shapes tuned once per lattice shape and reused by the later legs
        import atexit
        import tempfile
        fd, path = tempfile.mkstemp(prefix="lat_tune_", suffix=".json")
        os.close(fd)
        os.remove(path)
        os.environ["LAT_TUNE_CACHE"] = path
        atexit.register(lambda: os.path.exists(path) and os.remove(path))
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    import paper_1310_7087_amd as P

    seeds = tuple(int(x) for x in args.precision_seeds.split(",") if x.strip())
    pforms = tuple(x.strip() for x in args.precision_forms.split(",") if x.strip())
    large_forms = tuple(x.strip() for x in args.precision_large_forms.split(",") if x.strip())
    if args.precision_only:
        res = {"workload": "su3_32^3x8_beta5.9_flux1_cold_philox_1hb4or"}
        if args.precision_steps > 0:
            res["precision"] = precision_leg(P, args.precision_steps, forms=pforms, seeds=seeds)
        if args.precision_large_steps > 0:
            res["precision_64x16"] = precision_large(P, args.precision_large_steps, seed=args.precision_large_seed,
                                                     forms=large_forms)
        if args.precision_sweeps > 0:
            from inputs import batch_workloads
            descs = [dict(group=w.group, dims=w.dims, beta=w.beta, flux=w.flux, seed=w.seed, start=w.start,
                          lattice_id=w.lattice_id) for w in batch_workloads(64, seed=11)]
            bseeds = tuple(int(x) for x in args.batch_precision_seeds.split(",") if x.strip()) or (None,)
            res["batch_precision"] = batch_precision(P, descs, args.precision_sweeps, seeds=bseeds)
        print(json.dumps(res), flush=True)
        return 0

    o4_sizes = tuple(int(x) for x in args.o4_sizes.split(",") if x.strip())
    if args.o4_only:
        print(json.dumps({"o4": run_o4(P, sizes=o4_sizes)}), flush=True)
        return 0

    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.copy_mib} MiB done")
        del src, dst
    if args.large_only:
        print(json.dumps({"su3_64x16": run_large(P)}), flush=True)
        return 0
    if args.batch_only:
        print(json.dumps({"batch_64_lattices": run_batch(P, precision_sweeps=0)}), flush=True)
        return 0
    copy_gbs = copy_bandwidth(torch)

    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    results = {}
    for f in forms:
        results[f] = run_form(P, f, args.steps, args.warmup)
        log(f"[{f}] {results[f]['link_updates_per_s']:.3e} link updates/s, "
            f"{results[f]['algorithmic_GBs']:.0f} GB/s algorithmic")
    head = forms[0]
    r = results[head]
    # dominant kernel: the pass kind with the larger share of a compound sweep
    share_hb = N_HB * 8 * r["hb_pass_us"]
    share_or = N_OR * 8 * r["or_pass_us"]
    kname = "or_pass" if share_or >= share_hb else "hb_pass"
    t_us = r[kname + "_us"]
    achieved = r["pass_bytes"] / (t_us * 1e-6) / 1e9
    kshape = r["launch_shape"]["overrelaxation" if kname == "or_pass" else "heat_bath"]
    kfn = "su3_pass_lq" if kshape["stage_lds"] else "su3_pass"
    roofline = {"bound": "hbm", "kernel": f"{kfn}<{head},{'overrelax' if kname == 'or_pass' else 'heatbath'}>",
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic_for(kname, head),
                "traffic_kind": "L2-to-fabric bytes per launch (FETCH_SIZE and WRITE_SIZE, copy-calibrated)",
                "avg_launch_us": t_us,
                "algorithmic_bytes_per_launch": r["pass_bytes"],
                # the FP64 32^3x8 lattice (151 MB) fits the 256 MB last-level cache in front of
                # HBM; su3_64x16 (2.4 GB) gives the pass against HBM alone
                "lattice_bytes": 4 * volume(DIMS) * BYTES_PER_LINK[head],
                "fits_last_level_cache": 4 * volume(DIMS) * BYTES_PER_LINK[head] < 256 * 2 ** 20}
    out = {
        "metric": "SU(3) link updates/s at 32^3x8 HB+OR",
        "value": r["link_updates_per_s"],
        "unit": "link updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": "su3_32^3x8_beta5.9_flux1_cold_philox_1hb4or_plus_measure",
                   "lattice": list(DIMS), "beta": BETA, "flux_quanta": FLUX, "n_hb": N_HB, "n_or": N_OR,
                   "storage": head, "parallelism": "single_gpu"},
        "hbm_fraction_algorithmic": r["hbm_fraction"],
        "copy_GBs": copy_gbs,
        "roofline": roofline,
        "forms": {f: {k: v for k, v in results[f].items() if k != "pass_bytes"} for f in forms},
    }
    if "f64" in results:
        for f in forms:
            if f != "f64":
                fr = out["forms"][f]
                fr["speedup_vs_f64"] = results[f]["link_updates_per_s"] / results["f64"]["link_updates_per_s"]
                # the same start and random numbers: the first sweeps track the
                # FP64 trajectory until rounding differences grow
                fr["early_abs_delta_P_vs_f64"] = [
                    abs(a - b) for a, b in zip(results[f]["early_plaquettes"], results["f64"]["early_plaquettes"])]
    if not args.no_extras:
        flux = run_flux_observables(P, forms)
        flux["flux_1"] = {f: results[f]["observables"] for f in forms}
        out["observables_by_flux"] = flux
    if args.precision_steps > 0:
        out["precision"] = precision_leg(P, args.precision_steps, forms=pforms, seeds=seeds)
    if args.precision_large_steps > 0:
        out["precision_64x16"] = precision_large(P, args.precision_large_steps, seed=args.precision_large_seed,
                                                     forms=large_forms)
    if not args.no_extras:
        out["su3_64x16"] = run_large(P)
        out["batch_64_lattices"] = run_batch(P, precision_sweeps=args.precision_sweeps)
        out["ranlux_working_sweeps"] = run_ranlux_workloads(P)
        out["o4"] = run_o4(P, sizes=o4_sizes)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
