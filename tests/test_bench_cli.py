"""Host-side checks of bench.py's contract that need no GPU: more than one
GPU is refused with a message, and the roofline helpers read the committed
profiles only while the kernel sources they were taken on are unchanged."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_committed_traffic_is_used_only_for_the_kernels_it_was_taken_on(tmp_path, monkeypatch):
    with open(os.path.join(ROOT, "profiles", "pmc_traffic.json")) as fh:
        data = json.load(fh)
    real = bench.kernel_hash()
    t = bench.traffic_for("or_pass", "f64")
    if data["kernel_hash"] != real:
        assert t is None  # the kernels changed since the counters were taken: reported as null
    else:
        alg = 4.5 * 32 ** 3 * 8 * 144
        # the L2 fetches at least the algorithmic bytes, and not arbitrarily more
        assert 0.9 * alg < t < 2.5 * alg
    # a figure taken on the current kernels is used, a stale one is hidden
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_hash", lambda: real)
    (tmp_path / "profiles").mkdir()
    entry = {"kernels": {"f64:or_pass": {"fabric_bytes_per_launch": 1.5e8}}}
    (tmp_path / "profiles" / "pmc_traffic.json").write_text(json.dumps(dict(entry, kernel_hash=real)))
    assert bench.traffic_for("or_pass", "f64") == 1.5e8
    (tmp_path / "profiles" / "pmc_traffic.json").write_text(json.dumps(dict(entry, kernel_hash="0" * 16)))
    assert bench.traffic_for("or_pass", "f64") is None


def test_committed_valu_count_is_used_only_for_the_current_o4_kernel():
    import hashlib
    with open(os.path.join(ROOT, "profiles", "pmc_o4.json")) as fh:
        data = json.load(fh)
    h = hashlib.sha256()
    for f in bench.O4_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    per_hit = bench.o4_valu_per_hit()
    if data.get("kernel_hash") == h.hexdigest()[:16]:
        assert per_hit is not None and 1.0 < per_hit < 10.0
    else:
        assert per_hit is None  # counters of an older kernel: reported as null


def test_binned_error_matches_independent_samples():
    """The binned standard error of the precision legs equals sigma/sqrt(n)
    for independent samples (within the spread of a 50-bin estimate)."""
    import numpy as np
    rng = np.random.default_rng(7)
    x = rng.normal(0.25, 2.0, 100000)
    m, e = bench.binned(x, 50)
    assert abs(m - 0.25) < 5 * 2.0 / np.sqrt(x.size)
    assert 0.7 < e / (2.0 / np.sqrt(x.size)) < 1.3


def test_binned_error_sees_autocorrelation():
    """For an AR(1) series with integrated autocorrelation time
    (1 + a) / (1 - a) the binned error grows by its square root, which a
    naive sigma/sqrt(n) would miss."""
    import numpy as np
    rng = np.random.default_rng(8)
    a, n = 0.8, 200000
    x = np.empty(n)
    x[0] = 0.0
    eps = rng.normal(0.0, 1.0, n)
    for i in range(1, n):
        x[i] = a * x[i - 1] + eps[i]
    sigma = 1.0 / np.sqrt(1 - a * a)
    tau = (1 + a) / (1 - a)
    _, e = bench.binned(x, 50)
    assert 0.7 < e / (sigma * np.sqrt(tau / n)) < 1.3


def test_paired_difference_cancels_the_shared_part():
    """Two coupled chains share most of their fluctuation: the paired error
    of their difference reflects only the unshared part."""
    import numpy as np
    rng = np.random.default_rng(9)
    n = 100000
    shared = rng.normal(0.0, 10.0, n)
    x = shared + rng.normal(1e-3, 0.1, n)
    y = shared + rng.normal(0.0, 0.1, n)
    d, e = bench.paired(x, y)
    expect = np.sqrt(2) * 0.1 / np.sqrt(n)
    assert 0.7 < e / expect < 1.3
    assert abs(d - 1e-3) < 5 * expect
