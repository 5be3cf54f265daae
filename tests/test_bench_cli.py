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


def test_committed_traffic_matches_the_current_kernels():
    with open(os.path.join(ROOT, "profiles", "pmc_traffic.json")) as fh:
        data = json.load(fh)
    assert data["kernel_hash"] == bench.kernel_hash()
    t = bench.traffic_for("or_pass", "f64")
    alg = 4.5 * 32 ** 3 * 8 * 144
    # the L2 fetches more than the algorithmic bytes, but not arbitrarily more
    assert alg < t < 2.5 * alg


def test_committed_valu_count_matches_the_current_o4_kernel():
    per_hit = bench.o4_valu_per_hit()
    assert per_hit is not None and 1.0 < per_hit < 10.0
