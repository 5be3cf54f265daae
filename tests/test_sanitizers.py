"""CPU sanitizer runs (no GPU): the library's host-side file parsers (both
checkpoint formats and the tuning cache, lat_hostio.cpp) fuzzed with valid,
truncated, corrupted and crafted inputs, and the FP64 oracle exercised
through its C interface, each built with AddressSanitizer and
UndefinedBehaviorSanitizer (any report aborts the run)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXT = os.path.join(ROOT, "tests", "ext")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


def build_and_run(tmp_path, name, sources, extra, env_extra=None, timeout=600):
    exe = str(tmp_path / name)
    subprocess.run(["g++", "-std=c++17", *SAN, *extra, *sources, "-o", exe], check=True, capture_output=True,
                   text=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:allocator_may_return_null=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", **(env_extra or {}))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def test_host_io_fuzzed_under_sanitizers(tmp_path):
    out = build_and_run(tmp_path, "fuzz_hostio",
                        [os.path.join(EXT, "fuzz_hostio.cpp"),
                         os.path.join(ROOT, "paper_1310_7087_amd", "csrc", "lat_hostio.cpp")],
                        ["-I", os.path.join(ROOT, "paper_1310_7087_amd", "csrc")], {"FUZZ_DIR": str(tmp_path)})
    assert "ok" in out


def test_oracle_under_sanitizers(tmp_path):
    out = build_and_run(tmp_path, "oracle_sanitized",
                        [os.path.join(EXT, "oracle_sanitized.cpp"), os.path.join(ROOT, "oracle", "oracle.cpp")],
                        ["-I", os.path.join(ROOT, "oracle"), "-fopenmp", "-ffp-contract=off"])
    assert "ok" in out
