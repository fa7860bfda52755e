"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(host instrumentation only): csrc/host_check.cpp, built by
paper_2409_05734_amd/build.py against host-sanitized objects, runs every
argument and shape check of plan creation and of the entry points without a
GPU (and, on a GPU, whole plans through the tuner and every schedule)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECK = os.path.join(ROOT, "paper_2409_05734_amd", "sr_host_check")


def _run(args, timeout):
    if not os.path.exists(CHECK):
        pytest.fail("sr_host_check is not built (python paper_2409_05734_amd/build.py --host-check)")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([CHECK] + args, capture_output=True, text=True, timeout=timeout, env=env)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_argument_checks_under_sanitizers():
    out = _run(["--no-gpu"], 120)
    assert "host checks passed" in out


@pytest.mark.gpu
def test_plans_under_sanitizers(gpu):
    out = _run([], 300)
    assert "host checks passed" in out
