"""bench.py's JSON line (GPU): one short run with the CPU baseline and one
side workload, its keys and the relations between its figures (throughput
from the step time, roofline fraction from the algorithmic bytes and the
measured iteration time)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line(gpu):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1",
                        "--extras", "latency_floor"], capture_output=True, text=True, timeout=280, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    d = json.loads(r.stdout.strip().splitlines()[-1])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["higher_is_better"] is True and d["scaling"] == "weak" and d["vs_baseline"] is None
    assert d["data"] == "synthetic" and "workload" in d["config"]
    # one step = one GD solve of gd_iters_per_step iterations
    per_step = d["config"]["gd_iters_per_step"]
    assert abs(d["value"] - per_step * 1e3 / d["ms_per_step"]) <= 1e-9 * d["value"]
    rf = d["roofline"]
    assert rf["bound"] in ("hbm", "mfma", "alu") and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["bytes_per_unit"] == 17825792
    assert abs(rf["achieved"] - rf["bytes_per_unit"] / (d["gd_iteration_us"] * 1e-6) / 1e9) <= 1e-9 * rf["achieved"]
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) <= 1e-12
    assert rf["traffic"] is None or rf["traffic"] > 0
    # the iteration time from the solve's events and the wall clock's throughput agree
    assert 0.5 < d["value"] * d["gd_iteration_us"] * 1e-6 < 1.5
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["unit"] == d["unit"]
    assert d["extras"]["latency_floor"]["tiny_kernel_us"] > 0
