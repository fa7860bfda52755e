"""The measurement model bench.py reports against (CPU only).

The roofline fraction in the JSON line is algorithmic bytes per GD iteration
of the fused pass schedule (section III, Eq. (5): U, the phase diagonals and
the axis transforms, pass by pass) divided by the measured iteration time.
These checks pin that byte count to per-pass sums written out by hand for
the 256^2 -> 512^2, L = 2 image and the 1024^2 -> 2048^2, L = 3 grid, and the
compulsory-byte floor; and the benchmark's refusal to run on more than one
GPU.
"""
import importlib.util
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _bench():
    spec = importlib.util.spec_from_file_location("bench_model", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_headline_bytes_per_gd_iteration():
    b = _bench()
    n, m, mc = 256 * 256, 512 * 512, 512 * 256  # signal, grid, support columns (M1 x N2)
    c64, f32 = 8, 4
    passes = [
        c64 * n + f32 * n + c64 * mc,   # [U D1 F0]: x, theta_1 on the support, compact buffer out
        c64 * mc + f32 * m + c64 * m,   # [F1 D2 F1]: compact in, theta_2, grid out
        c64 * m + f32 * m + c64 * m,    # turnaround: grid in, y, grid out
        c64 * m + f32 * m + c64 * mc,   # [F1^H D2^* F1^H]: grid in, theta_2, compact out
        c64 * mc + f32 * n + 2 * c64 * n,  # [F0^H D1^* U^H] + update: compact in, theta_1, x in and out
    ]
    assert passes == [1835008, 4194304, 5242880, 4194304, 2359296]
    assert b.schedule_bytes_gd((256, 256), (512, 512), 2) == sum(passes) == 17825792
    # floor: x in and out, y, theta_1 on the support, theta_2 on the grid
    assert b.compulsory_bytes_gd((256, 256), (512, 512), 2) == 2 * c64 * n + f32 * m + f32 * n + f32 * m == 3407872


def test_large_grid_bytes_per_gd_iteration():
    b = _bench()
    n, m, mc = 1024 * 1024, 2048 * 2048, 2048 * 1024
    passes = [8 * n + 4 * n + 8 * mc,          # [U D1 F0]
              8 * mc + 4 * m + 8 * m,          # [F1 D2 F1]
              8 * m + 4 * m + 8 * m,           # [F0 D3 F0]
              8 * m + 4 * m + 8 * m,           # turnaround on axis 1
              8 * m + 4 * m + 8 * m,           # [F0^H D3^* F0^H]
              8 * m + 4 * m + 8 * mc,          # [F1^H D2^* F1^H]
              8 * mc + 4 * n + 16 * n]         # [F0^H D1^* U^H] + update
    assert b.schedule_bytes_gd((1024, 1024), (2048, 2048), 3) == sum(passes) == 452984832


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr
