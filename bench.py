"""Benchmark: gradient-descent iterations per second of structured random phase
retrieval on one MI355X, for the 2D image workload (256x256 complex image,
zero-padded to 512x512 so alpha = 4, L = 2 random phase layers, Poisson noise
at 1000 photons per pixel, complex64).

One step = one GD solve of 500 iterations (Eq. (2)) started from the spectral
estimate; the spectral initialisation (100 power iterations, Eq. (3)-(4)) and
single A / A^H applications are timed in the same run and reported beside it.
Inputs are synthetic and seeded and live in HBM before the timed region.

Prints one JSON line.  `python bench.py --steps K --warmup W`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
GD_ITERS = 500
PI_ITERS = 100


def schedule_bytes_gd(n_shape, m_shape, L):
    """Algorithmic HBM bytes of one GD iteration under the fused pass schedule.

    Pass 1 reads x (8n) and the support part of theta_1 (4n), writes the
    compact M1 x N2 buffer; each later pass reads and writes its buffer
    (compact next to the padding, full m-grid elsewhere) plus its phases
    (4 B per grid point) or measurements; the last pass reads the compact
    buffer, theta_1's support part and x, and writes x."""
    N1, N2 = n_shape
    M1, M2 = m_shape
    n, m, mc = N1 * N2, M1 * M2, M1 * N2
    b = 0
    b += 8 * n + 4 * n + 8 * mc                       # [U D1 F0]
    for k in range(2, L + 1):                          # [F D_k F]
        b += 8 * (mc if k == 2 else m) + 4 * m + 8 * m
    b += 8 * (mc if L == 1 else m) + 4 * m + 8 * (mc if L == 1 else m)  # turnaround (+ y)
    for k in range(L, 1, -1):                          # [F^H D_k^* F^H]
        b += 8 * m + 4 * m + 8 * (mc if k == 2 else m)
    b += 8 * mc + 4 * n + 8 * n + 8 * n               # [F0^H D1^* U^H] + x update
    return b


def schedule_bytes_op(n_shape, m_shape, L):
    """Algorithmic bytes of one A application (x in, z out)."""
    N1, N2 = n_shape
    M1, M2 = m_shape
    n, m, mc = N1 * N2, M1 * M2, M1 * N2
    b = 8 * n + 4 * n + 8 * mc
    for k in range(2, L + 1):
        b += 8 * (mc if k == 2 else m) + 4 * m + 8 * m
    b += 8 * (mc if L == 1 else m) + 8 * m
    return b


def cpu_baseline(d, y, x0, eta, budget_s=12.0):
    """Time the FP64 oracle's GD iterations on this host (bounded sample)."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    op = oracle.StructuredOperator(d["theta"], d["n_shape"])
    x = x0.astype(np.complex128)
    oracle.gd_solve(op, y, x, 1, eta)  # warm the DFT-matrix cache
    it, t0 = 0, time.perf_counter()
    while True:
        x = oracle.gd_solve(op, y, x, 1, eta)
        it += 1
        el = time.perf_counter() - t0
        if el >= budget_s or it >= 200:
            break
    return {"value": it / el, "unit": "GD iters/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{it} GD iterations of the FP64 explicit-DFT oracle on the same 256^2 -> 512^2, L=2 "
                      f"problem ({el:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU build: the benchmark runs on one GPU only; use --gpus 1"}))
        sys.exit(2)

    import torch
    import paper_2409_05734_amd as srpr
    import sr_inputs

    dev = torch.device("cuda:0")
    d = sr_inputs.image_2d(1)
    n_shape, m_shape, L = d["n_shape"], d["m_shape"], d["layers"]
    n, m = int(np.prod(n_shape)), int(np.prod(m_shape))
    plan = srpr.Plan([srpr.Problem(n_shape, m_shape, L)], d["theta"])
    stream = plan.stream

    # measurements: noiseless intensities from the library's own forward
    # operator, then Poisson photon noise drawn on the host
    xs = torch.from_numpy(d["x_star"].ravel()).to(dev)
    yclean = torch.empty(m, dtype=torch.float32, device=dev)
    srpr.sr_forward(plan, xs, None, yclean)
    torch.cuda.synchronize()
    y_h = sr_inputs.poisson_counts(d["noise_rng"], yclean.cpu().numpy(), d["photons"])
    y = torch.from_numpy(y_h).to(dev)
    v0 = torch.from_numpy(d["v0"].ravel()).to(dev)
    x0 = torch.empty(n, dtype=torch.complex64, device=dev)
    eta = float(d["mu"] * m / float(y_h.astype(np.float64).mean()))  # mu / (c * mean(y)), c = 1/m

    # spectral initialisation (timed separately)
    srpr.sr_spectral_init(plan, y, v0, PI_ITERS, d["lam"], x0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    srpr.sr_spectral_init(plan, y, v0, PI_ITERS, d["lam"], x0)
    e1.record(stream)
    torch.cuda.synchronize()
    pi_ms = e0.elapsed_time(e1)

    x = torch.empty_like(x0)
    for _ in range(args.warmup):
        x.copy_(x0)
        srpr.sr_gd_solve(plan, y, x, GD_ITERS, eta)
    torch.cuda.synchronize()

    # timed region: K GD solves of 500 iterations each (x reset between solves
    # by a 2 MB device copy, included)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        x.copy_(x0)
        ev[i][0].record(stream)
        srpr.sr_gd_solve(plan, y, x, GD_ITERS, eta)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    solve_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = wall * 1e3 / args.steps
    gd_rate = GD_ITERS * args.steps / wall

    # single-operator timing
    z = torch.empty(m, dtype=torch.complex64, device=dev)
    r = torch.randn(m, dtype=torch.complex64, device=dev)
    xa = torch.empty(n, dtype=torch.complex64, device=dev)
    reps = 200
    for _ in range(10):
        srpr.sr_forward(plan, xs, z, None)
    a0, a1, a2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    a0.record(stream)
    for _ in range(reps):
        srpr.sr_forward(plan, xs, z, None)
    a1.record(stream)
    for _ in range(reps):
        srpr.sr_adjoint(plan, r, xa)
    a2.record(stream)
    torch.cuda.synchronize()
    fwd_us = a0.elapsed_time(a1) * 1e3 / reps
    adj_us = a1.elapsed_time(a2) * 1e3 / reps
    op_bytes = schedule_bytes_op(n_shape, m_shape, L)

    # quality check of the solve just timed
    xh = x.cpu().numpy().astype(np.complex128)
    xt = d["x_star"].ravel().astype(np.complex128)
    cos = float(abs(np.vdot(xh, xt)) / (np.linalg.norm(xh) * np.linalg.norm(xt)))

    gd_bytes = schedule_bytes_gd(n_shape, m_shape, L)
    solve_avg_ms = float(np.mean(solve_ms))
    achieved = gd_bytes * GD_ITERS / (solve_avg_ms * 1e-3) / 1e9
    out = {
        "metric": "GD iters/s (n=256^2, alpha=4, L=2)",
        "value": gd_rate,
        "unit": "GD iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "2D image 256x256 -> 512x512 (alpha=4), L=2, Poisson 1000 photons, "
                               "GD solve of 500 iterations per step", "n": n, "m": m, "layers": L,
                   "gd_iters_per_step": GD_ITERS},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "GD iteration (fused passes)", "bytes_per_unit": gd_bytes},
        "operator": {"A_us": fwd_us, "AH_us": adj_us, "A_GBps": op_bytes / (fwd_us * 1e-6) / 1e9,
                     "AH_GBps": op_bytes / (adj_us * 1e-6) / 1e9, "bytes_per_application": op_bytes},
        "spectral_init": {"iters": PI_ITERS, "ms": pi_ms, "iters_per_s": PI_ITERS / (pi_ms * 1e-3)},
        "cosine_similarity": cos,
    }
    if not args.no_cpu_baseline:
        xr = x0.cpu().numpy().reshape(n_shape)
        out["cpu_baseline"] = cpu_baseline(d, y_h.reshape(m_shape), xr, eta)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
