"""Solver parity on grids with 2048-point axes (the large workload's FFT
length), against the FP64 oracle.

The large workload (1024^2 padded to 2048^2, L = 3) runs 2048-point column
passes (the first pass, the middle [F_0 D_3 F_0] pass and its adjoint, the
last pass fused with the next iteration's first) and 2048-point row passes
(the middle [F_1 D_2 F_1] pair and the GD / spectral turnaround).  Two thin
grids, 2048 x 128 and 128 x 2048, run each of those kernels on the tile
choice the tuner makes for the large workload (four-column tiles, one-row
tiles, phases evaluated with sincos) while keeping the oracle's explicit DFT
matrices affordable, and again with the wide shape's eight-column tiles
(radix-16 stages) for the [F D F] column passes; GD iterates (section
II-B.1, Eq. (2)) are compared at steps 1, 7 and 50, power-iteration iterates
(Eq. (3)-(4)) at 1 and 10, and the loss trace over 7 steps.  The full 2048^2
grid then takes one GD step and one power iteration from the same start as
the oracle, with the tuner's own choice and with both pinned ones.  Bars: 1e-4 on iterates after global-phase
alignment, 1e-4 on loss-trace entries.
"""
import numpy as np
import pytest

import oracle
import sr_inputs
from gpu_helpers import aligned, make_plan, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_IT = 1e-4
LARGE_CHOICE = "4,1,0"  # column tile 4, row tile 1, sincos phases
# eight-column single-buffered tiles of the sixteen-elements-per-thread shape
# (radix-16 stages) for the [F D F] column passes, the rest as above
WIDE_CHOICE = f"{8 | 256 | 1024},1,0"


def _gd(plan, y, x0, iters, eta, dev, loss=False):
    import torch
    import paper_2409_05734_amd as srpr
    xd = to_dev(x0.ravel().astype(np.complex64), dev)
    lt = torch.zeros(iters, dtype=torch.float32, device=dev) if loss else None
    srpr.sr_gd_solve(plan, to_dev(y.ravel().astype(np.float32), dev), xd, iters, eta, lt)
    torch.cuda.synchronize()
    return to_host(xd), (to_host(lt) if loss else None)


def _spec(plan, y, v0, iters, dev):
    import torch
    import paper_2409_05734_amd as srpr
    out = torch.empty(plan.n_total, dtype=torch.complex64, device=dev)
    srpr.sr_spectral_init(plan, to_dev(y.ravel().astype(np.float32), dev), to_dev(v0.ravel(), dev), iters, -1.0, out)
    torch.cuda.synchronize()
    return to_host(out)


@pytest.mark.parametrize("choice", [LARGE_CHOICE, WIDE_CHOICE])
@pytest.mark.parametrize("n_shape,m_shape", [((600, 102), (2048, 128)), ((102, 600), (128, 2048))])
def test_gd_and_spectral_on_2048_point_axes(gpu, monkeypatch, n_shape, m_shape, choice):
    monkeypatch.setenv("SR_TUNE_FORCE", choice)
    rng = np.random.default_rng(sum(m_shape))
    L = 3
    th = sr_inputs.phase_masks(rng, L, m_shape)
    xs = sr_inputs.complex_gaussian(rng, n_shape)
    op = oracle.StructuredOperator(th, n_shape)
    y = oracle.measurements(xs, th).astype(np.float32)
    x0 = (xs + 0.5 * sr_inputs.complex_gaussian(rng, n_shape)).astype(np.complex64)
    eta = np.float32(oracle.default_step(op, y, 0.2))
    plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
    print(f"large-axis GD/spectral parity: {n_shape} -> {m_shape}, L = {L}, tiles {choice}", flush=True)

    _, its, losses = oracle.gd_solve(op, y, x0, 50, float(eta), return_iterates=True, return_loss=True)
    for k in (1, 7, 50):
        xg, _ = _gd(plan, y, x0, k, eta, gpu)
        assert aligned(xg.reshape(n_shape), its[k - 1]) <= TOL_IT, k
    _, lg = _gd(plan, y, x0, 7, eta, gpu, loss=True)
    assert np.max(np.abs(lg - losses[:7]) / losses[:7]) <= TOL_IT

    yp = sr_inputs.poisson_counts(rng, oracle.measurements(xs, th), 1000.0)
    v0 = sr_inputs.complex_gaussian(rng, n_shape)
    _, sits = oracle.spectral_init(op, yp, v0, 10, -1.0, return_iterates=True)
    scale = np.sqrt(np.sum(yp.astype(np.float64)) / (op.m * op.c))
    for k in (1, 10):
        sg = _spec(plan, yp, v0, k, gpu)
        assert rel_l2(sg.reshape(n_shape), scale * sits[k - 1]) <= TOL_IT, k


def test_full_large_grid_one_step(gpu, monkeypatch):
    """1024^2 image padded to 2048^2, L = 3, Poisson noise at 1000 photons
    (the large workload's inputs): one GD step from a start near the image and
    one power iteration, on the tuner's choice and on both pinned ones."""
    d = sr_inputs.large_2d(4)
    n_shape, m_shape, L = d["n_shape"], d["m_shape"], d["layers"]
    th, xs = d["theta"], d["x_star"]
    op = oracle.StructuredOperator(th, n_shape)
    y = sr_inputs.poisson_counts(d["noise_rng"], oracle.measurements(xs, th), d["photons"])
    rng = np.random.default_rng(8)
    x0 = (xs + 0.3 * sr_inputs.complex_gaussian(rng, n_shape)).astype(np.complex64)
    eta = np.float32(oracle.default_step(op, y, d["mu"]))
    print("large-grid one-step parity: oracle", flush=True)
    x1 = oracle.gd_solve(op, y, x0, 1, float(eta))
    s1 = oracle.spectral_init(op, y, d["v0"], 1, d["lam"])
    for force in (None, LARGE_CHOICE, WIDE_CHOICE):
        if force is None:
            monkeypatch.delenv("SR_TUNE_FORCE", raising=False)
        else:
            monkeypatch.setenv("SR_TUNE_FORCE", force)
        print(f"large-grid one-step parity: GPU, tiles {force or 'tuned'}", flush=True)
        plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
        xg, _ = _gd(plan, y, x0, 1, eta, gpu)
        assert aligned(xg.reshape(n_shape), x1) <= TOL_IT, force
        sg = _spec(plan, y, d["v0"], 1, gpu)
        assert rel_l2(sg.reshape(n_shape), s1) <= TOL_IT, force
        del plan
