"""Divergence and bad inputs surface as SR_E_NONFINITE at sr_plan_sync.

A GD or spectral solve (section II-B, Eq. (2)-(4)) whose result holds NaN or
Inf -- NaN measurements, or a step so large that the iterates overflow --
raises the plan's non-finite flag on the GPU; sr_plan_sync reports it once
and clears it.  Covered: the 2D pass kernels (direct and graph-replayed
iterations, loss traces), stacked problems, level launches of uneven
problems, the LDS-resident 1D and 2D solvers and the dense model.  Finite
solves, including all-zero measurements, leave the flag down.  (NaN and Inf
here are values flowing through ordinary arithmetic, not faults.)
"""
import numpy as np
import pytest

import oracle
import sr_inputs
from gpu_helpers import make_plan, random_problem, to_dev

pytestmark = pytest.mark.gpu


def _expect(plan, nonfinite):
    import paper_2409_05734_amd as srpr
    if nonfinite:
        with pytest.raises(srpr.SrError) as ei:
            srpr.sr_plan_sync(plan)
        assert ei.value.status == srpr.SR_E_NONFINITE
    srpr.sr_plan_sync(plan)  # reported once, then clear


def _case(rng, n_shape, m_shape, L):
    th, xs = random_problem(rng, n_shape, m_shape, L)
    op = oracle.StructuredOperator(th, n_shape)
    y = oracle.measurements(xs, th).astype(np.float32)
    return th, xs, y, np.float32(oracle.default_step(op, y, 0.2))


@pytest.mark.parametrize("n_shape,m_shape,L", [((64,), (256,), 2), ((24, 20), (64, 64), 2), ((100, 90), (256, 256), 3)])
def test_single_problem_gd_and_spectral(gpu, n_shape, m_shape, L):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(3)
    th, xs, y, eta = _case(rng, n_shape, m_shape, L)
    plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
    x0 = (xs + 0.5 * sr_inputs.complex_gaussian(rng, n_shape)).ravel()  # in the basin of x*: GD converges
    yd = to_dev(y.ravel(), gpu)
    # finite solves: no flag (60 steps go past one replayed graph chunk)
    x = to_dev(x0, gpu)
    srpr.sr_gd_solve(plan, yd, x, 60, eta)
    out = torch.empty_like(x)
    srpr.sr_spectral_init(plan, yd, x, 12, -1.0, out)
    srpr.sr_spectral_init(plan, torch.zeros_like(yd), x, 3, -1.0, out)  # y = 0: estimate 0, finite
    _expect(plan, False)
    # NaN in the measurements
    ybad = y.copy().ravel()
    ybad[ybad.size // 3] = np.nan
    ybd = to_dev(ybad, gpu)
    srpr.sr_gd_solve(plan, ybd, to_dev(x0, gpu), 3, eta)
    _expect(plan, True)
    srpr.sr_spectral_init(plan, ybd, to_dev(x0, gpu), 4, -1.0, out)
    _expect(plan, True)
    # a step so large that the iterates overflow, past one graph chunk
    srpr.sr_gd_solve(plan, yd, to_dev(x0, gpu), 55, np.float32(1e20) * eta)
    _expect(plan, True)
    # with a loss trace
    lt = torch.zeros(4, dtype=torch.float32, device=gpu)
    srpr.sr_gd_solve(plan, yd, to_dev(x0, gpu), 4, np.float32(1e25) * eta, lt)
    _expect(plan, True)
    # and clean again afterwards
    srpr.sr_gd_solve(plan, yd, to_dev(x0, gpu), 5, eta)
    _expect(plan, False)


def test_stacked_and_batched_schedules(gpu, monkeypatch):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(4)
    # a stack of 3 problems of one shape, own masks
    n_shape, m_shape, L = (30, 30), (64, 64), 2
    cases = [_case(rng, n_shape, m_shape, L) for _ in range(3)]
    plan = make_plan([(n_shape, m_shape, L)] * 3, [c[0] for c in cases], gpu)
    y = np.concatenate([c[2].ravel() for c in cases])
    etas = np.array([c[3] for c in cases], np.float32)
    x0 = np.concatenate([(c[1] + 0.5 * sr_inputs.complex_gaussian(rng, n_shape)).ravel() for c in cases])
    srpr.sr_gd_solve(plan, to_dev(y, gpu), to_dev(x0, gpu), 7, etas)
    _expect(plan, False)
    y[2 * 4096 + 17] = np.inf
    srpr.sr_gd_solve(plan, to_dev(y, gpu), to_dev(x0, gpu), 7, etas)
    _expect(plan, True)
    # uneven problems by level launches, GD and power iteration (with the
    # LDS-resident solver for the small ones)
    specs = [((20, 20), (32, 64), 1), ((32, 30), (64, 64), 2), ((40, 36), (96, 64), 3), ((16,), (64,), 2)]
    cs = [_case(rng, *s) for s in specs]
    plan = make_plan(specs, [c[0] for c in cs], gpu)
    srpr.sr_plan_set_schedule(plan, srpr.SR_SCHED_BATCHED)
    y = np.concatenate([c[2].ravel() for c in cs])
    etas = np.array([c[3] for c in cs], np.float32)
    x0 = np.concatenate([(c[1] + 0.5 * sr_inputs.complex_gaussian(rng, s[0])).ravel() for c, s in zip(cs, specs)])
    out = torch.empty(plan.n_total, dtype=torch.complex64, device=gpu)
    srpr.sr_gd_solve(plan, to_dev(y, gpu), to_dev(x0, gpu), 9, etas)
    srpr.sr_spectral_init(plan, to_dev(y, gpu), to_dev(x0, gpu), 9, -1.0, out)
    _expect(plan, False)
    for i in range(len(specs)):  # NaN in one problem at a time
        yb = y.copy()
        yb[plan.y_off[i] + 5] = np.nan
        srpr.sr_gd_solve(plan, to_dev(yb, gpu), to_dev(x0, gpu), 9, etas)
        _expect(plan, True)
        srpr.sr_spectral_init(plan, to_dev(yb, gpu), to_dev(x0, gpu), 9, -1.0, out)
        _expect(plan, True)
    monkeypatch.setenv("SR_LDS_RESIDENT", "1")
    yb = y.copy()
    yb[plan.y_off[0] + 1] = np.nan
    srpr.sr_gd_solve(plan, to_dev(yb, gpu), to_dev(x0, gpu), 9, etas)
    _expect(plan, True)


def test_dense_model(gpu):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(5)
    m, n = 256, 64
    A = sr_inputs.complex_gaussian(rng, (m, n))
    xs = sr_inputs.complex_gaussian(rng, (n,))
    y = (np.abs(A.astype(np.complex128) @ xs) ** 2).astype(np.float32)
    Ad = to_dev(A, gpu)
    plan = srpr.Plan([srpr.Problem((n,), (m,), kind=srpr.SR_DENSE)], dense_A=Ad)
    x0 = xs + 0.5 * sr_inputs.complex_gaussian(rng, (n,))
    eta = np.float32(0.2 / np.mean(y))
    out = torch.empty(n, dtype=torch.complex64, device=gpu)
    srpr.sr_gd_solve(plan, to_dev(y, gpu), to_dev(x0, gpu), 10, eta)
    srpr.sr_spectral_init(plan, to_dev(y, gpu), to_dev(x0, gpu), 10, -1.0, out)
    _expect(plan, False)
    yb = y.copy()
    yb[7] = np.nan
    srpr.sr_gd_solve(plan, to_dev(yb, gpu), to_dev(x0, gpu), 10, eta)
    _expect(plan, True)
    srpr.sr_spectral_init(plan, to_dev(yb, gpu), to_dev(x0, gpu), 10, -1.0, out)
    _expect(plan, True)
    srpr.sr_gd_solve(plan, to_dev(y, gpu), to_dev(x0, gpu), 10, np.float32(1e25) * eta)
    _expect(plan, True)
