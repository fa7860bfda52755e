"""Degenerate cases of the method on the GPU, against the FP64 oracle or
exact values: phase masks that collapse the diagonals to +-I (theta = 0 or
pi, section III), the zero signal (a fixed point of both GD losses), all-zero
measurements (the spectral estimate is exactly zero, Eq. (3)-(4) with
T = lambda), no oversampling (alpha = 1 in 2D) and the smallest grids with a
one-point signal."""
import numpy as np
import pytest

import oracle
import sr_inputs
from gpu_helpers import aligned, make_plan, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_OP = 2e-5
TOL_IT = 1e-4


def _apply(plan, x, r, m, n, dev):
    import torch
    import paper_2409_05734_amd as srpr
    z = torch.empty(m, dtype=torch.complex64, device=dev)
    v = torch.empty(n, dtype=torch.complex64, device=dev)
    srpr.sr_forward(plan, to_dev(x.ravel(), dev), z, None)
    srpr.sr_adjoint(plan, to_dev(r.ravel(), dev), v)
    srpr.sr_plan_sync(plan)
    return to_host(z), to_host(v)


@pytest.mark.parametrize("value", [0.0, np.pi])
@pytest.mark.parametrize("n_shape,m_shape,L", [((16, 16), (32, 32), 2), ((48, 40), (96, 64), 3), ((64,), (256,), 2)])
def test_constant_phase_masks(gpu, value, n_shape, m_shape, L):
    """theta = 0 (D = I: A is a cascade of plain DFTs of the padded signal)
    and theta = pi (D = -I): operator and GD parity."""
    rng = np.random.default_rng(81)
    th = np.full((L,) + m_shape, value, np.float32)
    x = sr_inputs.complex_gaussian(rng, n_shape)
    r = sr_inputs.complex_gaussian(rng, m_shape)
    plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
    z, v = _apply(plan, x, r, int(np.prod(m_shape)), int(np.prod(n_shape)), gpu)
    assert rel_l2(z.reshape(m_shape), oracle.forward(x, th)) <= TOL_OP
    assert rel_l2(v.reshape(n_shape), oracle.adjoint(r, th, n_shape)) <= TOL_OP
    import torch
    import paper_2409_05734_amd as srpr
    op = oracle.StructuredOperator(th, n_shape)
    xs = sr_inputs.complex_gaussian(rng, n_shape)
    y = (np.abs(op.A(xs)) ** 2).astype(np.float32)
    x0 = (xs + 0.5 * sr_inputs.complex_gaussian(rng, n_shape)).astype(np.complex64)
    # with constant masks and even L, A only pads and reverses: GD fits each
    # pixel's magnitude on its own, which mu = 0.2 overshoots (oracle included)
    eta = np.float32(oracle.default_step(op, y, 0.02))
    xd = to_dev(x0.ravel(), gpu)
    srpr.sr_gd_solve(plan, to_dev(y.ravel(), gpu), xd, 10, eta)
    torch.cuda.synchronize()
    assert aligned(to_host(xd).reshape(n_shape), oracle.gd_solve(op, y, x0, 10, float(eta))) <= TOL_IT


@pytest.mark.parametrize("n_shape,m_shape,L", [((24, 24), (64, 64), 2), ((64,), (256,), 2)])
def test_zero_signal_and_zero_measurements(gpu, n_shape, m_shape, L):
    """A x = 0 exactly for x = 0; x = 0 is a fixed point of GD on both losses;
    with y = 0 the spectral estimate is exactly zero (its scale sqrt(sum y /
    (m c)) vanishes, T = lambda everywhere)."""
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(82)
    th = rng.uniform(0, 2 * np.pi, (L,) + m_shape).astype(np.float32)
    n, m = int(np.prod(n_shape)), int(np.prod(m_shape))
    plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
    zero = torch.zeros(n, dtype=torch.complex64, device=gpu)
    z = torch.empty(m, dtype=torch.complex64, device=gpu)
    yz = torch.empty(m, dtype=torch.float32, device=gpu)
    srpr.sr_forward(plan, zero, z, yz)
    torch.cuda.synchronize()
    assert not torch.any(z != 0) and not torch.any(yz != 0)
    op = oracle.StructuredOperator(th, n_shape)
    y = torch.from_numpy((np.abs(op.A(sr_inputs.complex_gaussian(rng, n_shape))) ** 2).astype(np.float32)).to(gpu)
    for loss, eps in ((srpr.SR_LOSS_L2, 0.0), (srpr.SR_LOSS_POISSON, 1e-3)):
        srpr.sr_plan_set_loss(plan, loss, eps)
        x = torch.zeros(n, dtype=torch.complex64, device=gpu)
        srpr.sr_gd_solve(plan, y, x, 25, 0.1)
        torch.cuda.synchronize()
        assert not torch.any(x != 0), loss
    srpr.sr_plan_set_loss(plan, srpr.SR_LOSS_L2)
    out = torch.empty(n, dtype=torch.complex64, device=gpu)
    v0 = to_dev(sr_inputs.complex_gaussian(rng, n_shape).ravel(), gpu)
    srpr.sr_spectral_init(plan, torch.zeros(m, dtype=torch.float32, device=gpu), v0, 7, -1.0, out)
    torch.cuda.synchronize()
    assert not torch.any(out != 0)


@pytest.mark.parametrize("n_shape,m_shape,L", [((64, 64), (64, 64), 2), ((16, 16), (16, 16), 1), ((1,), (16,), 2),
                                               ((1, 1), (16, 16), 2), ((16,), (16,), 3)])
def test_alpha_one_and_smallest_grids(gpu, n_shape, m_shape, L):
    """No oversampling (alpha = 1) and the smallest grids, down to a
    one-point signal: operator, GD and spectral parity."""
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(83 + L)
    th = rng.uniform(0, 2 * np.pi, (L,) + m_shape).astype(np.float32)
    x = sr_inputs.complex_gaussian(rng, n_shape)
    r = sr_inputs.complex_gaussian(rng, m_shape)
    n, m = int(np.prod(n_shape)), int(np.prod(m_shape))
    plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
    z, v = _apply(plan, x, r, m, n, gpu)
    assert rel_l2(z.reshape(m_shape), oracle.forward(x, th)) <= TOL_OP
    assert rel_l2(v.reshape(n_shape), oracle.adjoint(r, th, n_shape)) <= TOL_OP
    op = oracle.StructuredOperator(th, n_shape)
    y = (np.abs(op.A(x)) ** 2).astype(np.float32)
    x0 = (x + 0.3 * sr_inputs.complex_gaussian(rng, n_shape)).astype(np.complex64)
    eta = np.float32(oracle.default_step(op, y, 0.1))
    xd = to_dev(x0.ravel(), gpu)
    srpr.sr_gd_solve(plan, to_dev(y.ravel(), gpu), xd, 8, eta)
    v0 = sr_inputs.complex_gaussian(rng, n_shape)
    out = torch.empty(n, dtype=torch.complex64, device=gpu)
    srpr.sr_spectral_init(plan, to_dev(y.ravel(), gpu), to_dev(v0.ravel(), gpu), 6, -1.0, out)
    torch.cuda.synchronize()
    assert aligned(to_host(xd).reshape(n_shape), oracle.gd_solve(op, y, x0, 8, float(eta))) <= TOL_IT
    assert rel_l2(to_host(out).reshape(n_shape), oracle.spectral_init(op, y, v0, 6, -1.0)) <= TOL_IT
