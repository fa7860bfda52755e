"""GPU parity of the structured operator with undersampling (Eq. (5),
alpha <= 1: A = S prod(F D_i), the transforms on the signal grid, S the
centred trimming) and with mixed padding/trimming across axes, against the
FP64 oracle: A and A^H (2e-5 per application), GD iterates and spectral
iterates (1e-4), the derivative kernels, and the batched schedule."""
import numpy as np
import pytest

import oracle
import sr_inputs
from gpu_helpers import aligned, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_OP = 2e-5
TOL_IT = 1e-4

SHAPES = [
    ((64,), (40,), 2),            # 1D trim
    ((256,), (256,), 1),          # alpha = 1
    ((1024,), (700,), 2),
    ((64, 64), (40, 50), 2),      # 2D trim on both axes
    ((128, 96), (100, 96), 3),    # trim axis 0 only
    ((96, 128), (128, 90), 2),    # pad axis 0, trim axis 1
    ((512, 512), (300, 400), 2),
    ((64, 2048), (48, 1500), 1),  # longest row transform, trimmed
]


def _grid(n_shape, m_shape):
    return tuple(max(a, b) for a, b in zip(n_shape, m_shape))


def _problem(rng, n_shape, m_shape, L):
    th = rng.uniform(0, 2 * np.pi, (L,) + _grid(n_shape, m_shape)).astype(np.float32)
    x = sr_inputs.complex_gaussian(rng, n_shape)
    return th, x


def _plan(specs, thetas):
    import paper_2409_05734_amd as srpr
    probs = [srpr.Problem(tuple(n), tuple(m), L) for n, m, L in specs]
    return srpr.Plan(probs, np.concatenate([t.ravel() for t in thetas]))


@pytest.mark.parametrize("n_shape,m_shape,L", SHAPES)
def test_undersampled_forward_adjoint(gpu, n_shape, m_shape, L):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(hash((n_shape, m_shape, L)) % 2**32)
    th, x = _problem(rng, n_shape, m_shape, L)
    r = sr_inputs.complex_gaussian(rng, m_shape)
    plan = _plan([(n_shape, m_shape, L)], [th])
    m, n = int(np.prod(m_shape)), int(np.prod(n_shape))
    z = torch.empty(m, dtype=torch.complex64, device=gpu)
    y = torch.empty(m, dtype=torch.float32, device=gpu)
    v = torch.empty(n, dtype=torch.complex64, device=gpu)
    srpr.sr_forward(plan, to_dev(x.ravel(), gpu), z, y)
    srpr.sr_adjoint(plan, to_dev(r.ravel(), gpu), v)
    torch.cuda.synchronize()
    z_ref = oracle.forward(x, th, m_shape)
    assert rel_l2(to_host(z).reshape(m_shape), z_ref) <= TOL_OP
    y_ref = np.abs(z_ref) ** 2
    assert rel_l2(to_host(y).reshape(m_shape), y_ref) <= 2 * TOL_OP
    assert rel_l2(to_host(v).reshape(n_shape), oracle.adjoint(r, th, n_shape)) <= TOL_OP


@pytest.mark.parametrize("n_shape,m_shape,L", [((64,), (56,), 2), ((64, 64), (64, 48), 2),
                                               ((96, 128), (128, 90), 2), ((128, 128), (112, 128), 3)])
def test_undersampled_gd_iterates(gpu, n_shape, m_shape, L):
    rng = np.random.default_rng(41 + L)
    th, xs = _problem(rng, n_shape, m_shape, L)
    op = oracle.StructuredOperator(th, n_shape, m_shape)
    y = (np.abs(op.A(xs)) ** 2).astype(np.float32)
    x0 = (xs + 0.3 * sr_inputs.complex_gaussian(rng, n_shape)).astype(np.complex64)
    eta = np.float32(oracle.default_step(op, y, 0.1))
    plan = _plan([(n_shape, m_shape, L)], [th])
    import paper_2409_05734_amd as srpr
    for k in (1, 7, 30):
        xd = to_dev(x0.ravel(), gpu)
        srpr.sr_gd_solve(plan, to_dev(y.ravel(), gpu), xd, k, eta)
        srpr.sr_plan_sync(plan)
        xr = oracle.gd_solve(op, y, x0, k, float(eta))
        assert aligned(to_host(xd).reshape(n_shape), xr) <= TOL_IT, k


@pytest.mark.parametrize("n_shape,m_shape,L", [((64,), (48,), 2), ((64, 64), (48, 56), 2), ((96, 128), (128, 90), 2)])
def test_undersampled_spectral(gpu, n_shape, m_shape, L):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(51 + L)
    th, xs = _problem(rng, n_shape, m_shape, L)
    op = oracle.StructuredOperator(th, n_shape, m_shape)
    y = (np.abs(op.A(xs)) ** 2).astype(np.float32)
    v0 = sr_inputs.complex_gaussian(rng, n_shape)
    plan = _plan([(n_shape, m_shape, L)], [th])
    for k in (1, 10, 40):
        out = torch.empty(int(np.prod(n_shape)), dtype=torch.complex64, device=gpu)
        srpr.sr_spectral_init(plan, to_dev(y.ravel(), gpu), to_dev(v0.ravel(), gpu), k, -1.0, out)
        srpr.sr_plan_sync(plan)
        xr = oracle.spectral_init(op, y, v0, k, -1.0)
        assert rel_l2(to_host(out).reshape(n_shape), xr) <= TOL_IT, k


@pytest.mark.parametrize("n_shape,m_shape,L", [((64,), (40,), 2), ((64, 64), (40, 50), 2), ((96, 128), (128, 90), 3)])
def test_undersampled_vjp(gpu, n_shape, m_shape, L):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(61 + L)
    th, x = _problem(rng, n_shape, m_shape, L)
    gz = sr_inputs.complex_gaussian(rng, m_shape)
    r = sr_inputs.complex_gaussian(rng, m_shape)
    gv = sr_inputs.complex_gaussian(rng, n_shape)
    plan = _plan([(n_shape, m_shape, L)], [th])
    n, m = int(np.prod(n_shape)), int(np.prod(m_shape))
    gx = torch.empty(n, dtype=torch.complex64, device=gpu)
    gth = torch.zeros(th.size, dtype=torch.float32, device=gpu)
    srpr.sr_forward_vjp(plan, to_dev(x.ravel(), gpu), to_dev(gz.ravel(), gpu), gx, gth)
    gr = torch.empty(m, dtype=torch.complex64, device=gpu)
    gth2 = torch.zeros(th.size, dtype=torch.float32, device=gpu)
    srpr.sr_adjoint_vjp(plan, to_dev(r.ravel(), gpu), to_dev(gv.ravel(), gpu), gr, gth2)
    torch.cuda.synchronize()
    gx_o, gth_o = oracle.forward_vjp(x, th, gz)
    gr_o, gth2_o = oracle.adjoint_vjp(r, th, n_shape, gv, m_shape)
    assert rel_l2(to_host(gx).reshape(n_shape), gx_o) <= 1e-4
    assert rel_l2(to_host(gth).reshape(gth_o.shape), gth_o) <= 1e-4
    assert rel_l2(to_host(gr).reshape(m_shape), gr_o) <= 1e-4
    assert rel_l2(to_host(gth2).reshape(gth2_o.shape), gth2_o) <= 1e-4


def test_undersampled_batched_matches_loop(gpu):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(71)
    specs = [((64, 64), (64, 48), 2), ((96, 128), (128, 90), 2), ((128, 64), (96, 64), 1), ((64, 64), (128, 128), 2)]
    data = [_problem(rng, *s) for s in specs]
    plan = _plan(specs, [d[0] for d in data])
    xs = np.concatenate([d[1].ravel() for d in data])
    y = torch.empty(plan.m_total, dtype=torch.float32, device=gpu)
    srpr.sr_forward(plan, to_dev(xs, gpu), None, y)
    x0 = (xs + 0.3 * sr_inputs.complex_gaussian(rng, xs.shape)).astype(np.complex64)
    yh = to_host(y)
    eta = np.array([0.1 * int(np.prod(_grid(n, m))) / float(np.mean(yh[plan.y_off[i]:plan.y_off[i + 1]]))
                    for i, (n, m, L) in enumerate(specs)], np.float32)
    outs = []
    for sched in (srpr.SR_SCHED_BATCHED, srpr.SR_SCHED_LOOP):
        srpr.sr_plan_set_schedule(plan, sched)
        x = to_dev(x0, gpu)
        srpr.sr_gd_solve(plan, y, x, 20, eta)
        srpr.sr_plan_sync(plan)
        outs.append(to_host(x))
    for i in range(len(specs)):
        sl = slice(plan.x_off[i], plan.x_off[i + 1])
        assert np.linalg.norm(outs[0][sl] - outs[1][sl]) <= 1e-5 * np.linalg.norm(outs[1][sl]), i
