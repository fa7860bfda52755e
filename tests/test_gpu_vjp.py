"""GPU parity of the reverse-mode kernels (phase and signal cotangents through
A and A^H) against the FP64 oracle, and of the autograd Functions on the
mask-design objective (unrolled GD) against the oracle's reverse-mode
gradient, whose own correctness is pinned by central finite differences on
the CPU."""
import numpy as np
import pytest

import oracle
import sr_inputs
from gpu_helpers import make_plan, random_problem, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_VJP = 1e-4

SHAPES = [((64,), (256,), 2), ((40,), (96,), 3), ((30,), (64,), 1), ((16, 16), (32, 32), 2), ((20, 12), (32, 64), 1),
          ((48, 40), (96, 64), 3), ((100, 70), (192, 128), 2), ((128, 128), (256, 256), 2)]


@pytest.mark.parametrize("n_shape,m_shape,L", SHAPES)
def test_vjp_parity(gpu, n_shape, m_shape, L):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(60 + L + len(n_shape))
    th, x = random_problem(rng, n_shape, m_shape, L)
    gz = sr_inputs.complex_gaussian(rng, m_shape)
    r = sr_inputs.complex_gaussian(rng, m_shape)
    gv = sr_inputs.complex_gaussian(rng, n_shape)
    plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
    n, m = int(np.prod(n_shape)), int(np.prod(m_shape))
    gx = torch.empty(n, dtype=torch.complex64, device=gpu)
    gth = torch.zeros(L * m, dtype=torch.float32, device=gpu)
    srpr.sr_forward_vjp(plan, to_dev(x.ravel(), gpu), to_dev(gz.ravel(), gpu), gx, gth)
    gr = torch.empty(m, dtype=torch.complex64, device=gpu)
    gth2 = torch.full((L * m,), 0.25, dtype=torch.float32, device=gpu)  # accumulates onto existing values
    srpr.sr_adjoint_vjp(plan, to_dev(r.ravel(), gpu), to_dev(gv.ravel(), gpu), gr, gth2)
    torch.cuda.synchronize()
    gx_o, gth_o = oracle.forward_vjp(x, th, gz)
    gr_o, gth2_o = oracle.adjoint_vjp(r, th, n_shape, gv)
    assert rel_l2(to_host(gx).reshape(n_shape), gx_o) <= TOL_VJP
    assert rel_l2(to_host(gth).reshape(gth_o.shape), gth_o) <= TOL_VJP
    assert rel_l2(to_host(gr).reshape(m_shape), gr_o) <= TOL_VJP
    d2 = to_host(gth2).reshape(gth2_o.shape) - 0.25
    assert rel_l2(d2, gth2_o) <= TOL_VJP
    # NULL signal cotangent outputs are allowed
    srpr.sr_forward_vjp(plan, to_dev(x.ravel(), gpu), to_dev(gz.ravel(), gpu), None, gth)
    srpr.sr_adjoint_vjp(plan, to_dev(r.ravel(), gpu), to_dev(gv.ravel(), gpu), None, gth2)
    torch.cuda.synchronize()
    assert rel_l2(to_host(gth).reshape(gth_o.shape), 2 * gth_o) <= TOL_VJP


def _mask_design_case(B, n_side, L, T, seed):
    s = sr_inputs.streams(seed)
    n_shape, m_shape = (n_side, n_side), (2 * n_side, 2 * n_side)
    th = sr_inputs.phase_masks(s["theta"], L, m_shape)
    xs = sr_inputs.complex_gaussian(s["signal"], (B,) + n_shape)
    x0 = np.stack([sr_inputs.scaled_start(s["x0"], n_shape, float(np.vdot(xs[b].astype(np.complex128),
                                                                          xs[b].astype(np.complex128)).real))
                   for b in range(B)])
    return n_shape, m_shape, th, xs, x0


def _gpu_loss_grad(gpu, n_shape, m_shape, th, xs, x0, T, mu):
    import torch
    import paper_2409_05734_amd as srpr
    from paper_2409_05734_amd.autograd import unrolled_gd_loss
    B, L = xs.shape[0], th.shape[0]
    probs = [srpr.Problem(n_shape, m_shape, L, theta_offset=0) for _ in range(B)]
    plan = srpr.Plan(probs, th)
    theta = to_dev(th.ravel(), gpu).requires_grad_(True)
    loss = unrolled_gd_loss(plan, theta, to_dev(xs.reshape(B, -1), gpu), to_dev(x0.reshape(B, -1), gpu), T, mu)
    loss.backward()
    torch.cuda.synchronize()
    return float(loss.item()), to_host(theta.grad).reshape(th.shape)


def test_autograd_mask_gradient_small(gpu):
    n_shape, m_shape, th, xs, x0 = _mask_design_case(3, 16, 2, 3, seed=70)
    loss, g = _gpu_loss_grad(gpu, n_shape, m_shape, th, xs, x0, 3, 0.2)
    loss_o, g_o = oracle.unrolled_gd_loss_grad(th, xs, x0, 3, 0.2)
    assert abs(loss - loss_o) / abs(loss_o) < 1e-4
    assert rel_l2(g, g_o) < 1e-3
    # invariants the exact gradient satisfies
    assert np.abs(g.reshape(2, -1).sum(axis=1)).max() < 1e-3 * np.abs(g).sum()


def test_autograd_mask_gradient_full_size_subset(gpu):
    """The mask-design workload's shapes (128^2 -> 256^2, L = 2, 20 unrolled
    steps) on 2 of its 64 problems; the full batch's gradient is the mean of
    such per-problem terms."""
    d = sr_inputs.mask_design(3)
    th, xs, x0 = d["theta"], d["x_star"][:2], d["x0"][:2]
    loss, g = _gpu_loss_grad(gpu, d["n_shape"], d["m_shape"], th, xs, x0, d["steps"], d["mu"])
    loss_o, g_o = oracle.unrolled_gd_loss_grad(th, xs, x0, d["steps"], d["mu"])
    assert abs(loss - loss_o) / abs(loss_o) < 1e-4
    assert rel_l2(g, g_o) < 1e-3


def test_autograd_mask_gradient_against_central_differences(gpu):
    """The GPU mask gradient on the mask-design workload's shapes (first 2
    problems, 128^2 -> 256^2, L = 2, 20 unrolled steps) projected on 32
    seeded directions, against the stored FP64 central differences of the
    oracle's objective (eps = 1e-6).  Bars: loss 1e-4; the 32 directional
    derivatives 1e-3 in relative L2 (the gradient's bar: fp32 through 20
    unrolled steps and two derivative passes per step)."""
    from fixtures import read_mask_fd
    d, loss_fd, fd, dirs = read_mask_fd()
    th, xs, x0 = d["theta"], d["x_star"][:2], d["x0"][:2]
    loss, g = _gpu_loss_grad(gpu, d["n_shape"], d["m_shape"], th, xs, x0, d["steps"], d["mu"])
    assert abs(loss - loss_fd) / abs(loss_fd) < 1e-4
    dd = (dirs * g.astype(np.float64)[None]).reshape(len(fd), -1).sum(axis=1)
    assert rel_l2(dd, fd) < 1e-3


@pytest.mark.parametrize("n_shape,m_shape,L,B,shared", [((20, 12), (32, 64), 2, 1, False),
                                                        ((24, 24), (64, 64), 3, 3, True),
                                                        ((30, 20), (64, 32), 1, 2, False)])
def test_gd_step_and_intensity_vjp_against_finite_differences(gpu, n_shape, m_shape, L, B, shared):
    """sr_gd_step_vjp (reverse of one GD step of Eq. (2)) and sr_intensity_vjp
    (reverse of y = |A x|^2, Eq. (1)) against FP64 central differences of the
    oracle's step x - eta g(x) and of its intensities, in 6 seeded directions
    for x, y and theta each (single problems and several problems, with
    shared or separate masks)."""
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(B * 10 + L)
    n = int(np.prod(n_shape))
    m = int(np.prod(m_shape))
    ths = [sr_inputs.phase_masks(rng, L, m_shape) for _ in range(1 if shared else B)]
    probs = [srpr.Problem(n_shape, m_shape, L, theta_offset=0 if shared else b * L * m) for b in range(B)]
    plan = srpr.Plan(probs, np.concatenate([t.ravel() for t in ths]))
    th_of = (lambda b: ths[0]) if shared else (lambda b: ths[b])
    xs = [sr_inputs.complex_gaussian(rng, n_shape) for _ in range(B)]
    x = [(xs[b] + 0.5 * sr_inputs.complex_gaussian(rng, n_shape)).astype(np.complex64) for b in range(B)]
    y = [oracle.measurements(xs[b], th_of(b)).astype(np.float32) for b in range(B)]
    eta = np.array([oracle.default_step(oracle.StructuredOperator(th_of(b), n_shape), y[b], 0.2) for b in range(B)],
                   np.float32)
    gxn = [sr_inputs.complex_gaussian(rng, n_shape) for _ in range(B)]
    gyv = [rng.standard_normal(m_shape).astype(np.float32) for _ in range(B)]
    cat = lambda a: np.concatenate([v.ravel() for v in a])
    theta = to_dev(np.concatenate([t.ravel() for t in ths]), gpu)
    gx = torch.empty(B * n, dtype=torch.complex64, device=gpu)
    gy = torch.zeros(B * m, dtype=torch.float32, device=gpu)
    gth = torch.zeros_like(theta)
    srpr.sr_gd_step_vjp(plan, to_dev(cat(y), gpu), to_dev(cat(x), gpu), eta, to_dev(cat(gxn), gpu), gx, gy, gth)
    gx2 = torch.empty(B * n, dtype=torch.complex64, device=gpu)
    gth2 = torch.zeros_like(theta)
    srpr.sr_intensity_vjp(plan, to_dev(cat(x), gpu), to_dev(cat(gyv), gpu), gx2, gth2)
    torch.cuda.synchronize()
    gx, gy, gth = to_host(gx).reshape(B, *n_shape), to_host(gy).reshape(B, *m_shape), to_host(gth)
    gx2, gth2 = to_host(gx2).reshape(B, *n_shape), to_host(gth2)

    def thetas(th_flat):
        if shared:
            return [th_flat.reshape(L, *m_shape)] * B
        return [th_flat[b * L * m:(b + 1) * L * m].reshape(L, *m_shape) for b in range(B)]

    def f_step(xx, yy, th_flat):
        t = thetas(th_flat)
        tot = 0.0
        for b in range(B):
            op = oracle.StructuredOperator(t[b], n_shape)
            xp = xx[b] - float(eta[b]) * oracle.gd_gradient(op, yy[b], xx[b])
            tot += np.vdot(gxn[b], xp).real
        return tot

    def f_int(xx, th_flat):
        t = thetas(th_flat)
        return sum(float(np.sum(gyv[b] * oracle.measurements(xx[b], t[b]))) for b in range(B))

    x64 = [v.astype(np.complex128) for v in x]
    y64 = [v.astype(np.float64) for v in y]
    t64 = np.concatenate([t.ravel() for t in ths]).astype(np.float64)
    eps = 1e-6
    got, want = [], []
    for k in range(6):
        dx = [sr_inputs.complex_gaussian(rng, n_shape).astype(np.complex128) for _ in range(B)]
        dy = [rng.standard_normal(m_shape) for _ in range(B)]
        dt = rng.standard_normal(t64.shape)
        xp = [a + eps * d for a, d in zip(x64, dx)]
        xm = [a - eps * d for a, d in zip(x64, dx)]
        want.append((f_step(xp, y64, t64) - f_step(xm, y64, t64)) / (2 * eps))
        got.append(sum(np.vdot(gx[b].astype(np.complex128), dx[b]).real for b in range(B)))
        yp = [a + eps * d for a, d in zip(y64, dy)]
        ym = [a - eps * d for a, d in zip(y64, dy)]
        want.append((f_step(x64, yp, t64) - f_step(x64, ym, t64)) / (2 * eps))
        got.append(sum(float(np.sum(gy[b] * dy[b])) for b in range(B)))
        want.append((f_step(x64, y64, t64 + eps * dt) - f_step(x64, y64, t64 - eps * dt)) / (2 * eps))
        got.append(float(np.sum(gth * dt)))
        want.append((f_int(xp, t64) - f_int(xm, t64)) / (2 * eps))
        got.append(sum(np.vdot(gx2[b].astype(np.complex128), dx[b]).real for b in range(B)))
        want.append((f_int(x64, t64 + eps * dt) - f_int(x64, t64 - eps * dt)) / (2 * eps))
        got.append(float(np.sum(gth2 * dt)))
    got, want = np.array(got).reshape(6, 5), np.array(want).reshape(6, 5)
    for j in range(5):  # each derivative on its own scale
        assert np.linalg.norm(got[:, j] - want[:, j]) <= 1e-4 * np.linalg.norm(want[:, j]), (j, got[:, j], want[:, j])
