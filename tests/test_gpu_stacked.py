"""Stacked execution of uniform multi-problem plans (problems of one 2D
geometry whose phase blocks are shared or evenly spaced run every fused pass
as one launch): A, A^H and both reverse-mode derivatives agree bit for bit
with the problem-by-problem loop (same kernels, same tiles, the shared-phase
cotangents added in problem order), and with the FP64 oracle (section III,
Eq. (5))."""
import numpy as np
import pytest

import oracle
import sr_inputs
from gpu_helpers import rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


def _grid(n_shape, m_shape):
    return tuple(max(a, b) for a, b in zip(n_shape, m_shape))


CASES = [
    # (n_shape, m_shape, L, problems, shared phases)
    ((24, 24), (64, 64), 2, 5, True),
    ((48, 40), (96, 64), 3, 3, False),
    ((64, 64), (40, 50), 2, 4, True),     # trimmed measurement window
    ((100, 70), (192, 128), 1, 6, False),
    ((128, 128), (256, 256), 2, 9, True),
]


def _plan(n_shape, m_shape, L, P, shared, th_blocks, schedule):
    import paper_2409_05734_amd as srpr
    block = th_blocks[0].size
    probs = [srpr.Problem(n_shape, m_shape, L, theta_offset=0 if shared else i * block) for i in range(P)]
    plan = srpr.Plan(probs, np.concatenate([t.ravel() for t in th_blocks]))
    srpr.sr_plan_set_schedule(plan, schedule)
    return plan


def _run_all(plan, x, r, gz, gv, n_th, dev):
    import torch
    import paper_2409_05734_amd as srpr
    z = torch.empty(plan.m_total, dtype=torch.complex64, device=dev)
    y = torch.empty(plan.m_total, dtype=torch.float32, device=dev)
    v = torch.empty(plan.n_total, dtype=torch.complex64, device=dev)
    srpr.sr_forward(plan, x, z, y)
    srpr.sr_adjoint(plan, r, v)
    gx = torch.empty(plan.n_total, dtype=torch.complex64, device=dev)
    gr = torch.empty(plan.m_total, dtype=torch.complex64, device=dev)
    g1 = torch.full((n_th,), 0.25, dtype=torch.float32, device=dev)  # accumulates onto existing values
    g2 = torch.full((n_th,), -0.5, dtype=torch.float32, device=dev)
    srpr.sr_forward_vjp(plan, x, gz, gx, g1)
    srpr.sr_adjoint_vjp(plan, r, gv, gr, g2)
    srpr.sr_plan_sync(plan)
    return [t.clone() for t in (z, y, v, gx, gr, g1, g2)]


@pytest.mark.parametrize("n_shape,m_shape,L,P,shared", CASES)
def test_stacked_matches_loop_and_oracle(gpu, n_shape, m_shape, L, P, shared):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(hash((n_shape, m_shape, L, P)) % 2**32)
    g = _grid(n_shape, m_shape)
    nblk = 1 if shared else P
    th_blocks = [rng.uniform(0, 2 * np.pi, (L,) + g).astype(np.float32) for _ in range(nblk)]
    n, m = int(np.prod(n_shape)), int(np.prod(m_shape))
    x = to_dev(np.concatenate([sr_inputs.complex_gaussian(rng, n_shape).ravel() for _ in range(P)]), gpu)
    r = to_dev(np.concatenate([sr_inputs.complex_gaussian(rng, m_shape).ravel() for _ in range(P)]), gpu)
    gz = to_dev(np.concatenate([sr_inputs.complex_gaussian(rng, m_shape).ravel() for _ in range(P)]), gpu)
    gv = to_dev(np.concatenate([sr_inputs.complex_gaussian(rng, n_shape).ravel() for _ in range(P)]), gpu)
    n_th = nblk * th_blocks[0].size
    stacked = _run_all(_plan(n_shape, m_shape, L, P, shared, th_blocks, srpr.SR_SCHED_AUTO), x, r, gz, gv, n_th, gpu)
    looped = _run_all(_plan(n_shape, m_shape, L, P, shared, th_blocks, srpr.SR_SCHED_LOOP), x, r, gz, gv, n_th, gpu)
    for name, a, b in zip(("z", "y", "v", "gx", "gr", "gth_fwd", "gth_adj"), stacked, looped):
        assert torch.equal(a, b), name
    # the oracle: operator outputs of the first and the last problem, and the
    # phase cotangents summed over the problems (onto the initial values)
    z, y, v, gx, gr, g1, g2 = [to_host(t) for t in stacked]
    xh, rh, gzh, gvh = to_host(x), to_host(r), to_host(gz), to_host(gv)
    blk = th_blocks[0].size
    gt1 = np.zeros(n_th)
    gt2 = np.zeros(n_th)
    for i in range(P):
        th = th_blocks[0 if shared else i]
        xi = xh[i * n:(i + 1) * n].reshape(n_shape)
        ri = rh[i * m:(i + 1) * m].reshape(m_shape)
        if i in (0, P - 1):
            assert rel_l2(z[i * m:(i + 1) * m].reshape(m_shape), oracle.forward(xi, th, m_shape)) <= 2e-5
            assert rel_l2(v[i * n:(i + 1) * n].reshape(n_shape), oracle.adjoint(ri, th, n_shape)) <= 2e-5
        gxr, t1 = oracle.forward_vjp(xi, th, gzh[i * m:(i + 1) * m].reshape(m_shape))
        grr, t2 = oracle.adjoint_vjp(ri, th, n_shape, gvh[i * n:(i + 1) * n].reshape(n_shape), m_shape)
        if i in (0, P - 1):
            assert rel_l2(gx[i * n:(i + 1) * n].reshape(n_shape), gxr) <= 1e-4
            assert rel_l2(gr[i * m:(i + 1) * m].reshape(m_shape), grr) <= 1e-4
        o = 0 if shared else i * blk
        gt1[o:o + blk] += np.asarray(t1).ravel()
        gt2[o:o + blk] += np.asarray(t2).ravel()
    assert rel_l2(g1 - 0.25, gt1) <= 1e-4
    assert rel_l2(g2 + 0.5, gt2) <= 1e-4
