"""Randomised parity sweep (fixed seed): random 2D shapes (padded and
trimmed windows), L = 1..4, 1..10 problems of one shape or many, shared or
separate phases, every schedule and several forced tile sets.  A, A^H and
power iteration against the FP64 oracle on the first, last and one random
problem (2e-5 per application, 1e-4 on iterates); GD from a start near the
truth: 3 steps against the oracle's iterates (and loss trace) where the
measurements outnumber the unknowns, and, on trimmed windows (fewer
measurements than unknowns, where fp32 and fp64 trajectories drift apart),
one step from the oracle's own iterate (section III, Eq. (2)-(5))."""
import os

import numpy as np
import pytest

import oracle
import sr_inputs
from gpu_helpers import aligned, rel_l2

pytestmark = pytest.mark.gpu

LENS = [16, 32, 64, 96, 128, 192]
CASES = 40


def _pick(rng):
    M1, M2 = int(rng.choice(LENS)), int(rng.choice(LENS))
    if rng.random() < 0.2:  # the signal fills the grid, a trimmed window is measured
        return (M1, M2), (int(rng.integers(max(1, M1 // 2), M1 + 1)), int(rng.integers(max(1, M2 // 2), M2 + 1))), \
            int(rng.integers(1, 4))
    return (int(rng.integers(1, M1 + 1)), int(rng.integers(1, M2 + 1))), (M1, M2), int(rng.integers(1, 5))


@pytest.mark.parametrize("case", range(CASES))
def test_random_configuration(gpu, monkeypatch, case):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(20241203 + case)
    uniform = rng.random() < 0.5
    P = int(rng.integers(1, 11))
    base = _pick(rng)
    shapes = [base] * P if uniform else [_pick(rng) for _ in range(P)]
    shared = uniform and rng.random() < 0.4
    sched = [srpr.SR_SCHED_AUTO, srpr.SR_SCHED_LOOP, srpr.SR_SCHED_BATCHED][int(rng.integers(0, 3))]
    force = [None, "2,1,1", "4,1,0", "8,4,1", "16,1,1"][int(rng.integers(0, 5))]
    if force:
        monkeypatch.setenv("SR_TUNE_FORCE", force)
    grids = [tuple(max(a, b) for a, b in zip(n, m)) for n, m, _ in shapes]
    ths, offs, off = [], [], 0
    for i, (n, m, L) in enumerate(shapes):
        if shared and i > 0:
            ths.append(ths[0])
            offs.append(0)
            continue
        th = rng.uniform(0, 2 * np.pi, (L,) + grids[i]).astype(np.float32)
        ths.append(th)
        offs.append(off)
        off += th.size
    theta = np.concatenate([ths[i].ravel() for i in range(P) if not (shared and i > 0)])
    plan = srpr.Plan([srpr.Problem(n, m, L, theta_offset=offs[i]) for i, (n, m, L) in enumerate(shapes)], theta)
    srpr.sr_plan_set_schedule(plan, sched)
    ops = [oracle.StructuredOperator(ths[i], n, m) for i, (n, m, _) in enumerate(shapes)]
    xs = [sr_inputs.complex_gaussian(rng, n) for n, _, _ in shapes]
    ys = [(np.abs(ops[i].A(xs[i])) ** 2).astype(np.float32) for i in range(P)]
    rs = [sr_inputs.complex_gaussian(rng, m) for _, m, _ in shapes]
    v0s = [sr_inputs.complex_gaussian(rng, n) for n, _, _ in shapes]
    x0s = [(xs[i] + 0.3 * sr_inputs.complex_gaussian(rng, shapes[i][0])).astype(np.complex64) for i in range(P)]
    etas = np.array([oracle.default_step(ops[i], ys[i], 0.05) for i in range(P)], np.float32)
    cat = lambda arrs: torch.from_numpy(np.concatenate([np.asarray(a).ravel() for a in arrs])).to(gpu)  # noqa: E731
    z = torch.empty(plan.m_total, dtype=torch.complex64, device=gpu)
    v = torch.empty(plan.n_total, dtype=torch.complex64, device=gpu)
    srpr.sr_forward(plan, cat(xs), z, None)
    srpr.sr_adjoint(plan, cat(rs), v)
    kp = int(rng.choice([1, 4, 53]))
    est = torch.empty(plan.n_total, dtype=torch.complex64, device=gpu)
    yd = cat(ys)
    srpr.sr_spectral_init(plan, yd, cat(v0s), kp, -1.0, est)
    k = 3
    xg = cat(x0s)
    lt = torch.zeros(k * P, dtype=torch.float32, device=gpu)
    srpr.sr_gd_solve(plan, yd, xg, k, etas, lt)
    srpr.sr_plan_sync(plan)
    zh, vh, esth, xgh = (t.cpu().numpy() for t in (z, v, est, xg))
    lth = lt.cpu().numpy().reshape(P, k)
    for i in sorted({0, P - 1, int(rng.integers(0, P))}):
        n, m, _ = shapes[i]
        ya, yz, xa, xz = plan.y_off[i], plan.y_off[i + 1], plan.x_off[i], plan.x_off[i + 1]
        assert rel_l2(zh[ya:yz].reshape(m), ops[i].A(xs[i])) <= 2e-5, ("A", i)
        assert rel_l2(vh[xa:xz].reshape(n), ops[i].AH(rs[i])) <= 2e-5, ("A^H", i)
        assert rel_l2(esth[xa:xz].reshape(n), oracle.spectral_init(ops[i], ys[i], v0s[i], kp, -1.0)) <= 1e-4, \
            ("spectral", i, kp)
        if int(np.prod(m)) >= int(np.prod(n)):
            xr, lr = oracle.gd_solve(ops[i], ys[i], x0s[i], k, float(etas[i]), return_loss=True)
            assert aligned(xgh[xa:xz].reshape(n), xr) <= 1e-4, ("gd", i)
            assert np.max(np.abs(lth[i] - lr) / np.abs(lr)) <= 1e-4, ("loss trace", i)
    # trimmed windows: one step from the oracle's iterate after k - 1 steps
    under = [i for i in range(P) if int(np.prod(shapes[i][1])) < int(np.prod(shapes[i][0]))]
    if under:
        xk = [x0s[i] if i not in under else
              oracle.gd_solve(ops[i], ys[i], x0s[i], k - 1, float(etas[i])).astype(np.complex64) for i in range(P)]
        xs1 = cat(xk)
        srpr.sr_gd_solve(plan, yd, xs1, 1, etas)
        srpr.sr_plan_sync(plan)
        x1 = xs1.cpu().numpy()
        for i in under[:3]:
            n = shapes[i][0]
            xr = oracle.gd_solve(ops[i], ys[i], xk[i], 1, float(etas[i]))
            assert rel_l2(x1[plan.x_off[i]:plan.x_off[i + 1]].reshape(n), xr) <= 2e-5, ("gd one step", i)


@pytest.mark.parametrize("case", range(20))
def test_random_derivatives(gpu, case):
    """Both reverse-mode products on random plans (1D and 2D, padded and
    trimmed, shared or separate phases, every schedule): signal cotangents
    per problem and phase cotangents summed over the problems that share a
    block, within 1e-4 of the oracle."""
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(777 + case)
    uniform = rng.random() < 0.6
    P = int(rng.integers(1, 9))

    def pick():
        if rng.random() < 0.2:
            M = int(rng.choice([64, 128, 256, 512]))
            return (int(rng.integers(1, M + 1)),), (M,), int(rng.integers(1, 4))
        return _pick(rng)
    base = pick()
    shapes = [base] * P if uniform else [pick() for _ in range(P)]
    shared = uniform and rng.random() < 0.5
    sched = [srpr.SR_SCHED_AUTO, srpr.SR_SCHED_LOOP, srpr.SR_SCHED_BATCHED][int(rng.integers(0, 3))]
    grids = [tuple(max(a, b) for a, b in zip(n, m)) for n, m, _ in shapes]
    ths, offs, off = [], [], 0
    for i, (n, m, L) in enumerate(shapes):
        if shared and i > 0:
            ths.append(ths[0])
            offs.append(0)
            continue
        th = rng.uniform(0, 2 * np.pi, (L,) + grids[i]).astype(np.float32)
        ths.append(th)
        offs.append(off)
        off += th.size
    theta = np.concatenate([ths[i].ravel() for i in range(P) if not (shared and i > 0)])
    plan = srpr.Plan([srpr.Problem(n, m, L, theta_offset=offs[i]) for i, (n, m, L) in enumerate(shapes)], theta)
    srpr.sr_plan_set_schedule(plan, sched)
    xs = [sr_inputs.complex_gaussian(rng, n) for n, _, _ in shapes]
    gzs = [sr_inputs.complex_gaussian(rng, m) for _, m, _ in shapes]
    rs = [sr_inputs.complex_gaussian(rng, m) for _, m, _ in shapes]
    gvs = [sr_inputs.complex_gaussian(rng, n) for n, _, _ in shapes]
    cat = lambda arrs: torch.from_numpy(np.concatenate([np.asarray(a).ravel() for a in arrs])).to(gpu)  # noqa: E731
    gx = torch.empty(plan.n_total, dtype=torch.complex64, device=gpu)
    gr = torch.empty(plan.m_total, dtype=torch.complex64, device=gpu)
    g1 = torch.zeros(theta.size, dtype=torch.float32, device=gpu)
    g2 = torch.zeros(theta.size, dtype=torch.float32, device=gpu)
    srpr.sr_forward_vjp(plan, cat(xs), cat(gzs), gx, g1)
    srpr.sr_adjoint_vjp(plan, cat(rs), cat(gvs), gr, g2)
    srpr.sr_plan_sync(plan)
    gxh, grh = gx.cpu().numpy(), gr.cpu().numpy()
    t1, t2 = np.zeros(theta.size), np.zeros(theta.size)
    for i, (n, m, _) in enumerate(shapes):
        gxr, a1 = oracle.forward_vjp(xs[i], ths[i], gzs[i])
        grr, a2 = oracle.adjoint_vjp(rs[i], ths[i], n, gvs[i], m)
        t1[offs[i]:offs[i] + ths[i].size] += np.asarray(a1).ravel()
        t2[offs[i]:offs[i] + ths[i].size] += np.asarray(a2).ravel()
        assert rel_l2(gxh[plan.x_off[i]:plan.x_off[i + 1]].reshape(n), gxr) <= 1e-4, ("gx", i)
        assert rel_l2(grh[plan.y_off[i]:plan.y_off[i + 1]].reshape(m), grr) <= 1e-4, ("gr", i)
    assert rel_l2(g1.cpu().numpy(), t1) <= 1e-4
    assert rel_l2(g2.cpu().numpy(), t2) <= 1e-4
