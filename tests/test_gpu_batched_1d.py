"""Many 1D problems in one plan: the LDS-resident 1D kernels run one
workgroup per problem, one launch per grid length.  Operator, GD and spectral
results of every problem against the FP64 oracle (mixed lengths, padded and
trimmed problems, L = 1..3)."""
import numpy as np
import pytest

import oracle
import sr_inputs
from gpu_helpers import aligned, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


def _specs(rng, count):
    out = []
    for _ in range(count):
        grid = int(rng.choice([64, 128, 256, 512]))
        L = int(rng.integers(1, 4))
        if rng.uniform() < 0.7:
            n = int(rng.integers(grid // 8, grid // 2))   # padded, alpha in (2, 8)
            out.append(((n,), (grid,), L))
        else:
            m = int(rng.integers(grid // 2, grid))        # trimmed, alpha < 1
            out.append(((grid,), (m,), L))
    return out


def _setup(count, seed):
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(seed)
    specs = _specs(rng, count)
    data = []
    for n_shape, m_shape, L in specs:
        grid = (max(n_shape[0], m_shape[0]),)
        th = rng.uniform(0, 2 * np.pi, (L,) + grid).astype(np.float32)
        xs = sr_inputs.complex_gaussian(rng, n_shape)
        op = oracle.StructuredOperator(th, n_shape, m_shape)
        data.append(dict(th=th, xs=xs, op=op, n_shape=n_shape, m_shape=m_shape))
    plan = srpr.Plan([srpr.Problem(n, m, L) for n, m, L in specs], np.concatenate([d["th"].ravel() for d in data]))
    return plan, data, rng


def test_batched_1d_operator(gpu):
    import torch
    import paper_2409_05734_amd as srpr
    plan, data, rng = _setup(48, 3)
    x = np.concatenate([d["xs"].ravel() for d in data])
    r = np.concatenate([sr_inputs.complex_gaussian(rng, d["m_shape"]).ravel() for d in data])
    z = torch.empty(plan.m_total, dtype=torch.complex64, device=gpu)
    v = torch.empty(plan.n_total, dtype=torch.complex64, device=gpu)
    srpr.sr_forward(plan, to_dev(x, gpu), z, None)
    srpr.sr_adjoint(plan, to_dev(r, gpu), v)
    srpr.sr_plan_sync(plan)
    zh, vh = to_host(z), to_host(v)
    for i, d in enumerate(data):
        zi = zh[plan.y_off[i]:plan.y_off[i + 1]]
        assert rel_l2(zi, d["op"].A(d["xs"]).ravel()) <= 2e-5, i
        ri = r[plan.y_off[i]:plan.y_off[i + 1]]
        assert rel_l2(vh[plan.x_off[i]:plan.x_off[i + 1]], d["op"].AH(ri).ravel()) <= 2e-5, i


def test_batched_1d_solvers(gpu):
    import torch
    import paper_2409_05734_amd as srpr
    plan, data, rng = _setup(40, 4)
    ys = [(np.abs(d["op"].A(d["xs"])) ** 2).astype(np.float32) for d in data]
    y = to_dev(np.concatenate([a.ravel() for a in ys]), gpu)
    x0s = [(d["xs"] + 0.3 * sr_inputs.complex_gaussian(rng, d["n_shape"])).astype(np.complex64) for d in data]
    etas = np.array([oracle.default_step(d["op"], yy, 0.1) for d, yy in zip(data, ys)], np.float32)
    x = to_dev(np.concatenate([a.ravel() for a in x0s]), gpu)
    srpr.sr_gd_solve(plan, y, x, 20, etas)
    v0s = [sr_inputs.complex_gaussian(rng, d["n_shape"]) for d in data]
    out = torch.empty(plan.n_total, dtype=torch.complex64, device=gpu)
    srpr.sr_spectral_init(plan, y, to_dev(np.concatenate([a.ravel() for a in v0s]), gpu), 15, -1.0, out)
    srpr.sr_plan_sync(plan)
    xh, oh = to_host(x), to_host(out)
    for i, d in enumerate(data):
        xr = oracle.gd_solve(d["op"], ys[i], x0s[i], 20, float(etas[i]))
        assert aligned(xh[plan.x_off[i]:plan.x_off[i + 1]], xr.ravel()) <= 1e-4, i
        sr = oracle.spectral_init(d["op"], ys[i], v0s[i], 15, -1.0)
        assert rel_l2(oh[plan.x_off[i]:plan.x_off[i + 1]], sr.ravel()) <= 1e-4, i
