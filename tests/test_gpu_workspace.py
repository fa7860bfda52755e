"""The plan's workspace moved into caller-owned memory (a torch tensor):
every entry point gives bitwise the same results as before the move, on a
single-problem plan, a stacked plan, a batched plan and a dense plan; the
argument checks reject short, misaligned and NULL memory."""
import numpy as np
import pytest

import oracle
import sr_inputs
from gpu_helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


def _run(plan, x, r, y, v0, eta, dev):
    import torch
    import paper_2409_05734_amd as srpr
    z = torch.empty(plan.m_total, dtype=torch.complex64, device=dev)
    v = torch.empty(plan.n_total, dtype=torch.complex64, device=dev)
    srpr.sr_forward(plan, x, z, None)
    srpr.sr_adjoint(plan, r, v)
    xg = x.clone()
    srpr.sr_gd_solve(plan, y, xg, 57, eta)  # past one replayed graph chunk
    xs = torch.empty_like(x)
    srpr.sr_spectral_init(plan, y, v0, 57, -1.0, xs)
    srpr.sr_plan_sync(plan)
    return [t.clone() for t in (z, v, xg, xs)]


@pytest.mark.parametrize("shapes,shared", [([((48, 40), (96, 64), 2)], False),
                                           ([((24, 24), (64, 64), 2)] * 4, False),
                                           ([((24, 24), (64, 64), 2), ((40, 30), (96, 64), 3), ((12, 10), (16, 32), 1),
                                             ((64, 64), (128, 64), 2), ((30, 100), (32, 256), 3), ((9, 80), (16, 96), 2),
                                             ((20, 20), (32, 32), 1), ((48, 40), (96, 64), 2)], False)])
def test_workspace_moved_into_a_tensor(gpu, shapes, shared):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(101 + len(shapes))
    ths = [rng.uniform(0, 2 * np.pi, (L,) + tuple(max(a, b) for a, b in zip(n, m))).astype(np.float32)
           for n, m, L in shapes]
    offs = np.cumsum([0] + [t.size for t in ths])
    plan = srpr.Plan([srpr.Problem(n, m, L, theta_offset=int(offs[i])) for i, (n, m, L) in enumerate(shapes)],
                     np.concatenate([t.ravel() for t in ths]))
    x = to_dev(np.concatenate([sr_inputs.complex_gaussian(rng, n).ravel() for n, _, _ in shapes]), gpu)
    r = to_dev(np.concatenate([sr_inputs.complex_gaussian(rng, m).ravel() for _, m, _ in shapes]), gpu)
    v0 = to_dev(np.concatenate([sr_inputs.complex_gaussian(rng, n).ravel() for n, _, _ in shapes]), gpu)
    y = torch.empty(plan.m_total, dtype=torch.float32, device=gpu)
    srpr.sr_forward(plan, x, None, y)
    yh = to_host(y)
    eta = np.array([0.05 * int(np.prod(m)) / float(np.mean(yh[plan.y_off[i]:plan.y_off[i + 1]]))
                    for i, (_, m, _) in enumerate(shapes)], np.float32)
    before = _run(plan, x, r, y, v0, eta, gpu)
    size = srpr.sr_plan_workspace_size(plan)
    with pytest.raises(srpr.SrError):
        srpr.sr_plan_set_workspace(plan, torch.empty(size - 256, dtype=torch.uint8, device=gpu))
    big = torch.empty(size + 512, dtype=torch.uint8, device=gpu)
    with pytest.raises(srpr.SrError):
        srpr.sr_plan_set_workspace(plan, big[4:])  # misaligned
    ws = torch.full((size,), 0xAB, dtype=torch.uint8, device=gpu)
    srpr.sr_plan_set_workspace(plan, ws)
    after = _run(plan, x, r, y, v0, eta, gpu)
    ws2 = torch.empty(size, dtype=torch.uint8, device=gpu)
    srpr.sr_plan_set_workspace(plan, ws2)  # and on again: the first tensor is the caller's
    again = _run(plan, x, r, y, v0, eta, gpu)
    for name, a, b, c in zip(("z", "v", "gd", "spectral"), before, after, again):
        assert torch.equal(a, b) and torch.equal(a, c), name
    plan.close()


def test_dense_workspace_moved(gpu):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(103)
    m, n, nb = 256, 64, 2
    A = to_dev(np.ascontiguousarray(sr_inputs.complex_gaussian(rng, (m, n))), gpu)
    plan = srpr.Plan([srpr.Problem((n,), (m,), 1, kind=srpr.SR_DENSE) for _ in range(nb)], None, dense_A=A)
    x = to_dev(sr_inputs.complex_gaussian(rng, (nb * n,)), gpu)
    r = to_dev(sr_inputs.complex_gaussian(rng, (nb * m,)), gpu)
    v0 = to_dev(sr_inputs.complex_gaussian(rng, (nb * n,)), gpu)
    y = torch.empty(nb * m, dtype=torch.float32, device=gpu)
    srpr.sr_forward(plan, x, None, y)
    eta = np.full(nb, 0.05 / float(to_host(y).mean()), np.float32)
    before = _run(plan, x, r, y, v0, eta, gpu)
    srpr.sr_plan_set_workspace(plan, torch.empty(srpr.sr_plan_workspace_size(plan), dtype=torch.uint8, device=gpu))
    after = _run(plan, x, r, y, v0, eta, gpu)
    for name, a, b in zip(("z", "v", "gd", "spectral"), before, after):
        assert torch.equal(a, b), name
