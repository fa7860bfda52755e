"""GPU parity of gradient descent on the Poisson negative log-likelihood
(the noise-model loss section II-B.1 allows; guard eps, residual
(1 - y/(|z|^2 + eps)) z) against the FP64 oracle: iterates within 1e-4
after global-phase alignment and loss traces within 1e-4, on every GD path
(2D passes with and without trimming, 1D LDS-resident kernels alone and
batched, the batched level launches, the LDS-resident 2D solver and the
dense model), plus the loss switch's argument checks."""
import numpy as np
import pytest

import oracle
import sr_inputs
from gpu_helpers import aligned, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_IT = 1e-4
MU = 0.05  # dimensionless step: eta = MU / c for the Poisson loss


def _grid(n_shape, m_shape):
    return tuple(max(a, b) for a, b in zip(n_shape, m_shape))


def _data(rng, n_shape, m_shape, L):
    th = rng.uniform(0, 2 * np.pi, (L,) + _grid(n_shape, m_shape)).astype(np.float32)
    xs = sr_inputs.complex_gaussian(rng, n_shape)
    op = oracle.StructuredOperator(th, n_shape, m_shape)
    y = sr_inputs.poisson_counts(rng, np.abs(op.A(xs)) ** 2, 1000.0)
    x0 = (xs + 0.5 * sr_inputs.complex_gaussian(rng, n_shape)).astype(np.complex64)
    eps = float(1e-2 * np.mean(y))
    eta = np.float32(MU / op.c)
    return dict(th=th, op=op, y=y, x0=x0, eps=eps, eta=eta, n_shape=n_shape, m_shape=m_shape, L=L)


def _plan(ds, eps):
    import paper_2409_05734_amd as srpr
    probs = [srpr.Problem(d["n_shape"], d["m_shape"], d["L"]) for d in ds]
    plan = srpr.Plan(probs, np.concatenate([d["th"].ravel() for d in ds]))
    srpr.sr_plan_set_loss(plan, srpr.SR_LOSS_POISSON, eps)
    return plan


def _cat(arrs):
    return np.concatenate([np.asarray(a).ravel() for a in arrs])


def _gd(plan, ds, k, dev, trace):
    import torch
    import paper_2409_05734_amd as srpr
    x = to_dev(_cat([d["x0"] for d in ds]), dev)
    lt = torch.zeros(k * len(ds), dtype=torch.float32, device=dev) if trace else None
    srpr.sr_gd_solve(plan, to_dev(_cat([d["y"] for d in ds]), dev), x, k,
                     np.array([d["eta"] for d in ds], np.float32), lt)
    srpr.sr_plan_sync(plan)
    return to_host(x), (to_host(lt).reshape(len(ds), k) if trace else None)


def _check(plan, ds, xh, lt, k, eps):
    for i, d in enumerate(ds):
        xr, lr = oracle.gd_solve(d["op"], d["y"], d["x0"], k, float(d["eta"]), return_loss=True,
                                 loss="poisson", eps=eps)
        xi = xh[plan.x_off[i]:plan.x_off[i + 1]].reshape(d["n_shape"])
        assert aligned(xi, xr) <= TOL_IT, (d["n_shape"], d["m_shape"], k)
        if lt is not None:
            assert np.max(np.abs(lt[i] - lr) / np.abs(lr)) <= 1e-4, (d["n_shape"], k)


@pytest.mark.parametrize("n_shape,m_shape,L", [((16, 16), (32, 32), 2), ((48, 40), (96, 64), 3),
                                               ((64, 64), (128, 64), 2), ((64, 64), (40, 50), 2),
                                               ((256, 256), (512, 512), 2)])
def test_poisson_gd_2d(gpu, n_shape, m_shape, L):
    rng = np.random.default_rng(hash((n_shape, m_shape, L)) % 2**32)
    d = _data(rng, n_shape, m_shape, L)
    plan = _plan([d], d["eps"])
    for k in ((1, 7) if n_shape[0] >= 256 else (1, 7, 30)):
        xh, lt = _gd(plan, [d], k, gpu, trace=True)
        _check(plan, [d], xh, lt, k, d["eps"])
    # the steady-state (graph-replayed, fused) schedule past one graph chunk
    xh, _ = _gd(plan, [d], 60, gpu, trace=False)
    _check(plan, [d], xh, None, 60, d["eps"])


def test_poisson_gd_1d(gpu):
    rng = np.random.default_rng(71)
    shapes = [((64,), (256,), 2), ((40,), (96,), 3), ((64,), (40,), 2)]
    ds = [_data(rng, *s) for s in shapes]
    eps = float(np.mean([d["eps"] for d in ds]))
    for sub in ([ds[0]], ds):  # one problem alone, then all in one call (batched launches)
        plan = _plan(sub, eps)
        for k in (1, 20):
            xh, lt = _gd(plan, sub, k, gpu, trace=True)
            _check(plan, sub, xh, lt, k, eps)


@pytest.mark.parametrize("resident", ["0", "1"])
def test_poisson_gd_batched(gpu, monkeypatch, resident):
    """The level launches (SR_LDS_RESIDENT=0) and the LDS-resident solver
    (=1) on a batched plan of uneven problems (no loss trace on these paths)."""
    import paper_2409_05734_amd as srpr
    monkeypatch.setenv("SR_LDS_RESIDENT", resident)
    rng = np.random.default_rng(72)
    shapes = [((24, 24), (64, 64), 2), ((12, 10), (16, 32), 1), ((40, 30), (96, 64), 3), ((100, 60), (128, 128), 2),
              ((30, 100), (32, 256), 3), ((64, 64), (128, 64), 2), ((9, 80), (16, 96), 2), ((200, 150), (512, 256), 2)]
    ds = [_data(rng, *s) for s in shapes]
    eps = float(np.mean([d["eps"] for d in ds]))
    plan = _plan(ds, eps)
    srpr.sr_plan_set_schedule(plan, srpr.SR_SCHED_BATCHED)
    for k in (1, 20):
        xh, _ = _gd(plan, ds, k, gpu, trace=False)
        _check(plan, ds, xh, None, k, eps)


@pytest.mark.parametrize("m,n,nb", [(256, 64, 1), (600, 100, 3)])
def test_poisson_gd_dense(gpu, m, n, nb):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(73 + nb)
    A = sr_inputs.complex_gaussian(rng, (m, n))
    op = oracle.DenseOperator(A)
    xs = sr_inputs.complex_gaussian(rng, (nb, n))
    Y = np.stack([sr_inputs.poisson_counts(rng, np.abs(op.A(xs[p])) ** 2) for p in range(nb)])
    X0 = (xs + 0.5 * sr_inputs.complex_gaussian(rng, (nb, n))).astype(np.complex64)
    eps = float(1e-2 * np.mean(Y))
    eta = np.float32(MU)  # c = 1
    Ad = to_dev(np.ascontiguousarray(A), gpu)
    plan = srpr.Plan([srpr.Problem((n,), (m,), 1, kind=srpr.SR_DENSE) for _ in range(nb)], None, dense_A=Ad)
    srpr.sr_plan_set_loss(plan, srpr.SR_LOSS_POISSON, eps)
    for k in (1, 30):
        x = to_dev(X0.ravel(), gpu)
        lt = torch.zeros(k * nb, dtype=torch.float32, device=gpu)
        srpr.sr_gd_solve(plan, to_dev(Y.ravel(), gpu), x, k, eta, lt)
        srpr.sr_plan_sync(plan)
        for p in range(nb):
            xr, lr = oracle.gd_solve(op, Y[p], X0[p], k, float(eta), return_loss=True, loss="poisson", eps=eps)
            assert aligned(to_host(x).reshape(nb, n)[p], xr) <= TOL_IT
            assert np.max(np.abs(to_host(lt).reshape(nb, k)[p] - lr) / np.abs(lr)) <= 1e-4


def test_loss_switch_arguments_and_return_to_l2(gpu):
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(74)
    d = _data(rng, (16, 16), (32, 32), 2)
    plan = _plan([d], d["eps"])
    for loss, eps in ((srpr.SR_LOSS_POISSON, 0.0), (srpr.SR_LOSS_POISSON, -1.0), (srpr.SR_LOSS_POISSON, float("nan")),
                      (srpr.SR_LOSS_POISSON, float("inf")), (7, 1.0)):
        with pytest.raises(srpr.SrError):
            srpr.sr_plan_set_loss(plan, loss, eps)
    # back to the l2 loss: the plan's GD follows the l2 oracle again
    srpr.sr_plan_set_loss(plan, srpr.SR_LOSS_L2)
    eta = np.float32(oracle.default_step(d["op"], d["y"], 0.2))
    d2 = dict(d, eta=eta)
    xh, _ = _gd(plan, [d2], 10, gpu, trace=False)
    xr = oracle.gd_solve(d["op"], d["y"], d["x0"], 10, float(eta))
    assert aligned(xh.reshape(d["n_shape"]), xr) <= TOL_IT
