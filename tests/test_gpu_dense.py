"""GPU parity of the dense i.i.d. complex Gaussian baseline (section II-A) on
FP32 MFMA against the FP64 oracle: A x and A^H r per application (relative
L2 <= 2e-5), GD iterates (<= 1e-4 after phase alignment), spectral
initialisation, loss traces, ragged shapes and the full 16384 x 4096 x 32
baseline size, each on the hand-written products and on the library GEMM."""
import numpy as np
import pytest

import oracle
import sr_inputs
from gpu_helpers import aligned, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_OP = 2e-5
TOL_IT = 1e-4


@pytest.fixture(autouse=True, params=["own", "lib"])
def dense_products(request, monkeypatch):
    """Every test on both implementations of the two real products: the
    hand-written MFMA kernel and the library GEMM (the plan's timed choice
    is one of the two)."""
    monkeypatch.setenv("SR_DENSE_GEMM", request.param)
    return request.param


def _plan(A, nb, dev):
    import paper_2409_05734_amd as srpr
    m, n = A.shape
    probs = [srpr.Problem((n,), (m,), 1, kind=srpr.SR_DENSE) for _ in range(nb)]
    Ad = to_dev(np.ascontiguousarray(A.astype(np.complex64)), dev)
    return srpr.Plan(probs, None, dense_A=Ad), Ad


@pytest.mark.parametrize("m,n,nb", [(256, 64, 1), (200, 50, 3), (1000, 130, 33), (64, 2, 2), (4096, 1024, 32)])
def test_dense_forward_adjoint(gpu, m, n, nb):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(m + n + nb)
    A = sr_inputs.complex_gaussian(rng, (m, n))
    X = sr_inputs.complex_gaussian(rng, (nb, n))
    R = sr_inputs.complex_gaussian(rng, (nb, m))
    plan, _ = _plan(A, nb, gpu)
    z = torch.empty(nb * m, dtype=torch.complex64, device=gpu)
    y = torch.empty(nb * m, dtype=torch.float32, device=gpu)
    v = torch.empty(nb * n, dtype=torch.complex64, device=gpu)
    srpr.sr_forward(plan, to_dev(X.ravel(), gpu), z, y)
    srpr.sr_adjoint(plan, to_dev(R.ravel(), gpu), v)
    torch.cuda.synchronize()
    op = oracle.DenseOperator(A)
    zh, vh = to_host(z).reshape(nb, m), to_host(v).reshape(nb, n)
    for p in range(nb):
        zr = op.A(X[p])
        assert rel_l2(zh[p], zr) <= TOL_OP
        assert rel_l2(to_host(y).reshape(nb, m)[p], np.abs(zr) ** 2) <= 2 * TOL_OP
        assert rel_l2(vh[p], op.AH(R[p])) <= TOL_OP


def test_dense_full_size_baseline(gpu):
    """16384 x 4096 complex64 A (512 MiB) on 32 signals, every output checked."""
    import torch
    import paper_2409_05734_amd as srpr
    d = sr_inputs.dense_batch(4)
    A, X, R = d["dense_A"], d["X"], d["R"]
    plan, _ = _plan(A, 32, gpu)
    z = torch.empty(32 * 16384, dtype=torch.complex64, device=gpu)
    v = torch.empty(32 * 4096, dtype=torch.complex64, device=gpu)
    srpr.sr_forward(plan, to_dev(X.ravel(), gpu), z, None)
    srpr.sr_adjoint(plan, to_dev(R.ravel(), gpu), v)
    torch.cuda.synchronize()
    A64 = A.astype(np.complex128)
    Z = X.astype(np.complex128) @ A64.T
    V = R.astype(np.complex128) @ A64.conj()
    assert rel_l2(to_host(z).reshape(32, 16384), Z) <= TOL_OP
    assert rel_l2(to_host(v).reshape(32, 4096), V) <= TOL_OP


@pytest.mark.parametrize("m,n,nb", [(256, 64, 1), (600, 100, 3)])
def test_dense_solvers(gpu, m, n, nb):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(7 + nb)
    A = sr_inputs.complex_gaussian(rng, (m, n))
    op = oracle.DenseOperator(A)
    xs = sr_inputs.complex_gaussian(rng, (nb, n))
    Y = np.stack([(np.abs(op.A(xs[p])) ** 2) for p in range(nb)]).astype(np.float32)
    V0 = sr_inputs.complex_gaussian(rng, (nb, n))
    plan, _ = _plan(A, nb, gpu)
    yd = to_dev(Y.ravel(), gpu)
    for K in (1, 20):
        out = torch.empty(nb * n, dtype=torch.complex64, device=gpu)
        srpr.sr_spectral_init(plan, yd, to_dev(V0.ravel(), gpu), K, -1.0, out)
        torch.cuda.synchronize()
        for p in range(nb):
            assert rel_l2(to_host(out).reshape(nb, n)[p], oracle.spectral_init(op, Y[p], V0[p], K, -1.0)) <= TOL_IT
    X0 = (xs + 0.5 * sr_inputs.complex_gaussian(rng, (nb, n))).astype(np.complex64)
    eta = np.float32(0.2 / float(np.mean(Y.astype(np.float64))))
    for K in (1, 30):
        x = to_dev(X0.ravel(), gpu)
        lt = torch.zeros(K * nb, dtype=torch.float32, device=gpu)
        srpr.sr_gd_solve(plan, yd, x, K, eta, lt)
        torch.cuda.synchronize()
        for p in range(nb):
            xr, lr = oracle.gd_solve(op, Y[p], X0[p], K, float(eta), return_loss=True)
            assert aligned(to_host(x).reshape(nb, n)[p], xr) <= TOL_IT
            assert np.max(np.abs(to_host(lt).reshape(nb, K)[p] - lr) / lr) <= 1e-4


def test_tiny_dense_end_to_end(gpu):
    import torch
    import paper_2409_05734_amd as srpr
    d = sr_inputs.tiny_1d(0)
    A, xs = d["dense_A"], d["x_star"]
    op = oracle.DenseOperator(A)
    y = (np.abs(op.A(xs)) ** 2).astype(np.float32)
    plan, _ = _plan(A, 1, gpu)
    x = torch.empty(64, dtype=torch.complex64, device=gpu)
    yd = to_dev(y, gpu)
    srpr.sr_spectral_init(plan, yd, to_dev(d["v0"], gpu), d["pi_iters"], d["lam"], x)
    srpr.sr_gd_solve(plan, yd, x, d["gd_iters"], np.float32(oracle.default_step(op, y, 0.2)))
    torch.cuda.synchronize()
    assert oracle.cosine_similarity(to_host(x), xs) > 0.999
