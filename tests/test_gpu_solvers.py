"""GPU parity of the solvers against the FP64 oracle: gradient-descent
iterates (section II-B.1, Eq. (2)) within 1e-4 relative error after global
phase alignment for the first 50 steps, spectral initialisation (Eq. (3)-(4))
iterates, loss traces, and determinism."""
import numpy as np
import pytest

import oracle
import sr_inputs
from gpu_helpers import aligned, make_plan, random_problem, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_IT = 1e-4


def _run_gd(plan, y, x0, iters, eta, dev, loss=False):
    import torch
    import paper_2409_05734_amd as srpr
    xd = to_dev(x0.ravel().astype(np.complex64), dev)
    lt = torch.zeros(iters * plan.nprob, dtype=torch.float32, device=dev) if loss else None
    srpr.sr_gd_solve(plan, to_dev(y.ravel().astype(np.float32), dev), xd, iters, eta, lt)
    torch.cuda.synchronize()
    return to_host(xd), (to_host(lt) if loss else None)


def _run_spec(plan, y, v0, iters, lam, dev):
    import torch
    import paper_2409_05734_amd as srpr
    out = torch.empty(plan.n_total, dtype=torch.complex64, device=dev)
    srpr.sr_spectral_init(plan, to_dev(y.ravel().astype(np.float32), dev), to_dev(v0.ravel().astype(np.complex64), dev),
                          iters, lam, out)
    torch.cuda.synchronize()
    return to_host(out)


GD_CASES = [
    ((64,), (256,), 2),
    ((40,), (96,), 3),
    ((16, 16), (32, 32), 2),
    ((20, 12), (32, 64), 1),
    ((48, 40), (96, 64), 3),
    ((64, 64), (128, 64), 2),
]


@pytest.mark.parametrize("n_shape,m_shape,L", GD_CASES)
def test_gd_iterates(gpu, n_shape, m_shape, L):
    """Start in the basin of x* (x* plus CN(0, 1/4) noise) so that GD at
    mu = 0.2 converges for every shape (the oracle's own trajectory)."""
    rng = np.random.default_rng(10 + len(n_shape) * 7 + L)
    th, xs = random_problem(rng, n_shape, m_shape, L)
    op = oracle.StructuredOperator(th, n_shape)
    y = (np.abs(op.A(xs)) ** 2).astype(np.float32)
    x0 = (xs + 0.5 * sr_inputs.complex_gaussian(rng, n_shape)).astype(np.complex64)
    eta = np.float32(oracle.default_step(op, y, 0.2))
    plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
    for k in (1, 7, 50):
        xg, _ = _run_gd(plan, y, x0, k, eta, gpu)
        xr = oracle.gd_solve(op, y, x0, k, float(eta))
        assert aligned(xg.reshape(n_shape), xr) <= TOL_IT, k


@pytest.mark.parametrize("force", ["8,1,1", "2,4,0", "16,1,1", "2|n,1|n,1", "8|n,2|n,0", "4|n,1,1"])
def test_gd_iterates_every_pass_shape(gpu, monkeypatch, force):
    """The fused solver passes (turnaround with the residual, the update fused
    with the next first pass) on pinned tile shapes, default and narrow,
    against the oracle's GD iterates on a 512 x 512 grid and a 128 x 256 grid."""
    c, r, t = (int(v.replace("|n", "")) | (512 if "|n" in v else 0) for v in force.split(","))
    monkeypatch.setenv("SR_TUNE_FORCE", f"{c},{r},{t}")
    for n_shape, m_shape, L in (((200, 180), (512, 512), 2), ((60, 100), (128, 256), 3)):
        rng = np.random.default_rng(77 + L)
        th, xs = random_problem(rng, n_shape, m_shape, L)
        op = oracle.StructuredOperator(th, n_shape)
        y = (np.abs(op.A(xs)) ** 2).astype(np.float32)
        x0 = (xs + 0.5 * sr_inputs.complex_gaussian(rng, n_shape)).astype(np.complex64)
        eta = np.float32(oracle.default_step(op, y, 0.2))
        plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
        for k in (1, 20):
            xg, _ = _run_gd(plan, y, x0, k, eta, gpu)
            xr = oracle.gd_solve(op, y, x0, k, float(eta))
            assert aligned(xg.reshape(n_shape), xr) <= TOL_IT, (n_shape, k)


@pytest.mark.parametrize("n_shape,m_shape,L", [((64, 64), (128, 64), 1), ((128, 128), (256, 128), 1),
                                               ((64,), (128,), 1)])
def test_gd_steps_along_unstable_trajectory(gpu, n_shape, m_shape, L):
    """alpha = 2, L = 1 from a random start: GD amplifies rounding along the
    trajectory, so whole trajectories of any two FP32 implementations drift
    apart.  The arithmetic is checked step by step instead: from each oracle
    iterate x_k (k = 0..50), one GPU step must reproduce the oracle's x_{k+1}."""
    rng = np.random.default_rng(91 + len(n_shape))
    th, xs = random_problem(rng, n_shape, m_shape, L)
    op = oracle.StructuredOperator(th, n_shape)
    y = (np.abs(op.A(xs)) ** 2).astype(np.float32)
    x = sr_inputs.scaled_start(rng, n_shape, float(np.sum(y))).astype(np.complex128)
    eta = np.float32(oracle.default_step(op, y, 0.2))
    plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
    for k in range(51):
        xr = oracle.gd_solve(op, y, x, 1, float(eta))
        xg, _ = _run_gd(plan, y, x.astype(np.complex64), 1, eta, gpu)
        assert rel_l2(xg.reshape(n_shape), xr) <= 2e-5, k
        x = xr


def test_gd_loss_trace(gpu):
    rng = np.random.default_rng(21)
    for n_shape, m_shape, L in [((64,), (256,), 2), ((24, 24), (64, 64), 2)]:
        th, xs = random_problem(rng, n_shape, m_shape, L)
        op = oracle.StructuredOperator(th, n_shape)
        y = (np.abs(op.A(xs)) ** 2).astype(np.float32)
        x0 = sr_inputs.scaled_start(rng, n_shape, float(np.sum(y)))
        eta = np.float32(oracle.default_step(op, y, 0.2))
        plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
        _, lg = _run_gd(plan, y, x0, 12, eta, gpu, loss=True)
        _, lr = oracle.gd_solve(op, y, x0, 12, float(eta), return_loss=True)
        assert np.max(np.abs(lg - lr) / lr) <= 1e-4


@pytest.mark.parametrize("n_shape,m_shape,L", GD_CASES)
def test_spectral_init(gpu, n_shape, m_shape, L):
    rng = np.random.default_rng(30 + L)
    th, xs = random_problem(rng, n_shape, m_shape, L)
    op = oracle.StructuredOperator(th, n_shape)
    z = op.A(xs)
    y = sr_inputs.poisson_counts(rng, np.abs(z) ** 2, 1000.0)
    v0 = sr_inputs.complex_gaussian(rng, n_shape)
    plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
    for k in (1, 10, 40):
        xg = _run_spec(plan, y, v0, k, -1.0, gpu)
        xr = oracle.spectral_init(op, y, v0, k, -1.0)
        assert rel_l2(xg.reshape(n_shape), xr) <= TOL_IT, k


def test_image_workload_parity(gpu):
    """The 2D image workload at full size: 256^2 smooth image padded to 512^2,
    L = 2, Poisson noise at 1000 photons.  20 power iterations, then GD
    iterates compared at steps 1, 10 and 50."""
    d = sr_inputs.image_2d(1)
    n_shape, m_shape, L = d["n_shape"], d["m_shape"], d["layers"]
    th, xs = d["theta"], d["x_star"]
    op = oracle.StructuredOperator(th, n_shape)
    y = sr_inputs.poisson_counts(d["noise_rng"], np.abs(op.A(xs)) ** 2, d["photons"])
    plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
    xg0 = _run_spec(plan, y, d["v0"], 20, d["lam"], gpu)
    xr0 = oracle.spectral_init(op, y, d["v0"], 20, d["lam"])
    assert rel_l2(xg0.reshape(n_shape), xr0) <= TOL_IT
    x0 = xr0.astype(np.complex64)
    eta = np.float32(oracle.default_step(op, y, d["mu"]))
    xr = x0.astype(np.complex128)
    done = 0
    for k in (1, 10, 50):
        xr = oracle.gd_solve(op, y, xr, k - done, float(eta))
        done = k
        xg, _ = _run_gd(plan, y, x0, k, eta, gpu)
        assert aligned(xg.reshape(n_shape), xr) <= TOL_IT, k


def test_tiny_1d_end_to_end_recovers(gpu):
    d = sr_inputs.tiny_1d(0)
    th, xs = d["theta"], d["x_star"]
    op = oracle.StructuredOperator(th, d["n_shape"])
    y = (np.abs(op.A(xs)) ** 2).astype(np.float32)
    plan = make_plan([(d["n_shape"], d["m_shape"], d["layers"])], [th], gpu)
    x0 = _run_spec(plan, y, d["v0"], d["pi_iters"], d["lam"], gpu)
    eta = np.float32(oracle.default_step(op, y, d["mu"]))
    x, _ = _run_gd(plan, y, x0, d["gd_iters"], eta, gpu)
    assert oracle.cosine_similarity(x, xs) > 0.9999


def test_determinism(gpu):
    rng = np.random.default_rng(40)
    th, xs = random_problem(rng, (48, 40), (96, 64), 3)
    op = oracle.StructuredOperator(th, (48, 40))
    y = (np.abs(op.A(xs)) ** 2).astype(np.float32)
    v0 = sr_inputs.complex_gaussian(rng, (48, 40))
    plan = make_plan([((48, 40), (96, 64), 3)], [th], gpu)
    a = _run_spec(plan, y, v0, 15, -1.0, gpu)
    b = _run_spec(plan, y, v0, 15, -1.0, gpu)
    assert np.array_equal(a, b)
    g1, l1 = _run_gd(plan, y, a, 20, 0.5, gpu, loss=True)
    g2, l2 = _run_gd(plan, y, a, 20, 0.5, gpu, loss=True)
    assert np.array_equal(g1, g2) and np.array_equal(l1, l2)


def test_zero_iterations_and_edge_inputs(gpu):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(41)
    th, xs = random_problem(rng, (16, 16), (32, 32), 2)
    plan = make_plan([((16, 16), (32, 32), 2)], [th], gpu)
    x = to_dev(xs.ravel(), gpu)
    before = x.clone()
    y = torch.zeros(1024, dtype=torch.float32, device=gpu)
    srpr.sr_gd_solve(plan, y, x, 0, 1.0)
    torch.cuda.synchronize()
    assert torch.equal(x, before)
    # all-zero measurements: T = lambda everywhere, the spectral estimate is 0 * v
    with pytest.raises(srpr.SrError):
        srpr.sr_spectral_init(plan, y, x, 3, 0.5, torch.empty_like(x))  # lambda must be < 0
    with pytest.raises(srpr.SrError):
        srpr.sr_gd_solve(plan, y, x, 3, float("nan"))


@pytest.mark.parametrize("n_shape,m_shape,L", [((256, 256), (512, 512), 2), ((100, 120), (256, 256), 3),
                                               ((128, 128), (256, 256), 1)])
def test_schedules_agree(gpu, monkeypatch, n_shape, m_shape, L):
    """Graph-replayed chunks and direct launches run the same kernels: GD
    iterates agree bit for bit.  The single-launch persistent solver runs the
    unfused pass sequence and groups partial norms by its own tiles: it agrees
    to rounding."""
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(50 + L)
    th, xs = random_problem(rng, n_shape, m_shape, L)
    op = oracle.StructuredOperator(th, n_shape)
    y = (np.abs(op.A(xs)) ** 2).astype(np.float32)
    v0 = sr_inputs.complex_gaussian(rng, n_shape)
    x0 = (xs + 0.5 * sr_inputs.complex_gaussian(rng, n_shape)).astype(np.complex64)
    eta = np.float32(oracle.default_step(op, y, 0.2))
    plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
    g_auto, _ = _run_gd(plan, y, x0, 120, eta, gpu)            # two graph chunks + 20 direct iterations
    s_auto = _run_spec(plan, y, v0, 111, -1.0, gpu)
    g_auto2, _ = _run_gd(plan, y, x0, 120, eta, gpu)           # cached graphs
    monkeypatch.setenv("SR_PERSIST_B", "8")
    g_pers, l_pers = _run_gd(plan, y, x0, 120, eta, gpu, loss=True)
    s_pers = _run_spec(plan, y, v0, 111, -1.0, gpu)
    monkeypatch.delenv("SR_PERSIST_B")
    srpr.sr_plan_set_schedule(plan, srpr.SR_SCHED_LOOP)
    g_loop, l_loop = _run_gd(plan, y, x0, 120, eta, gpu, loss=True)
    s_loop = _run_spec(plan, y, v0, 111, -1.0, gpu)
    srpr.sr_plan_sync(plan)
    assert np.array_equal(g_auto, g_loop) and np.array_equal(g_auto2, g_loop)
    # the persistent solver runs the unfused pass sequence (separate first pass)
    assert rel_l2(g_pers, g_loop) < 1e-5
    assert np.max(np.abs(l_pers - l_loop) / l_loop) < 1e-5
    assert rel_l2(s_auto, s_loop) < 1e-5 and rel_l2(s_pers, s_loop) < 1e-5
    assert rel_l2(s_auto.reshape(n_shape), oracle.spectral_init(op, y, v0, 111, -1.0)) <= TOL_IT
