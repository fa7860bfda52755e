"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-type the oracle's formulas: they compare it with a library
DFT (numpy.fft), hand-derived worked examples (tests/golden), brute-force
explicit matrices built through a different route, closed forms that follow
from F being unitary and |D_l| = 1 (section III), an eigendecomposition
(spectral method, Eq. (3)-(4)), and finite differences (Eq. (2) gradient and
the mask-design gradients).
"""
import os

import numpy as np
import pytest

import oracle
import sr_inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cgauss(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- DFT, padding

@pytest.mark.parametrize("N", [1, 2, 3, 4, 6, 8, 12, 16, 24, 64, 96])
def test_dft_matrix_matches_library_fft(N):
    F = oracle.dft_matrix(N)
    ref = np.fft.fft(np.eye(N), axis=0, norm="ortho")
    assert np.abs(F - ref).max() < 1e-13


@pytest.mark.parametrize("shape", [(8,), (6, 10), (12, 8), (3, 16)])
def test_apply_dft_matches_library_fftn(shape):
    rng = np.random.default_rng(1)
    X = _cgauss(rng, shape)
    assert np.abs(oracle.apply_dft(X) - np.fft.fftn(X, norm="ortho")).max() < 1e-12
    assert np.abs(oracle.apply_dft(X, inverse=True) - np.fft.ifftn(X, norm="ortho")).max() < 1e-12


def test_pad_offsets_and_window_by_hand():
    assert oracle.pad_offsets((64,), (256,)) == (96,)
    assert oracle.pad_offsets((256, 256), (512, 512)) == (128, 128)
    assert oracle.pad_offsets((5, 3), (8, 3)) == (1, 0)
    x = np.array([[1, 2], [3, 4]], dtype=complex)
    X = oracle.zero_pad(x, (4, 5))  # offsets (1, 1)
    expect = np.zeros((4, 5), dtype=complex)
    expect[1, 1], expect[1, 2], expect[2, 1], expect[2, 2] = 1, 2, 3, 4
    assert np.array_equal(X, expect)
    assert np.array_equal(oracle.crop(X, (2, 2)), x)


# ------------------------------------------------------- hand worked examples

def test_golden_hand_operator_1d():
    rows = _read_golden("hand_structured_1d_m4.txt")
    d = {}
    A = np.zeros((4, 2), dtype=complex)
    for r in rows:
        if r[0] == "A":
            i, j = map(int, r[1].split(","))
            A[i, j] = float(r[2]) + 1j * float(r[3])
        else:
            d[r[0]] = np.array([float(v) for v in r[1:]])
    th1 = d["theta1"].reshape(1, 4)
    assert np.abs(oracle.dense_matrix(th1, (2,)) - A).max() < 1e-15
    for tag in ("a", "b"):
        xv = d["x_" + tag]
        x = xv[0::2] + 1j * xv[1::2]
        assert np.abs(oracle.measurements(x, th1) - d["y_" + tag]).max() < 1e-15
    th2 = np.stack([d["theta1"], np.zeros(4)])
    zv = d["z2_b"]
    z2 = zv[0::2] + 1j * zv[1::2]
    xb = np.array([1, 1j])
    assert np.abs(oracle.forward(xb, th2) - z2).max() < 1e-15


def test_golden_hand_preprocess():
    rows = _read_golden("hand_preprocess.txt")
    y = np.array([float(v) for v in rows[0][1:]])
    for r in rows[1:]:
        lam = float(r[1])
        T = np.array([float(v) for v in r[3:]])
        assert np.abs(oracle.preprocess(y, lam) - T).max() < 1e-15
        assert np.abs(oracle.preprocess(7.5 * y, lam) - T).max() < 1e-15


# ------------------------------------------------ special cases (theta == 0)

@pytest.mark.parametrize("n_shape,m_shape", [((4,), (16,)), ((3, 5), (6, 10)), ((4, 4), (16, 8))])
def test_zero_phase_single_layer_is_padded_fft(n_shape, m_shape):
    rng = np.random.default_rng(2)
    x = _cgauss(rng, n_shape)
    Xp = np.zeros(m_shape, dtype=complex)
    off = [(M - N) // 2 for N, M in zip(n_shape, m_shape)]
    Xp[tuple(slice(o, o + N) for o, N in zip(off, n_shape))] = x
    th = np.zeros((1,) + m_shape)
    assert np.abs(oracle.forward(x, th) - np.fft.fftn(Xp, norm="ortho")).max() < 1e-12


@pytest.mark.parametrize("m_shape", [(16,), (6, 10)])
def test_zero_phase_two_layers_is_index_reversal(m_shape):
    rng = np.random.default_rng(3)
    n_shape = tuple(M // 2 for M in m_shape)
    x = _cgauss(rng, n_shape)
    Xp = oracle.zero_pad(x, m_shape)
    idx = np.ix_(*[(-np.arange(M)) % M for M in m_shape])
    th = np.zeros((2,) + m_shape)
    assert np.abs(oracle.forward(x, th) - Xp[idx]).max() < 1e-12


def test_zero_phase_four_layers_is_identity():
    rng = np.random.default_rng(4)
    x = _cgauss(rng, (3, 4))
    th = np.zeros((4, 6, 8))
    assert np.abs(oracle.forward(x, th) - oracle.zero_pad(x, (6, 8))).max() < 1e-12


# ------------------------------------------------------------ brute force A

def _brute_force_A(thetas, n_shape):
    """A = prod_l (F D_l) U with F built from numpy.fft on identity columns
    (Kronecker product across axes) and U as an explicit 0/1 selection."""
    m_shape = thetas.shape[1:]
    m, n = int(np.prod(m_shape)), int(np.prod(n_shape))
    F = np.ones((1, 1))
    for M in m_shape:
        F = np.kron(F, np.fft.fft(np.eye(M), axis=0, norm="ortho"))
    U = np.zeros((m, n))
    off = [(M - N) // 2 for N, M in zip(n_shape, m_shape)]
    for j in range(n):
        jj = np.unravel_index(j, n_shape)
        ii = tuple(o + a for o, a in zip(off, jj))
        U[np.ravel_multi_index(ii, m_shape), j] = 1.0
    A = U.astype(complex)
    for th in thetas:
        A = F @ (np.exp(1j * th.ravel())[:, None] * A)
    return A


@pytest.mark.parametrize("n_shape,m_shape,L", [
    ((4,), (16,), 1), ((4,), (16,), 2), ((16,), (64,), 2), ((5,), (12,), 3),
    ((2, 3), (4, 6), 1), ((3, 2), (6, 4), 2), ((4, 4), (8, 8), 2), ((2, 2), (8, 4), 3),
    ((4, 4), (8, 4), 2),
])
def test_operator_matches_brute_force_dense(n_shape, m_shape, L):
    rng = np.random.default_rng(5)
    th = rng.uniform(0, 2 * np.pi, (L,) + m_shape)
    A_or = oracle.dense_matrix(th, n_shape)
    A_bf = _brute_force_A(th, n_shape)
    assert np.abs(A_or - A_bf).max() < 1e-12
    # adjoint = conjugate transpose, column by column
    m = int(np.prod(m_shape))
    r = _cgauss(rng, m_shape)
    assert np.abs(oracle.adjoint(r, th, n_shape).ravel() - A_bf.conj().T @ r.ravel()).max() < 1e-12
    assert m == A_bf.shape[0]


@pytest.mark.parametrize("n_shape,m_shape,L", [((16,), (64,), 2), ((6, 5), (12, 10), 1),
                                                ((6, 6), (12, 12), 3), ((4, 4), (16, 8), 2)])
def test_unitarity_parseval_and_adjoint_identity(n_shape, m_shape, L):
    rng = np.random.default_rng(6)
    th = rng.uniform(0, 2 * np.pi, (L,) + m_shape)
    A = oracle.dense_matrix(th, n_shape)
    n = A.shape[1]
    assert np.abs(A.conj().T @ A - np.eye(n)).max() < 1e-12          # A^H A = I_n
    x = _cgauss(rng, n_shape)
    z = _cgauss(rng, m_shape)
    Ax = oracle.forward(x, th)
    assert abs(np.linalg.norm(Ax) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)
    assert abs(oracle.measurements(x, th).sum() - np.vdot(x, x).real) < 1e-11 * np.vdot(x, x).real
    lhs = np.vdot(Ax, z)
    rhs = np.vdot(x, oracle.adjoint(z, th, n_shape))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) + 1e-12


# -------------------------------------------------------------- spectral init

def _spectral_closed_form(M, lam, v0, K):
    mu, E = np.linalg.eigh(M)
    c = E.conj().T @ v0
    v = E @ (c * (mu - 2 * lam) ** K)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("kind", ["structured", "dense"])
def test_power_iteration_matches_eigendecomposition(kind):
    rng = np.random.default_rng(7)
    n, m = 16, 64
    xs = _cgauss(rng, (n,))
    if kind == "structured":
        th = rng.uniform(0, 2 * np.pi, (2, m))
        op = oracle.StructuredOperator(th, (n,))
        A = _brute_force_A(th, (n,))
        c = 1.0 / m
    else:
        A = _cgauss(rng, (m, n)) / np.sqrt(2)
        op = oracle.DenseOperator(A)
        c = 1.0
    y = np.abs(A @ xs) ** 2
    lam = -0.7
    T = oracle.preprocess(y, lam)
    M = A.conj().T @ (T[:, None] * A) / (m * c)
    assert np.abs(M - M.conj().T).max() < 1e-13
    if kind == "structured":
        ev = np.linalg.eigvalsh(M)
        assert ev.min() >= lam - 1e-12 and ev.max() < 1.0
    v0 = _cgauss(rng, (n,))
    for K in (1, 5, 30):
        out, its = oracle.spectral_init(op, y, v0, K, lam, return_iterates=True)
        vk = its[-1]
        assert np.abs(vk - _spectral_closed_form(M, lam, v0, K)).max() < 1e-10
        assert abs(np.linalg.norm(out) - np.sqrt(y.sum() / (m * c))) < 1e-10
    # converged limit: the top eigenvector (up to phase)
    out = oracle.spectral_init(op, y, v0, 3000, lam)
    top = np.linalg.eigh(M)[1][:, -1]
    assert oracle.cosine_similarity(out, top) > 1 - 1e-8


# ---------------------------------------------------------- gradient descent

def test_gd_gradient_matches_finite_differences():
    rng = np.random.default_rng(8)
    th = rng.uniform(0, 2 * np.pi, (2, 6, 8))
    op = oracle.StructuredOperator(th, (3, 4))
    xs = _cgauss(rng, (3, 4))
    y = oracle.measurements(xs, th) * rng.uniform(0.5, 1.5, (6, 8))
    x = _cgauss(rng, (3, 4))
    g = oracle.gd_gradient(op, y, x)
    for _ in range(8):
        d = _cgauss(rng, (3, 4))
        eps = 1e-6
        fd = (oracle.intensity_loss(op, y, x + eps * d) - oracle.intensity_loss(op, y, x - eps * d)) / (2 * eps)
        # L = sum (|z|^2 - y)^2 has dL = 4 m Re<g, dx>
        assert abs(fd - 4 * op.m * np.vdot(g, d).real) < 1e-6 * (abs(fd) + 1)


def test_gd_gradient_vanishes_at_truth_up_to_global_phase():
    rng = np.random.default_rng(9)
    th = rng.uniform(0, 2 * np.pi, (2, 64))
    op = oracle.StructuredOperator(th, (16,))
    xs = _cgauss(rng, (16,))
    y = oracle.measurements(xs, th)
    for phi in (0.0, 1.3, -2.9):
        assert np.abs(oracle.gd_gradient(op, y, xs * np.exp(1j * phi))).max() < 1e-12


def test_poisson_gradient_matches_finite_differences():
    """Reading R18: the Poisson gradient against central differences of the
    Poisson loss, on a 2D structured and a dense model (noisy y, so the point
    is not a stationary one)."""
    rng = np.random.default_rng(31)
    th = rng.uniform(0, 2 * np.pi, (2, 6, 8))
    ops = [oracle.StructuredOperator(th, (3, 4)),
           oracle.DenseOperator((rng.standard_normal((40, 12)) + 1j * rng.standard_normal((40, 12))) / np.sqrt(2))]
    for op in ops:
        n_shape = (3, 4) if op is ops[0] else (12,)
        xs = _cgauss(rng, n_shape)
        y = np.abs(op.A(xs)) ** 2 * rng.uniform(0.5, 1.5, np.shape(op.A(xs)))
        x = _cgauss(rng, n_shape)
        for eps in (1e-3, 0.5):
            g = oracle.poisson_gradient(op, y, x, eps)
            for _ in range(6):
                d = _cgauss(rng, n_shape)
                h = 1e-6
                fd = (oracle.poisson_loss(op, y, x + h * d, eps) - oracle.poisson_loss(op, y, x - h * d, eps)) / (2 * h)
                # a real f with Wirtinger gradient G has df = 2 Re<G, dx>; g = G / m
                assert abs(fd - 2 * op.m * np.vdot(g, d).real) < 1e-6 * (abs(fd) + 1)


def test_poisson_gradient_vanishes_at_truth_and_differs_from_l2():
    """With noiseless y the truth (any global phase) is a stationary point of
    the Poisson loss as eps -> 0; away from it the Poisson and l2 steps point
    in different directions (the loss switch is not a no-op)."""
    rng = np.random.default_rng(32)
    th = rng.uniform(0, 2 * np.pi, (2, 64))
    op = oracle.StructuredOperator(th, (16,))
    xs = _cgauss(rng, (16,))
    y = oracle.measurements(xs, th)
    for phi in (0.0, 2.2):
        assert np.abs(oracle.poisson_gradient(op, y, xs * np.exp(1j * phi), 1e-14)).max() < 1e-10
    x = xs + 0.3 * _cgauss(rng, (16,))
    gp, gl = oracle.poisson_gradient(op, y, x, 1e-6), oracle.gd_gradient(op, y, x)
    assert oracle.cosine_similarity(gp, gl) < 0.999
    # a small Poisson GD run from near the truth lowers the Poisson loss monotonically
    _, losses = oracle.gd_solve(op, y, x, 20, 0.05 * op.m, return_loss=True, loss="poisson", eps=1e-6)
    assert np.all(np.diff(losses) < 0)
    with pytest.raises(ValueError):
        oracle.gd_solve(op, y, x, 1, 0.1, loss="poisson", eps=0.0)


def test_tiny_1d_recovers_signal():
    d = sr_inputs.tiny_1d(0)
    xs = d["x_star"].astype(np.complex128)
    op = oracle.StructuredOperator(d["theta"], d["n_shape"])
    y = np.abs(op.A(xs)) ** 2
    x0 = oracle.spectral_init(op, y, d["v0"], d["pi_iters"], d["lam"])
    eta = oracle.default_step(op, y, d["mu"])
    x, losses = oracle.gd_solve(op, y, x0, d["gd_iters"], eta, return_loss=True)
    assert oracle.cosine_similarity(x, xs) > 0.9999
    assert np.all(np.diff(losses) <= 1e-12 * losses[0])  # monotone at mu = 0.2
    # dense i.i.d. model on the same signal
    opd = oracle.DenseOperator(d["dense_A"])
    yd = np.abs(opd.A(xs)) ** 2
    x0d = oracle.spectral_init(opd, yd, d["v0"], d["pi_iters"], d["lam"])
    xd = oracle.gd_solve(opd, yd, x0d, d["gd_iters"], oracle.default_step(opd, yd, 0.2))
    assert oracle.cosine_similarity(xd, xs) > 0.999


# ------------------------------------------------------------------ metrics

def test_cosine_similarity_and_alignment():
    a = np.array([1.0, 0.0])
    b = np.array([1.0, 1.0])
    assert abs(oracle.cosine_similarity(a, b) - 1 / np.sqrt(2)) < 1e-15
    assert oracle.cosine_similarity(np.array([1.0, 0]), np.array([0, 1.0])) == 0.0
    rng = np.random.default_rng(10)
    x = _cgauss(rng, (5, 3))
    y = 3.7 * np.exp(0.8j) * x
    assert abs(oracle.cosine_similarity(y, x) - 1.0) < 1e-14
    assert oracle.aligned_rel_error(np.exp(2.1j) * x, x) < 1e-14


# ------------------------------------------------------- mask-design gradients

def test_forward_and_adjoint_vjp_match_finite_differences():
    rng = np.random.default_rng(11)
    n_shape, m_shape, L = (3, 4), (6, 8), 2
    th = rng.uniform(0, 2 * np.pi, (L,) + m_shape)
    x = _cgauss(rng, n_shape)
    r = _cgauss(rng, m_shape)
    gz = _cgauss(rng, m_shape)
    gv = _cgauss(rng, n_shape)
    f_fwd = lambda t, xx: np.vdot(gz, oracle.forward(xx, t)).real
    f_adj = lambda t, rr: np.vdot(gv, oracle.adjoint(rr, t, n_shape)).real
    gx, gth = oracle.forward_vjp(x, th, gz)
    gr, gth2 = oracle.adjoint_vjp(r, th, n_shape, gv)
    eps = 1e-6
    for _ in range(6):
        d = rng.standard_normal(th.shape)
        fd = (f_fwd(th + eps * d, x) - f_fwd(th - eps * d, x)) / (2 * eps)
        assert abs(fd - np.sum(gth * d)) < 1e-7
        fd = (f_adj(th + eps * d, r) - f_adj(th - eps * d, r)) / (2 * eps)
        assert abs(fd - np.sum(gth2 * d)) < 1e-7
        dx = _cgauss(rng, n_shape)
        fd = (f_fwd(th, x + eps * dx) - f_fwd(th, x - eps * dx)) / (2 * eps)
        assert abs(fd - np.vdot(gx, dx).real) < 1e-7
        dr = _cgauss(rng, m_shape)
        fd = (f_adj(th, r + eps * dr) - f_adj(th, r - eps * dr)) / (2 * eps)
        assert abs(fd - np.vdot(gr, dr).real) < 1e-7


def test_unrolled_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(12)
    B, n_shape, m_shape, L, T = 2, (4, 4), (8, 8), 2, 3
    th = rng.uniform(0, 2 * np.pi, (L,) + m_shape)
    xs = _cgauss(rng, (B,) + n_shape)
    x0 = _cgauss(rng, (B,) + n_shape)
    loss, g = oracle.unrolled_gd_loss_grad(th, xs, x0, T, 0.2)
    assert abs(loss - oracle.unrolled_gd_loss(th, xs, x0, T, 0.2)) < 1e-12
    eps = 1e-6
    dirs = sr_inputs.fd_directions(5, 8, th.shape)
    for d in dirs:
        fd = (oracle.unrolled_gd_loss(th + eps * d, xs, x0, T, 0.2)
              - oracle.unrolled_gd_loss(th - eps * d, xs, x0, T, 0.2)) / (2 * eps)
        assert abs(fd - np.sum(g * d)) < 1e-6 * max(1.0, abs(fd))
    # a global phase on any D_l leaves every iterate unchanged: sum_j thetabar_lj = 0
    assert np.abs(g.reshape(L, -1).sum(axis=1)).max() < 1e-10
    # D_1 only multiplies zero-padded entries off the support
    mask = np.ones(m_shape, bool)
    mask[2:6, 2:6] = False
    assert np.abs(g[0][mask]).max() == 0.0


# ------------------------------------------------ undersampling (alpha <= 1)

def _brute_force_general(thetas, n_shape, m_shape):
    """S prod_l (F D_l) U on the grid max(n, m) per axis, with F from numpy.fft
    on identity columns (Kronecker product), U and S explicit 0/1 matrices
    built from centred offsets by index arithmetic."""
    grid = tuple(max(a, b) for a, b in zip(n_shape, m_shape))
    assert grid == thetas.shape[1:]
    g, n, m = int(np.prod(grid)), int(np.prod(n_shape)), int(np.prod(m_shape))
    F = np.ones((1, 1))
    for G in grid:
        F = np.kron(F, np.fft.fft(np.eye(G), axis=0, norm="ortho"))
    U = np.zeros((g, n))
    off = [(G - N) // 2 for N, G in zip(n_shape, grid)]
    for j in range(n):
        jj = np.unravel_index(j, n_shape)
        U[np.ravel_multi_index(tuple(o + a for o, a in zip(off, jj)), grid), j] = 1.0
    S = np.zeros((m, g))
    cut = [(G - M) // 2 for M, G in zip(m_shape, grid)]
    for i in range(m):
        ii = np.unravel_index(i, m_shape)
        S[i, np.ravel_multi_index(tuple(c + a for c, a in zip(cut, ii)), grid)] = 1.0
    A = U.astype(complex)
    for th in thetas:
        A = F @ (np.exp(1j * th.ravel())[:, None] * A)
    return S @ A


@pytest.mark.parametrize("n_shape,m_shape,L", [
    ((16,), (10,), 1), ((16,), (9,), 2), ((12,), (12,), 3),        # 1D trim, alpha = 1
    ((8, 6), (5, 4), 2), ((6, 8), (8, 5), 2), ((8, 8), (3, 8), 1),  # 2D trim, mixed pad/trim
])
def test_undersampled_operator_matches_brute_force(n_shape, m_shape, L):
    rng = np.random.default_rng(21)
    grid = tuple(max(a, b) for a, b in zip(n_shape, m_shape))
    th = rng.uniform(0, 2 * np.pi, (L,) + grid)
    A_bf = _brute_force_general(th, n_shape, m_shape)
    A_or = oracle.dense_matrix(th, n_shape, m_shape)
    assert A_or.shape == A_bf.shape
    assert np.abs(A_or - A_bf).max() < 1e-12
    r = _cgauss(rng, m_shape)
    assert np.abs(oracle.adjoint(r, th, n_shape).ravel() - A_bf.conj().T @ r.ravel()).max() < 1e-12
    # mean squared entry: 1 / (grid size)
    op = oracle.StructuredOperator(th, n_shape, m_shape)
    if all(M <= N for N, M in zip(n_shape, m_shape)) or all(M >= N for N, M in zip(n_shape, m_shape)):
        assert abs(np.mean(np.abs(A_bf) ** 2) - op.c) < 1e-12


@pytest.mark.parametrize("n_shape,m_shape,L", [((32,), (20,), 2), ((12, 10), (7, 10), 2), ((9, 9), (9, 9), 1)])
def test_undersampled_rows_are_orthonormal(n_shape, m_shape, L):
    """alpha <= 1: A A^H = I_m (the rows of a unitary matrix); Parseval on
    the range of A^H; adjoint identity."""
    rng = np.random.default_rng(22)
    th = rng.uniform(0, 2 * np.pi, (L,) + tuple(n_shape))
    A = oracle.dense_matrix(th, n_shape, m_shape)
    assert np.abs(A @ A.conj().T - np.eye(A.shape[0])).max() < 1e-12
    r = _cgauss(rng, m_shape)
    assert abs(np.linalg.norm(oracle.adjoint(r, th, n_shape)) - np.linalg.norm(r)) < 1e-12 * np.linalg.norm(r)
    x = _cgauss(rng, n_shape)
    lhs = np.vdot(oracle.forward(x, th, m_shape), r)
    rhs = np.vdot(x, oracle.adjoint(r, th, n_shape))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_undersampled_zero_phase_single_layer_is_trimmed_fft():
    rng = np.random.default_rng(23)
    x = _cgauss(rng, (10, 12))
    th = np.zeros((1, 10, 12))
    z = oracle.forward(x, th, (6, 7))
    ref = np.fft.fft2(x, norm="ortho")[2:8, 2:9]
    assert np.abs(z - ref).max() < 1e-12


def test_undersampled_spectral_iterates_match_eigendecomposition():
    rng = np.random.default_rng(24)
    n, m = 32, 24
    th = rng.uniform(0, 2 * np.pi, (2, n))
    op = oracle.StructuredOperator(th, (n,), (m,))
    A = _brute_force_general(th, (n,), (m,))
    y = np.abs(A @ _cgauss(rng, (n,))) ** 2
    lam = -1.0
    T = oracle.preprocess(y, lam)
    c = 1.0 / n
    M = A.conj().T @ (T[:, None] * A) / (m * c)
    v0 = _cgauss(rng, (n,))
    for K in (1, 6, 25):
        _, its = oracle.spectral_init(op, y, v0, K, lam, return_iterates=True)
        assert np.abs(its[-1] - _spectral_closed_form(M, lam, v0, K)).max() < 1e-10


def test_undersampled_gd_gradient_matches_finite_differences():
    rng = np.random.default_rng(25)
    th = rng.uniform(0, 2 * np.pi, (2, 8, 10))
    op = oracle.StructuredOperator(th, (8, 10), (6, 7))
    xs = _cgauss(rng, (8, 10))
    y = oracle.measurements(xs, th, (6, 7)) * rng.uniform(0.5, 1.5, (6, 7))
    x = _cgauss(rng, (8, 10))
    g = oracle.gd_gradient(op, y, x)
    for _ in range(6):
        d = _cgauss(rng, (8, 10))
        eps = 1e-6
        fd = (oracle.intensity_loss(op, y, x + eps * d) - oracle.intensity_loss(op, y, x - eps * d)) / (2 * eps)
        assert abs(fd - 4 * op.m * np.vdot(g, d).real) < 1e-6 * (abs(fd) + 1)


def test_undersampled_vjps_match_finite_differences():
    """Phase cotangents of z = A x and v = A^H r for a trimmed operator,
    against central differences of Re<w, A(theta) x> and Re<w, A(theta)^H r>."""
    rng = np.random.default_rng(26)
    n_shape, m_shape = (6, 8), (4, 8)
    th = rng.uniform(0, 2 * np.pi, (2,) + n_shape)
    x, r = _cgauss(rng, n_shape), _cgauss(rng, m_shape)
    gz, gv = _cgauss(rng, m_shape), _cgauss(rng, n_shape)
    _, gth_f = oracle.forward_vjp(x, th, gz)
    gr, gth_a = oracle.adjoint_vjp(r, th, n_shape, gv, m_shape)
    assert gr.shape == m_shape
    assert np.abs(gr - oracle.forward(gv, th, m_shape)).max() < 1e-12  # cotangent of r is A gv
    d = rng.standard_normal(th.shape)
    eps = 1e-6
    f = lambda t: np.vdot(gz, oracle.forward(x, t, m_shape)).real
    fd = (f(th + eps * d) - f(th - eps * d)) / (2 * eps)
    assert abs(fd - np.sum(gth_f * d)) < 1e-6 * (abs(fd) + 1)
    h = lambda t: np.vdot(gv, oracle.adjoint(r, t, n_shape)).real
    fd = (h(th + eps * d) - h(th - eps * d)) / (2 * eps)
    assert abs(fd - np.sum(gth_a * d)) < 1e-6 * (abs(fd) + 1)
