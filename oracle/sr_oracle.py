"""FP64 reference oracle for structured random phase retrieval.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, links or calls this module; only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark do.  It shares no code
with the HIP path: plain numpy in float64/complex128, with explicit O(N^2)
DFT matrices and no FFT, no blocking and no fusion.

Every function follows the paper (Hu, Tachella, Unser, Dong, "Structured Random
Model for Fast and Robust Phase Retrieval", arXiv 2409.05734) and cites the
section or equation it writes out.  Where the paper is silent or garbled the
reading taken is named in the docstring (the full list of readings is kept in
the project's design notes):

* R1  Eq. (2) prints diag(x^) acting on an m-vector; it is read as diag(A x^),
      i.e. the Wirtinger-flow gradient A^H((|Ax|^2 - y) . Ax); the constant 2
      and a 1/m go into the step size (gradient g = A^H r / m).
* R2  F is the unitary DFT, entries exp(-2 pi i jk/N)/sqrt(N) per axis.
* R3  M(T) = A^H diag(T(y)) A / (m c) with c the mean squared entry of A
      (1/m for the structured operator, 1 for dense CN(0,1)).
* R4  T is applied to y normalised by its mean, T(0) = lambda.
* R5  Power iterations are L2-normalised each step; the output is scaled to
      sqrt(sum(y) / (m c)).
* R6  D_1 acts first, right after the zero padding U.
* R7  Zero padding is centred: offset floor((M - N)/2) per axis.
* R14 Undersampling (alpha <= 1, A = S prod(F D_i)): the transforms run on
      the signal's grid and S keeps the centred measurement window, offset
      floor((N - M)/2) per axis; in general the grid is max(N, M) per axis,
      U pads into it and S trims it, and c = 1 / (grid size).
* R18 Noise-model loss (section II-B.1 says other losses follow from the
      noise statistics; none is written out): the negative Poisson
      log-likelihood of the intensities, sum |z|^2 - y log(|z|^2 + eps) with a
      guard eps > 0, whose Wirtinger gradient is A^H((1 - y/(|z|^2 + eps)) . z);
      as in R1 the gradient is taken as g = A^H r / m.

Parity pins for every function live in the CPU test-suite (library DFT,
brute-force dense products, closed forms, invariants, eigendecomposition,
finite differences); none of them re-types these formulas.
"""
from __future__ import annotations

import numpy as np

# ----------------------------------------------------------------------------
# Building blocks: DFT matrix, padding geometry, phase diagonals
# ----------------------------------------------------------------------------

_DFT_CACHE: dict = {}


def dft_matrix(N: int) -> np.ndarray:
    """Unitary DFT matrix F_N[j, k] = exp(-2 pi i j k / N) / sqrt(N).

    Section III calls F "the FFT matrix"; reading R2 fixes the unitary scale
    and the negative-exponent sign.  The exponent jk is reduced mod N in exact
    integer arithmetic before the float64 evaluation.
    """
    F = _DFT_CACHE.get(N)
    if F is None:
        j = np.arange(N, dtype=np.int64)
        jk = np.outer(j, j) % N
        F = np.exp(-2j * np.pi * jk / N) / np.sqrt(N)
        _DFT_CACHE[N] = F
    return F


def pad_offsets(n_shape, m_shape) -> tuple:
    """Centred zero-padding offsets floor((M_k - N_k)/2) (reading R7, section III)."""
    return tuple((M - N) // 2 for N, M in zip(n_shape, m_shape))


def zero_pad(x: np.ndarray, m_shape) -> np.ndarray:
    """U: embed the n-signal in an m-array of zeros (section III, oversampling)."""
    off = pad_offsets(x.shape, m_shape)
    X = np.zeros(m_shape, dtype=np.complex128)
    X[tuple(slice(o, o + N) for o, N in zip(off, x.shape))] = x
    return X


def crop(X: np.ndarray, n_shape) -> np.ndarray:
    """U^H: keep the support window of the padding (adjoint of zero_pad)."""
    off = pad_offsets(n_shape, X.shape)
    return X[tuple(slice(o, o + N) for o, N in zip(off, n_shape))].copy()


def apply_dft(X: np.ndarray, inverse: bool = False) -> np.ndarray:
    """Separable unitary DFT along every axis: F_M1 X F_M2^T in 2D, F_M X in 1D.

    inverse=True applies F^H.  Explicit matrices, one matrix product per axis.
    """
    Y = np.asarray(X, dtype=np.complex128)
    for ax in range(Y.ndim):
        F = dft_matrix(Y.shape[ax])
        if inverse:
            F = F.conj()  # F is symmetric, so F^H = conj(F)
        Y = np.moveaxis(np.tensordot(F, np.moveaxis(Y, ax, 0), axes=(1, 0)), 0, ax)
    return Y


def phase_diagonal(theta_l: np.ndarray) -> np.ndarray:
    """Entries of D_l: unit modulus, phase theta_l (section III)."""
    return np.exp(1j * np.asarray(theta_l, dtype=np.float64))


# ----------------------------------------------------------------------------
# The structured sensing operator, Eq. (5)
# ----------------------------------------------------------------------------

def forward(x: np.ndarray, thetas: np.ndarray, m_shape=None) -> np.ndarray:
    """A x = S F D_L ... F D_1 U x   (Eq. (5); readings R6, R7, R14).

    x: complex signal of shape n_shape; thetas: (L, *grid) phases on the
    transform grid (max(n, m) per axis).  U pads x into the grid, S keeps the
    centred m_shape window (default: the whole grid, i.e. alpha >= 1).
    Returns z = A x of shape m_shape (complex128).
    """
    thetas = np.asarray(thetas, dtype=np.float64)
    grid = thetas.shape[1:]
    Z = zero_pad(np.asarray(x, dtype=np.complex128), grid)
    for th in thetas:
        Z = apply_dft(phase_diagonal(th) * Z)
    return Z if m_shape is None else crop(Z, tuple(m_shape))


def adjoint(r: np.ndarray, thetas: np.ndarray, n_shape) -> np.ndarray:
    """A^H r = U^H D_1^* F^H ... D_L^* F^H S^H r   (adjoint of Eq. (5)).

    r has the measurement shape; S^H embeds it in the grid with zeros."""
    thetas = np.asarray(thetas, dtype=np.float64)
    V = zero_pad(np.asarray(r, dtype=np.complex128), thetas.shape[1:])
    for th in thetas[::-1]:
        V = np.conj(phase_diagonal(th)) * apply_dft(V, inverse=True)
    return crop(V, n_shape)


def dense_matrix(thetas: np.ndarray, n_shape, m_shape=None) -> np.ndarray:
    """Explicit m x n matrix of the structured operator, one column per unit
    vector e_j (row-major vectorisation).  Tiny sizes only (brute force)."""
    thetas = np.asarray(thetas, dtype=np.float64)
    n = int(np.prod(n_shape))
    cols = []
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        cols.append(forward(e.reshape(n_shape), thetas, m_shape).ravel())
    return np.stack(cols, axis=1)


def measurements(x: np.ndarray, thetas: np.ndarray, m_shape=None) -> np.ndarray:
    """Noiseless intensities y = |A x|^2   (Eq. (1))."""
    return np.abs(forward(x, thetas, m_shape)) ** 2


# ----------------------------------------------------------------------------
# Operator wrappers used by the solvers: structured and dense i.i.d.
# ----------------------------------------------------------------------------

class StructuredOperator:
    """A of Eq. (5) with its adjoint; m = number of measurements, mean squared
    entry c = 1/g with g the grid size (reading R14): the rows (alpha <= 1) or
    columns (alpha >= 1) of A are orthonormal."""

    def __init__(self, thetas, n_shape, m_shape=None):
        self.thetas = np.asarray(thetas, dtype=np.float64)
        self.n_shape = tuple(n_shape)
        self.grid_shape = tuple(self.thetas.shape[1:])
        self.m_shape = self.grid_shape if m_shape is None else tuple(m_shape)
        self.m = int(np.prod(self.m_shape))
        self.n = int(np.prod(self.n_shape))
        self.c = 1.0 / int(np.prod(self.grid_shape))

    def A(self, x):
        return forward(x, self.thetas, self.m_shape)

    def AH(self, r):
        return adjoint(r, self.thetas, self.n_shape)


class DenseOperator:
    """i.i.d. CN(0,1) sensing matrix (section II-A random model); c = 1."""

    def __init__(self, A):
        self.M = np.asarray(A, dtype=np.complex128)
        self.m, self.n = self.M.shape
        self.n_shape = (self.n,)
        self.m_shape = (self.m,)
        self.c = 1.0

    def A(self, x):
        return self.M @ np.asarray(x, dtype=np.complex128).ravel()

    def AH(self, r):
        return self.M.conj().T @ np.asarray(r, dtype=np.complex128).ravel()


# ----------------------------------------------------------------------------
# Solvers: spectral initialisation (Eq. (3), (4)) and gradient descent (Eq. (2))
# ----------------------------------------------------------------------------

def preprocess(y: np.ndarray, lam: float) -> np.ndarray:
    """T(y~) = max(1 - 1/y~, lambda) with y~ = y / mean(y), and T(0) = lambda.

    The preprocessing of section II-B.2 (optimal for the noiseless i.i.d. model,
    lambda < 0); readings R4 (normalisation by the mean) and T(0) = lambda.
    """
    y = np.asarray(y, dtype=np.float64)
    yt = y / y.mean()
    T = np.full(y.shape, float(lam))
    pos = yt > 0
    T[pos] = np.maximum(1.0 - 1.0 / yt[pos], lam)
    return T


def spectral_step(op, T: np.ndarray, v: np.ndarray, lam: float) -> np.ndarray:
    """One shifted power-iteration product  M v - 2 lambda v   (Eq. (4)),
    with M = A^H diag(T) A / (m c)   (Eq. (3), reading R3)."""
    Mv = op.AH(T * op.A(v)) / (op.m * op.c)
    return Mv - 2.0 * lam * v


def spectral_init(op, y, v0, iters: int, lam: float, return_iterates: bool = False):
    """Spectral initialisation by shifted power iteration (Eq. (3)-(4), R5).

    v_0 = v0/||v0||; v_{k+1} = B v_k / ||B v_k|| with B = M - 2 lambda I;
    output x0 = sqrt(sum(y) / (m c)) * v_K.
    """
    T = preprocess(y, lam)
    v = np.asarray(v0, dtype=np.complex128)
    v = v / np.linalg.norm(v)
    its = []
    for _ in range(iters):
        u = spectral_step(op, T, v, lam)
        v = u / np.linalg.norm(u)
        if return_iterates:
            its.append(v.copy())
    scale = np.sqrt(np.sum(np.asarray(y, dtype=np.float64)) / (op.m * op.c))
    out = scale * v
    return (out, its) if return_iterates else out


def gd_gradient(op, y, x) -> np.ndarray:
    """g = A^H((|Ax|^2 - y) . Ax) / m   (Eq. (2) with reading R1)."""
    z = op.A(x)
    r = (np.abs(z) ** 2 - np.asarray(y, dtype=np.float64)) * z
    return op.AH(r) / op.m


def intensity_loss(op, y, x) -> float:
    """L(x) = || |Ax|^2 - y ||^2, the l2 intensity loss of section II-B.1."""
    z = op.A(x)
    return float(np.sum((np.abs(z) ** 2 - np.asarray(y, dtype=np.float64)) ** 2))


def poisson_gradient(op, y, x, eps: float) -> np.ndarray:
    """g = A^H((1 - y/(|Ax|^2 + eps)) . Ax) / m: the Wirtinger gradient of the
    Poisson negative log-likelihood (reading R18), scaled like gd_gradient."""
    z = op.A(x)
    r = (1.0 - np.asarray(y, dtype=np.float64) / (np.abs(z) ** 2 + eps)) * z
    return op.AH(r) / op.m


def poisson_loss(op, y, x, eps: float) -> float:
    """sum_i |z_i|^2 - y_i log(|z_i|^2 + eps), z = Ax (reading R18)."""
    z2 = np.abs(op.A(x)) ** 2
    return float(np.sum(z2 - np.asarray(y, dtype=np.float64) * np.log(z2 + eps)))


def gd_solve(op, y, x0, iters: int, eta: float, return_iterates: bool = False,
             return_loss: bool = False, loss: str = "l2", eps: float = 0.0):
    """Fixed-step gradient descent x <- x - eta g(x) on the intensity loss (Eq. (2)),
    or with loss="poisson" on the Poisson negative log-likelihood (reading R18,
    guard eps > 0).

    eta is the raw multiplier of g; no early stopping (fixed iteration count).
    The optional loss trace records the loss at x_t before each step.
    """
    if loss not in ("l2", "poisson"):
        raise ValueError(f"unknown loss {loss!r}")
    if loss == "poisson" and not eps > 0:
        raise ValueError("the Poisson loss needs eps > 0")
    grad = gd_gradient if loss == "l2" else (lambda o, yy, xx: poisson_gradient(o, yy, xx, eps))
    value = intensity_loss if loss == "l2" else (lambda o, yy, xx: poisson_loss(o, yy, xx, eps))
    x = np.asarray(x0, dtype=np.complex128).copy()
    its, losses = [], []
    for _ in range(iters):
        if return_loss:
            losses.append(value(op, y, x))
        x = x - eta * grad(op, y, x)
        if return_iterates:
            its.append(x.copy())
    out = [x]
    if return_iterates:
        out.append(its)
    if return_loss:
        out.append(np.array(losses))
    return out[0] if len(out) == 1 else tuple(out)


def default_step(op, y, mu: float = 0.2) -> float:
    """Dimensionless step mu turned into the raw multiplier eta = mu / (c * mean(y))."""
    return mu / (op.c * float(np.mean(np.asarray(y, dtype=np.float64))))


# ----------------------------------------------------------------------------
# Metrics (Eq. (6)) and phase alignment
# ----------------------------------------------------------------------------

def cosine_similarity(xhat, xstar) -> float:
    """|<xhat, x*>| / (||xhat|| ||x*||) with <a, b> = a^H b   (Eq. (6))."""
    a = np.asarray(xhat, dtype=np.complex128).ravel()
    b = np.asarray(xstar, dtype=np.complex128).ravel()
    return float(abs(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b)))


def phase_align(xhat, xref) -> np.ndarray:
    """Multiply xhat by the global phase exp(-i arg(xref^H xhat)) that best
    matches xref (the measurements fix x only up to a global phase)."""
    a = np.asarray(xhat, dtype=np.complex128)
    s = np.vdot(np.asarray(xref, dtype=np.complex128).ravel(), a.ravel())
    return a * np.exp(-1j * np.angle(s))


def aligned_rel_error(xhat, xref) -> float:
    """||align(xhat) - xref|| / ||xref||."""
    a = phase_align(xhat, xref)
    r = np.asarray(xref, dtype=np.complex128)
    return float(np.linalg.norm(a - r) / np.linalg.norm(r))


def rel_l2(a, b) -> float:
    """||a - b|| / ||b||."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ----------------------------------------------------------------------------
# Reverse-mode derivatives for mask design (gradients in PyTorch's convention:
# for a real loss l and complex w, grad w = dl/dRe(w) + i dl/dIm(w)).
# ----------------------------------------------------------------------------

def forward_vjp(x, thetas, gz):
    """Cotangents of z = A x: returns (gx, gtheta) for cotangent gz of z.

    Intermediates: w_0 = U x, u_l = D_l w_{l-1}, w_l = F u_l (Eq. (5)).
    Reverse: ubar_l = F^H wbar_l, thetabar_l = Im(ubar_l * conj(u_l)),
    wbar_{l-1} = D_l^* ubar_l, gx = U^H wbar_0.
    """
    thetas = np.asarray(thetas, dtype=np.float64)
    n_shape = np.shape(x)
    w = zero_pad(np.asarray(x, dtype=np.complex128), thetas.shape[1:])
    us = []
    for th in thetas:
        u = phase_diagonal(th) * w
        us.append(u)
        w = apply_dft(u)
    wbar = zero_pad(np.asarray(gz, dtype=np.complex128), thetas.shape[1:])  # S^H gz
    gth = np.zeros_like(thetas)
    for l in range(len(thetas) - 1, -1, -1):
        ubar = apply_dft(wbar, inverse=True)
        gth[l] = np.imag(ubar * np.conj(us[l]))
        wbar = np.conj(phase_diagonal(thetas[l])) * ubar
    return crop(wbar, n_shape), gth


def adjoint_vjp(r, thetas, n_shape, gv, m_shape=None):
    """Cotangents of v = A^H r: returns (gr, gtheta) for cotangent gv of v.

    Intermediates: s_L = r, t_l = F^H s_l, q_l = D_l^* t_l, s_{l-1} = q_l,
    v = U^H s_0.  Reverse: qbar_l = sbar_{l-1} (sbar_0 = U gv),
    thetabar_l = Im(conj(qbar_l) * q_l), sbar_l = F D_l qbar_l, gr = sbar_L.
    """
    thetas = np.asarray(thetas, dtype=np.float64)
    s = zero_pad(np.asarray(r, dtype=np.complex128), thetas.shape[1:])  # S^H r
    qs = [None] * len(thetas)
    for l in range(len(thetas) - 1, -1, -1):
        q = np.conj(phase_diagonal(thetas[l])) * apply_dft(s, inverse=True)
        qs[l] = q
        s = q
    sbar = zero_pad(np.asarray(gv, dtype=np.complex128), thetas.shape[1:])
    gth = np.zeros_like(thetas)
    for l in range(len(thetas)):
        gth[l] = np.imag(np.conj(sbar) * qs[l])
        sbar = apply_dft(phase_diagonal(thetas[l]) * sbar)
    return (sbar if m_shape is None else crop(sbar, tuple(m_shape))), gth


def unrolled_gd_loss(thetas, x_star, x0, steps: int, mu: float) -> float:
    """Mask-design objective: mean over the batch of the phase-aligned relative
    squared error after `steps` unrolled GD steps (Eq. (2)) on y_b = |A x*_b|^2.

    l_b = (||x_T||^2 + ||x*||^2 - 2 |x_T^H x*|) / ||x*||^2.  The step size is
    eta_b = mu m^2 / ||x*_b||^2, i.e. mu / (c mean(y_b)) with mean(y_b) =
    ||x*_b||^2 / m, written through ||x*_b|| so that it does not depend on theta.
    """
    thetas = np.asarray(thetas, dtype=np.float64)
    B = x_star.shape[0]
    n_shape = x_star.shape[1:]
    op = StructuredOperator(thetas, n_shape)
    total = 0.0
    for b in range(B):
        xs = np.asarray(x_star[b], dtype=np.complex128)
        ns2 = float(np.vdot(xs, xs).real)
        y = np.abs(op.A(xs)) ** 2
        eta = mu * op.m ** 2 / ns2
        x = np.asarray(x0[b], dtype=np.complex128)
        for _ in range(steps):
            x = x - eta * gd_gradient(op, y, x)
        total += (np.vdot(x, x).real + ns2 - 2.0 * abs(np.vdot(x, xs))) / ns2
    return total / B


def unrolled_gd_loss_grad(thetas, x_star, x0, steps: int, mu: float):
    """Loss of unrolled_gd_loss and its gradient with respect to theta, by
    reverse-mode differentiation through every GD step, recomputing iterates.

    Step t: z = A x, r = (|z|^2 - y) z, v = A^H r, x+ = x - (eta/m) v.  Reverse
    with xbar+ given:  vbar = -(eta/m) xbar+; (rbar, theta) from adjoint_vjp;
    zbar = (2|z|^2 - y) rbar + z^2 conj(rbar); ybar += -Re(conj(rbar) z);
    (A^H zbar, theta) from forward_vjp; xbar = xbar+ + A^H zbar.
    The measurements y = |A x*|^2 contribute forward_vjp(x*, 2 ybar z*).
    """
    thetas = np.asarray(thetas, dtype=np.float64)
    B = x_star.shape[0]
    n_shape = x_star.shape[1:]
    op = StructuredOperator(thetas, n_shape)
    m = op.m
    gth = np.zeros_like(thetas)
    total = 0.0
    for b in range(B):
        xs = np.asarray(x_star[b], dtype=np.complex128)
        ns2 = float(np.vdot(xs, xs).real)
        zs = op.A(xs)
        y = np.abs(zs) ** 2
        eta = mu * m ** 2 / ns2
        xs_t = [np.asarray(x0[b], dtype=np.complex128)]
        for _ in range(steps):
            xs_t.append(xs_t[-1] - eta * gd_gradient(op, y, xs_t[-1]))
        xT = xs_t[-1]
        s = np.vdot(xT, xs)
        total += (np.vdot(xT, xT).real + ns2 - 2.0 * abs(s)) / ns2
        xbar = (2.0 * xT - 2.0 * np.exp(-1j * np.angle(s)) * xs) / ns2 / B
        ybar = np.zeros(op.m_shape)
        for t in range(steps - 1, -1, -1):
            x = xs_t[t]
            z = op.A(x)
            r = (np.abs(z) ** 2 - y) * z
            vbar = -(eta / m) * xbar
            rbar, g1 = adjoint_vjp(r, thetas, n_shape, vbar)
            zbar = (2.0 * np.abs(z) ** 2 - y) * rbar + z ** 2 * np.conj(rbar)
            ybar += -np.real(np.conj(rbar) * z)
            gx, g2 = forward_vjp(x, thetas, zbar)
            gth += g1 + g2
            xbar = xbar + gx
        _, g3 = forward_vjp(xs, thetas, 2.0 * ybar * zs)
        gth += g3
    return total / B, gth
