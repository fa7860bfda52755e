"""CPU pins of two oracle results that the other pins do not reach.

1. The mask-design objective (`oracle.unrolled_gd_loss`): its value is
   rebuilt from separately pinned pieces -- the GD solver (section II-B.1,
   Eq. (2); pinned by finite differences and recovery), the recommended step
   `default_step` computed from the measurements themselves, and the
   phase-aligned error `aligned_rel_error` (the global-phase ambiguity of
   section II-B; pinned against the cosine of Eq. (6)).  A dropped term, a
   wrong exponent in the step or a missing modulus in the loss shows up here.
   Closed forms: zero steps give the aligned error of the start; the truth
   (up to any global phase) is a fixed point with loss zero.

2. Reading R13 (what "1e-4 on iterates over the first 50 GD steps" can mean
   on a trajectory that amplifies rounding): on the random-start case
   64 x 64 -> 128 x 64, L = 1, mu = 0.2, a complex64 implementation of the
   same GD step (numpy's single-precision FFT, independent of the oracle's
   explicit DFT matrices) reproduces every single oracle step to 2e-5, yet its
   50-step trajectory leaves the float64 one by more than 1e-4; the float64
   trajectory itself separates from a copy started 1e-7 away by more than
   1e-4.  So no float32 implementation can meet a whole-trajectory bar there,
   and the step-by-step comparison is the meaningful one.

3. The reverse-mode mask gradient at the mask-design workload's full shapes
   against 32 stored FP64 central differences of the objective (written by
   tests/golden/make_mask_fd.py from the oracle alone).
"""
import numpy as np
import pytest

import oracle
import sr_inputs
from fixtures import read_mask_fd


def _cg(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ------------------------------------------------------ mask-design objective

@pytest.mark.parametrize("n_shape,m_shape,L,T,mu", [
    ((4, 4), (8, 8), 2, 3, 0.2),
    ((6, 5), (12, 10), 3, 5, 0.1),
    ((8,), (32,), 2, 4, 0.2),
])
def test_unrolled_objective_is_mean_aligned_error_of_gd(n_shape, m_shape, L, T, mu):
    rng = np.random.default_rng(31 + L + T)
    B = 3
    th = rng.uniform(0, 2 * np.pi, (L,) + m_shape)
    xs = _cg(rng, (B,) + n_shape)
    x0 = _cg(rng, (B,) + n_shape)
    op = oracle.StructuredOperator(th, n_shape)
    errs = []
    for b in range(B):
        y = oracle.measurements(xs[b], th)
        eta = oracle.default_step(op, y, mu)
        # the objective's step mu m^2/||x*||^2 is the recommended step, because
        # mean(y) = ||x*||^2 / m when A has orthonormal columns
        assert abs(eta - mu * op.m ** 2 / np.vdot(xs[b], xs[b]).real) <= 1e-12 * eta
        xT = oracle.gd_solve(op, y, x0[b], T, eta)
        errs.append(oracle.aligned_rel_error(xT, xs[b]) ** 2)
    want = float(np.mean(errs))
    got = oracle.unrolled_gd_loss(th, xs, x0, T, mu)
    assert abs(got - want) <= 1e-12 * max(1.0, want)
    # the reverse-mode routine reports the same value
    assert abs(oracle.unrolled_gd_loss_grad(th, xs, x0, T, mu)[0] - want) <= 1e-12 * max(1.0, want)


def test_unrolled_objective_closed_forms():
    rng = np.random.default_rng(5)
    n_shape, m_shape, L = (4, 4), (8, 8), 2
    th = rng.uniform(0, 2 * np.pi, (L,) + m_shape)
    xs = _cg(rng, (2,) + n_shape)
    x0 = _cg(rng, (2,) + n_shape)
    # no steps: the squared aligned error of the start, written out by hand
    want = 0.0
    for b in range(2):
        s = abs(np.vdot(x0[b], xs[b]))
        ns = np.vdot(xs[b], xs[b]).real
        want += (np.vdot(x0[b], x0[b]).real + ns - 2 * s) / ns
    assert abs(oracle.unrolled_gd_loss(th, xs, x0, 0, 0.2) - want / 2) < 1e-12
    # the truth under any global phase is a fixed point of GD: loss zero
    phased = xs * np.exp(1j * np.array([0.7, -2.1]))[:, None, None]
    assert oracle.unrolled_gd_loss(th, xs, phased, 6, 0.2) < 1e-20
    # a positive multiple c x* has loss (1 - c)^2 before any step
    assert abs(oracle.unrolled_gd_loss(th, xs, 0.5 * xs, 0, 0.2) - 0.25) < 1e-12


# --------------------------------------------------------------- reading R13

def _gd_step_c64(x, y, thetas, m_shape, eta):
    """One GD step x - eta A^H((|Ax|^2 - y) Ax)/m entirely in complex64, with
    numpy's single-precision FFTs (unitary) on the zero-padded grid."""
    c64 = np.complex64
    n_shape = x.shape
    off = [(M - N) // 2 for N, M in zip(n_shape, m_shape)]
    win = tuple(slice(o, o + N) for o, N in zip(off, n_shape))
    d = [np.exp(1j * t.astype(np.float32)).astype(c64) for t in thetas]
    Z = np.zeros(m_shape, c64)
    Z[win] = x
    for dl in d:
        Z = np.fft.fft2(dl * Z, norm="ortho").astype(c64)
    R = ((np.abs(Z) ** 2 - y).astype(np.float32) * Z).astype(c64)
    for dl in d[::-1]:
        R = (np.conj(dl) * np.fft.ifft2(R, norm="ortho")).astype(c64)
    m = np.float32(np.prod(m_shape))
    return (x - np.float32(eta) * (R[win] / m)).astype(c64)


def test_random_start_trajectory_amplifies_rounding():
    rng = np.random.default_rng(2024)
    n_shape, m_shape, L, steps = (64, 64), (128, 64), 1, 50
    th = sr_inputs.phase_masks(rng, L, m_shape)
    xs = sr_inputs.complex_gaussian(rng, n_shape)
    x0 = sr_inputs.complex_gaussian(rng, n_shape)
    op = oracle.StructuredOperator(th, n_shape)
    y = oracle.measurements(xs, th).astype(np.float32)
    x0 = (x0 * np.sqrt(np.sum(y, dtype=np.float64) / np.vdot(x0, x0).real)).astype(np.complex64)
    eta = oracle.default_step(op, y, 0.2)
    _, its = oracle.gd_solve(op, y, x0, steps, eta, return_iterates=True)
    traj = [np.asarray(x0, np.complex128)] + its

    # single steps: complex64 arithmetic reproduces the oracle's step to 2e-5
    one_step = max(oracle.rel_l2(_gd_step_c64(traj[k].astype(np.complex64), y, th, m_shape, eta), traj[k + 1])
                   for k in range(steps))
    assert one_step <= 2e-5, one_step

    # whole trajectory in complex64: leaves the float64 one by more than 1e-4
    x = np.asarray(x0, np.complex64)
    for _ in range(steps):
        x = _gd_step_c64(x, y, th, m_shape, eta)
    drift32 = oracle.aligned_rel_error(x, traj[-1])
    assert drift32 > 1e-4, drift32

    # the float64 trajectory alone: a start 1e-7 away ends more than 1e-4 away
    pert = x0 + 1e-7 * np.linalg.norm(x0) / np.sqrt(x0.size) * _cg(rng, n_shape) / np.sqrt(2)
    xp = oracle.gd_solve(op, y, pert, steps, eta)
    drift64 = oracle.aligned_rel_error(xp, traj[-1])
    assert drift64 > 1e-4, drift64


# ------------------------------------- mask-design gradient at full shapes

def test_mask_gradient_matches_stored_central_differences():
    """The oracle's reverse-mode mask gradient on the mask-design workload's
    shapes (128^2 -> 256^2, L = 2, 20 unrolled steps, first 2 problems) against
    32 FP64 central differences, eps = 1e-6."""
    d, loss_fd, fd, dirs = read_mask_fd()
    th = d["theta"].astype(np.float64)
    loss, g = oracle.unrolled_gd_loss_grad(th, d["x_star"][:2], d["x0"][:2], d["steps"], d["mu"])
    assert abs(loss - loss_fd) <= 1e-12 * abs(loss_fd)
    dd = (dirs * g[None]).reshape(len(fd), -1).sum(axis=1)
    assert np.max(np.abs(dd - fd)) <= 1e-8 + 1e-6 * np.max(np.abs(fd)), np.max(np.abs(dd - fd))
