"""Helpers shared by the GPU tests: build plans, move arrays, compare.

Comparisons return one number that a test holds against its tolerance tol:
the relative L2 error ||a - b|| / ||b|| together with an element bound,

    err = max(||a - b|| / ||b||,  max_i |a_i - b_i| / (ELEM * rms(b))),

so that `err <= tol` means both ||a - b|| <= tol ||b|| and every element
within ELEM * tol of the reference's root-mean-square magnitude.  Rounding
errors of the FFT-based kernels spread evenly over the elements (their
maximum is a few times their RMS), while a few wrong elements in a large
grid hardly move the L2 norm but break the element bound.
"""
import numpy as np

import oracle

ELEM = 10.0


def to_dev(a, dev):
    import torch
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a).to(dev)


def to_host(t):
    return t.detach().cpu().numpy()


def _err(a, b):
    a = np.asarray(a, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    nb = np.linalg.norm(b)
    e = a - b
    rel = float(np.linalg.norm(e) / nb)
    if e.size == 0:
        return rel
    rms = nb / np.sqrt(b.size)
    return max(rel, float(np.max(np.abs(e)) / (ELEM * rms)))


def rel_l2(a, b):
    """Relative L2 error combined with the element bound (module docstring)."""
    return _err(a, b)


def rel_l2_only(a, b):
    """Plain relative L2 error ||a - b|| / ||b||."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def aligned(a, ref):
    """As rel_l2 after multiplying a by the global phase that best matches ref
    (the measurements fix the signal only up to a global phase)."""
    return _err(oracle.phase_align(np.asarray(a).reshape(np.shape(ref)), ref), ref)


def make_plan(problems, thetas, dev):
    """problems: list of (n_shape, m_shape, L); thetas: list of float32 arrays (L, *m)."""
    import paper_2409_05734_amd as srpr
    probs = [srpr.Problem(tuple(n), tuple(m), L) for n, m, L in problems]
    theta = np.concatenate([np.asarray(t, np.float32).ravel() for t in thetas])
    return srpr.Plan(probs, theta)


def random_problem(rng, n_shape, m_shape, L):
    th = rng.uniform(0, 2 * np.pi, (L,) + tuple(m_shape)).astype(np.float32)
    x = ((rng.standard_normal(n_shape) + 1j * rng.standard_normal(n_shape)) / np.sqrt(2)).astype(np.complex64)
    return th, x
