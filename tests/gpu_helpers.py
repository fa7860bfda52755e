"""Helpers shared by the GPU tests: build plans, move arrays, compare."""
import numpy as np

import oracle


def to_dev(a, dev):
    import torch
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a).to(dev)


def to_host(t):
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def aligned(a, ref):
    return oracle.aligned_rel_error(a, ref)


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
