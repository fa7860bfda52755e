"""Seeded synthetic inputs for structured random phase retrieval.

This module only draws random numbers and shapes them into the inputs of the
method: signals x*, phase masks theta_l, power-iteration start vectors, GD start
points, dense i.i.d. sensing matrices and the Poisson photon-count noise model.
It holds none of the method's arithmetic (no DFT, no sensing operator, no
solver step), so that the FP64 oracle and the HIP library can both consume it
without sharing any computation.

All arrays are drawn in float64 on the host and cast once to the storage types
the library uses: complex64 for signals and matrices, float32 for phases and
intensities.  The reproducibility recipe: one master seed per workload,
``numpy.random.SeedSequence(seed).spawn`` gives independent streams for each
named input, in the fixed order of ``STREAMS``.
"""
from __future__ import annotations

import numpy as np

STREAMS = ("signal", "theta", "v0", "x0", "noise", "dense", "extra")

TWO_PI = 2.0 * np.pi


def streams(seed: int) -> dict:
    """Independent numpy Generators, one per named input, from one master seed."""
    children = np.random.SeedSequence(seed).spawn(len(STREAMS))
    return {name: np.random.default_rng(c) for name, c in zip(STREAMS, children)}


def complex_gaussian(rng, shape) -> np.ndarray:
    """i.i.d. CN(0,1) entries (real and imaginary parts N(0, 1/2)), complex64."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return ((re + 1j * im) / np.sqrt(2.0)).astype(np.complex64)


def phase_masks(rng, layers: int, m_shape) -> np.ndarray:
    """Random phases theta_l ~ U[0, 2 pi), shape (layers, *m_shape), float32.

    The paper draws the diagonal entries of every D_l with unit modulus and a
    phase uniform on [0, 2 pi) (section III).  Drawn in float64, cast once.
    """
    th = rng.uniform(0.0, TWO_PI, size=(layers,) + tuple(m_shape))
    th = th.astype(np.float32)
    # float32 rounding of values just below 2 pi can land on 2 pi; fold back.
    th[th >= np.float32(TWO_PI)] = 0.0
    return th


def smooth_field_image(rng, n_shape, sigma: float | None = None) -> np.ndarray:
    """Complex test image a * exp(i phi): amplitude a is a Gaussian-smoothed
    white-noise field min-max scaled to [0, 1]; phase phi ~ U[0, pi] per pixel.

    Stands in for the paper's phantom test image, which is not available here.
    sigma defaults to N/32 (N = first image side).
    """
    from scipy.ndimage import gaussian_filter

    n_shape = tuple(n_shape)
    if sigma is None:
        sigma = n_shape[0] / 32.0
    field = gaussian_filter(rng.standard_normal(n_shape), sigma=sigma, mode="wrap")
    lo, hi = field.min(), field.max()
    amp = (field - lo) / (hi - lo)
    phi = rng.uniform(0.0, np.pi, size=n_shape)
    return (amp * np.exp(1j * phi)).astype(np.complex64)


def phase_only_image(rng, n_shape) -> np.ndarray:
    """Unit-magnitude image whose phase is a smooth field mapped to [-pi/2, pi/2).

    Mirrors the paper's construction (grey levels in [0,1) mapped linearly to a
    phase in [-pi/2, pi/2) on a unit-modulus signal) with a synthetic image.
    """
    from scipy.ndimage import gaussian_filter

    n_shape = tuple(n_shape)
    field = gaussian_filter(rng.standard_normal(n_shape), sigma=n_shape[0] / 16.0, mode="wrap")
    g = (field - field.min()) / (field.max() - field.min() + 1e-300)
    g = np.minimum(g, np.nextafter(1.0, 0.0))
    return np.exp(1j * (np.pi * g - np.pi / 2.0)).astype(np.complex64)


def poisson_counts(rng, intensity, photons: float = 1000.0) -> np.ndarray:
    """Photon-count noise: Poisson(gamma * I) / gamma with gamma = photons / mean(I).

    ``intensity`` is a noiseless intensity array; the result is float32 with the
    same mean scale.  Both the oracle-side tests and the GPU-side benchmark pass
    in their own noiseless intensities.
    """
    inten = np.asarray(intensity, dtype=np.float64)
    gamma = photons / inten.mean()
    return (rng.poisson(gamma * inten) / gamma).astype(np.float32)


def scaled_start(rng, n_shape, target_sq_norm: float) -> np.ndarray:
    """A CN(0,1) start point rescaled so that its squared norm is target_sq_norm."""
    x0 = complex_gaussian(rng, n_shape).astype(np.complex128)
    x0 *= np.sqrt(target_sq_norm / np.vdot(x0, x0).real)
    return x0.astype(np.complex64)


# --------------------------------------------------------------------------
# Workload recipes.  Sizes follow the paper's setting (oversampling alpha =
# m/n by centred zero padding, L random-phase layers, 2D images); the exact
# sizes are the benchmark workloads of this library.
# --------------------------------------------------------------------------

def pad_shape(n_side: int, alpha: int) -> tuple:
    """Rectangular pad giving exactly m = alpha * n for square n_side^2 images."""
    if alpha == 2:
        return (2 * n_side, n_side)
    if alpha == 4:
        return (2 * n_side, 2 * n_side)
    if alpha == 8:
        return (4 * n_side, 2 * n_side)
    raise ValueError(f"unsupported alpha {alpha}")


def tiny_1d(seed: int = 0) -> dict:
    """x in C^64 i.i.d. CN(0,1), alpha=4 (m=256), L=2; plus a dense 256x64 CN(0,1) A."""
    s = streams(seed)
    n, m, L = 64, 256, 2
    return {
        "n_shape": (n,), "m_shape": (m,), "layers": L,
        "x_star": complex_gaussian(s["signal"], (n,)),
        "theta": phase_masks(s["theta"], L, (m,)),
        "v0": complex_gaussian(s["v0"], (n,)),
        "x0_random": complex_gaussian(s["x0"], (n,)),
        "dense_A": complex_gaussian(s["dense"], (m, n)),
        "lam": -1.0, "pi_iters": 50, "gd_iters": 200, "mu": 0.2,
    }


def image_2d(seed: int = 1, n_side: int = 256, layers: int = 2, photons: float = 1000.0) -> dict:
    """Smooth-amplitude, random-phase image n_side^2 padded to (2 n_side)^2 (alpha=4)."""
    s = streams(seed)
    n_shape = (n_side, n_side)
    m_shape = (2 * n_side, 2 * n_side)
    return {
        "n_shape": n_shape, "m_shape": m_shape, "layers": layers,
        "x_star": smooth_field_image(s["signal"], n_shape),
        "theta": phase_masks(s["theta"], layers, m_shape),
        "v0": complex_gaussian(s["v0"], n_shape),
        "noise_rng": s["noise"], "photons": photons,
        "lam": -1.0, "pi_iters": 100, "gd_iters": 500, "mu": 0.05,
    }


def large_2d(seed: int = 4) -> dict:
    """n = 1024^2 smooth image padded to 2048^2, L=3, Poisson noise at 1000 photons."""
    d = image_2d(seed, n_side=1024, layers=3)
    d["pi_iters"], d["gd_iters"] = 50, 100
    return d


def dense_batch(seed: int = 4, m: int = 16384, n: int = 4096, batch: int = 32) -> dict:
    """Dense i.i.d. CN(0,1) A (m x n, complex64) and a batch of CN(0,1) signals."""
    s = streams(seed + 1000)
    return {
        "dense_A": complex_gaussian(s["dense"], (m, n)),
        "X": complex_gaussian(s["signal"], (batch, n)),
        "R": complex_gaussian(s["extra"], (batch, m)),
    }


def batched_mixed(seed: int = 2, count: int = 256) -> list:
    """count independent problems: side N in {32,64,96,128}, alpha in {2,4,8},
    L in {1,2,3}, each uniform; x* i.i.d. CN(0,1); start x0 CN(0,1) rescaled to
    squared norm ||x*||^2 (equal to sum(y) for these operators); mu = 0.2."""
    s = streams(seed)
    pick = s["extra"]
    sides = pick.choice([32, 64, 96, 128], size=count)
    alphas = pick.choice([2, 4, 8], size=count)
    layers = pick.choice([1, 2, 3], size=count)
    probs = []
    for b in range(count):
        N, a, L = int(sides[b]), int(alphas[b]), int(layers[b])
        n_shape = (N, N)
        m_shape = pad_shape(N, a)
        xs = complex_gaussian(s["signal"], n_shape)
        sq = float(np.vdot(xs.astype(np.complex128), xs.astype(np.complex128)).real)
        probs.append({
            "n_shape": n_shape, "m_shape": m_shape, "layers": L,
            "x_star": xs,
            "theta": phase_masks(s["theta"], L, m_shape),
            "x0": scaled_start(s["x0"], n_shape, sq),
            "mu": 0.2,
        })
    return probs


def mask_design(seed: int = 3, batch: int = 64, n_side: int = 128, layers: int = 2) -> dict:
    """Shared masks theta (L, 2N, 2N) and a batch of CN(0,1) signals with θ-free
    start points (CN(0,1) rescaled to ||x*||^2)."""
    s = streams(seed)
    n_shape = (n_side, n_side)
    m_shape = (2 * n_side, 2 * n_side)
    xs = complex_gaussian(s["signal"], (batch,) + n_shape)
    x0 = np.stack([
        scaled_start(s["x0"], n_shape,
                     float(np.vdot(xs[b].astype(np.complex128), xs[b].astype(np.complex128)).real))
        for b in range(batch)])
    return {
        "n_shape": n_shape, "m_shape": m_shape, "layers": layers,
        "theta": phase_masks(s["theta"], layers, m_shape),
        "x_star": xs, "x0": x0, "steps": 20, "mu": 0.2,
    }


def fd_directions(seed: int, count: int, shape) -> np.ndarray:
    """Seeded N(0,1) directions for finite-difference checks, float64."""
    rng = streams(seed)["extra"]
    return rng.standard_normal((count,) + tuple(shape))
