"""GPU parity of the structured operator A and its adjoint (section III,
Eq. (5)) against the FP64 oracle: relative L2 error <= 2e-5 per application,
element by element, over 1D and 2D shapes that span several tiles, ragged
support windows, rectangular pads, one to four layers and every FFT length
the library supports; plus unitarity properties at the largest size."""
import numpy as np
import pytest

import oracle
from gpu_helpers import make_plan, random_problem, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_OP = 2e-5

SHAPES = [
    # (n_shape, m_shape, L)
    ((64,), (256,), 2),          # tiny 1D workload
    ((8,), (32,), 1),
    ((40,), (96,), 3),
    ((100,), (384,), 2),
    ((333,), (1024,), 2),
    ((1000,), (4096,), 1),       # largest 1D
    ((16, 16), (32, 32), 2),
    ((20, 12), (32, 64), 1),     # ragged offsets, rectangular
    ((48, 40), (96, 64), 3),
    ((64, 64), (128, 64), 2),    # alpha = 2 pad (no padding on axis 1)
    ((100, 70), (192, 128), 2),
    ((90, 160), (384, 192), 3),
    ((128, 128), (256, 256), 4),
    ((256, 256), (512, 512), 2),  # the 2D image workload
    ((300, 500), (768, 1024), 1),
    ((33, 17), (2048, 32), 2),   # longest column FFT
    ((17, 33), (32, 2048), 2),   # longest row FFT
]


@pytest.mark.parametrize("n_shape,m_shape,L", SHAPES)
def test_forward_adjoint_parity(gpu, n_shape, m_shape, L):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(hash((n_shape, m_shape, L)) % 2**32)
    th, x = random_problem(rng, n_shape, m_shape, L)
    r = ((rng.standard_normal(m_shape) + 1j * rng.standard_normal(m_shape)) / np.sqrt(2)).astype(np.complex64)
    plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
    xd = to_dev(x.ravel(), gpu)
    zd = torch.empty(int(np.prod(m_shape)), dtype=torch.complex64, device=gpu)
    yd = torch.empty(int(np.prod(m_shape)), dtype=torch.float32, device=gpu)
    srpr.sr_forward(plan, xd, zd, yd)
    rd = to_dev(r.ravel(), gpu)
    vd = torch.empty(int(np.prod(n_shape)), dtype=torch.complex64, device=gpu)
    srpr.sr_adjoint(plan, rd, vd)
    torch.cuda.synchronize()
    z_ref = oracle.forward(x, th)
    v_ref = oracle.adjoint(r, th, n_shape)
    assert rel_l2(to_host(zd).reshape(m_shape), z_ref) <= TOL_OP
    y_ref = np.abs(z_ref) ** 2
    assert rel_l2(to_host(yd).reshape(m_shape), y_ref) <= 2 * TOL_OP
    assert rel_l2(to_host(vd).reshape(n_shape), v_ref) <= TOL_OP
    # y only / z only
    y2 = torch.empty_like(yd)
    srpr.sr_forward(plan, xd, None, y2)
    z2 = torch.empty_like(zd)
    srpr.sr_forward(plan, xd, z2, None)
    torch.cuda.synchronize()
    assert torch.equal(y2, yd) and torch.equal(z2, zd)


def test_multi_problem_plan_matches_each_problem(gpu):
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(3)
    specs = [((64,), (256,), 2), ((16, 16), (32, 32), 2), ((48, 40), (96, 64), 3), ((32, 32), (64, 32), 1)]
    data = [random_problem(rng, *s) for s in specs]
    plan = make_plan(specs, [d[0] for d in data], gpu)
    x = np.concatenate([d[1].ravel() for d in data])
    zd = torch.empty(plan.m_total, dtype=torch.complex64, device=gpu)
    srpr.sr_forward(plan, to_dev(x, gpu), zd, None)
    torch.cuda.synchronize()
    z = to_host(zd)
    for i, (s, d) in enumerate(zip(specs, data)):
        zi = z[plan.y_off[i]:plan.y_off[i + 1]].reshape(s[1])
        assert rel_l2(zi, oracle.forward(d[1], d[0])) <= TOL_OP


def test_shared_phase_blocks(gpu):
    """Two problems pointing at one set of phases give identical operators."""
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(4)
    th, x1 = random_problem(rng, (24, 24), (64, 64), 2)
    _, x2 = random_problem(rng, (24, 24), (64, 64), 2)
    probs = [srpr.Problem((24, 24), (64, 64), 2, theta_offset=0), srpr.Problem((24, 24), (64, 64), 2, theta_offset=0)]
    plan = srpr.Plan(probs, th)
    zd = torch.empty(plan.m_total, dtype=torch.complex64, device=gpu)
    srpr.sr_forward(plan, to_dev(np.concatenate([x1.ravel(), x2.ravel()]), gpu), zd, None)
    torch.cuda.synchronize()
    z = to_host(zd)
    assert rel_l2(z[:4096].reshape(64, 64), oracle.forward(x1, th)) <= TOL_OP
    assert rel_l2(z[4096:].reshape(64, 64), oracle.forward(x2, th)) <= TOL_OP


def test_large_grid_properties(gpu):
    """2048^2 grid, L = 3 (the large workload): properties that hold at any
    size, computed in fp32 on the GPU: ||Ax|| = ||x||, A^H A x = x, and the
    adjoint identity <Ax, r> = <x, A^H r>."""
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(5)
    n_shape, m_shape, L = (1024, 1024), (2048, 2048), 3
    th = rng.uniform(0, 2 * np.pi, (L,) + m_shape).astype(np.float32)
    plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
    x = torch.randn(1024 * 1024, dtype=torch.complex64, device=gpu)
    r = torch.randn(2048 * 2048, dtype=torch.complex64, device=gpu)
    z = torch.empty(2048 * 2048, dtype=torch.complex64, device=gpu)
    v = torch.empty(1024 * 1024, dtype=torch.complex64, device=gpu)
    w = torch.empty_like(v)
    srpr.sr_forward(plan, x, z, None)
    srpr.sr_adjoint(plan, z, v)
    srpr.sr_adjoint(plan, r, w)
    torch.cuda.synchronize()
    c128 = torch.complex128
    xn = torch.linalg.vector_norm(x.to(c128)).item()
    assert abs(torch.linalg.vector_norm(z.to(c128)).item() / xn - 1) < 1e-5
    assert (torch.linalg.vector_norm((v - x).to(c128)) / xn).item() < 2e-5
    lhs = torch.vdot(z.to(torch.complex128), r.to(torch.complex128)).item()
    rhs = torch.vdot(x.to(torch.complex128), w.to(torch.complex128)).item()
    assert abs(lhs - rhs) / abs(lhs) < 1e-4


def test_sampled_outputs_at_large_size(gpu):
    """Full-size single-layer check with sampled rows: for L = 1,
    z = F D_1 U x, so any row of z is a DFT of one padded, phase-multiplied
    row combination the oracle can compute exactly; compare 4 sampled rows."""
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(6)
    n_shape, m_shape = (1024, 1024), (2048, 2048)
    th, x = random_problem(rng, n_shape, m_shape, 1)
    plan = make_plan([(n_shape, m_shape, 1)], [th], gpu)
    zd = torch.empty(2048 * 2048, dtype=torch.complex64, device=gpu)
    srpr.sr_forward(plan, to_dev(x.ravel(), gpu), zd, None)
    torch.cuda.synchronize()
    z = to_host(zd).reshape(m_shape)
    U = oracle.zero_pad(x, m_shape) * np.exp(1j * th[0].astype(np.float64))
    F2 = oracle.dft_matrix(2048)
    W = U @ F2.T  # axis-1 transform of every row (F symmetric)
    for k1 in (0, 1, 1023, 2047):
        row = F2[k1] @ W  # axis-0 transform, row k1 only
        assert rel_l2(z[k1], row) <= TOL_OP


NARROW = 512  # tile-width flag of the four-elements-per-thread shape
WIDE = 1024   # ... of the sixteen-elements-per-thread shape (2048-point columns, single-buffered)


@pytest.mark.parametrize("n_shape,m_shape,L", [((256, 256), (512, 512), 2), ((600, 300), (2048, 512), 3),
                                               ((300, 700), (768, 2048), 2), ((40, 50), (96, 128), 3),
                                               ((100, 30), (256, 64), 2), ((500, 200), (1024, 256), 3)])
@pytest.mark.parametrize("col_tile", [2, 4, 8, 16, 2 | 256, 4 | 256, 8 | 256, 16 | 256,
                                      2 | NARROW, 4 | NARROW, 8 | NARROW, 8 | 256 | WIDE])
def test_every_tile_variant(gpu, monkeypatch, n_shape, m_shape, L, col_tile):
    """Every compiled column tile (double- and single-buffered LDS, default,
    narrow and wide thread shape) and the row tiles of both shapes, with and
    without the exp(i theta) table, against the oracle.  Widths a length does
    not offer fall back to its default tile (and the wide shape, built for the
    [F D F] column passes only, to the default tile in every other pass)."""
    import torch
    import paper_2409_05734_amd as srpr
    rng = np.random.default_rng(col_tile + L)
    th, x = random_problem(rng, n_shape, m_shape, L)
    z_ref = oracle.forward(x, th)
    r = z_ref.astype(np.complex64)
    v_ref = oracle.adjoint(r, th, n_shape)
    for row_tile, table in ((1, 0), (4, 1), (64, 1), (1 | NARROW, 1), (2 | NARROW, 0), (4 | NARROW, 1)):
        monkeypatch.setenv("SR_TUNE_FORCE", f"{col_tile},{row_tile},{table}")
        plan = make_plan([(n_shape, m_shape, L)], [th], gpu)
        zd = torch.empty(int(np.prod(m_shape)), dtype=torch.complex64, device=gpu)
        vd = torch.empty(int(np.prod(n_shape)), dtype=torch.complex64, device=gpu)
        srpr.sr_forward(plan, to_dev(x.ravel(), gpu), zd, None)
        srpr.sr_adjoint(plan, to_dev(r.ravel(), gpu), vd)
        torch.cuda.synchronize()
        assert rel_l2(to_host(zd).reshape(m_shape), z_ref) <= TOL_OP
        assert rel_l2(to_host(vd).reshape(n_shape), v_ref) <= TOL_OP
