"""Pins the oracle's reverse-mode convention to PyTorch's own autograd on the
CPU: the same operator written with torch.fft (an independent library FFT)
and differentiated by torch gives the oracle's forward_vjp / adjoint_vjp."""
import numpy as np
import torch

import oracle


def _torch_forward(x, th, m_shape):
    off = [(M - N) // 2 for N, M in zip(x.shape, m_shape)]
    Z = torch.zeros(m_shape, dtype=torch.complex128)
    Z = Z.index_put((torch.arange(off[0], off[0] + x.shape[0])[:, None],
                     torch.arange(off[1], off[1] + x.shape[1])[None, :]), x)
    for l in range(th.shape[0]):
        Z = torch.fft.fftn(torch.exp(1j * th[l]) * Z, norm="ortho")
    return Z


def test_forward_vjp_matches_torch_autograd():
    rng = np.random.default_rng(0)
    n_shape, m_shape, L = (3, 4), (6, 8), 2
    th_np = rng.uniform(0, 2 * np.pi, (L,) + m_shape)
    x_np = rng.standard_normal(n_shape) + 1j * rng.standard_normal(n_shape)
    gz_np = rng.standard_normal(m_shape) + 1j * rng.standard_normal(m_shape)
    th = torch.tensor(th_np, requires_grad=True)
    x = torch.tensor(x_np, requires_grad=True)
    z = _torch_forward(x, th, m_shape)
    # real scalar with dL/dz = gz in torch's convention: L = Re <gz, z>
    loss = (torch.conj(torch.tensor(gz_np)) * z).real.sum()
    gx_t, gth_t = torch.autograd.grad(loss, (x, th))
    gx_o, gth_o = oracle.forward_vjp(x_np, th_np, gz_np)
    assert np.abs(gx_t.numpy() - gx_o).max() < 1e-12
    assert np.abs(gth_t.numpy() - gth_o).max() < 1e-12


def test_adjoint_vjp_matches_torch_autograd():
    rng = np.random.default_rng(1)
    n_shape, m_shape, L = (3, 4), (6, 8), 3
    th_np = rng.uniform(0, 2 * np.pi, (L,) + m_shape)
    r_np = rng.standard_normal(m_shape) + 1j * rng.standard_normal(m_shape)
    gv_np = rng.standard_normal(n_shape) + 1j * rng.standard_normal(n_shape)
    th = torch.tensor(th_np, requires_grad=True)
    r = torch.tensor(r_np, requires_grad=True)
    V = r
    for l in range(L - 1, -1, -1):
        V = torch.exp(-1j * th[l]) * torch.fft.ifftn(V, norm="ortho")
    off = [(M - N) // 2 for N, M in zip(n_shape, m_shape)]
    v = V[off[0]:off[0] + n_shape[0], off[1]:off[1] + n_shape[1]]
    loss = (torch.conj(torch.tensor(gv_np)) * v).real.sum()
    gr_t, gth_t = torch.autograd.grad(loss, (r, th))
    gr_o, gth_o = oracle.adjoint_vjp(r_np, th_np, n_shape, gv_np)
    assert np.abs(gr_t.numpy() - gr_o).max() < 1e-12
    assert np.abs(gth_t.numpy() - gth_o).max() < 1e-12
