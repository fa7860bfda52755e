"""torch.autograd Functions over the library's structured operator.

StructuredA(x, theta) = A(theta) x and StructuredAH(r, theta) = A(theta)^H r
(section III, Eq. (5)) with gradients with respect to both the signal and the
phase masks, computed by the library's reverse-mode kernels
(sr_forward_vjp / sr_adjoint_vjp, intermediates recomputed per call).
Gradients follow PyTorch's complex convention (dL/dRe + i dL/dIm).

`theta` is the plan's whole phase buffer as a float32 device tensor (for a
batch of problems sharing one set of masks: shape (L * m,)).  A Function
copies it into the plan only when it differs from the last one set (another
tensor, or the same tensor modified in place), so a loop of calls with one
theta re-uploads nothing.

unrolled_gd_loss() builds the mask-design objective: the mean phase-aligned
relative squared error after T unrolled gradient-descent steps (Eq. (2)) on
intensities y = |A(theta) x*|^2 (Eq. (1)).  The measurements (Intensity) and
the T steps (UnrolledGD) are one Function each: the forward runs the
library's GD passes step by step and keeps only the signal-sized iterates;
the backward runs the library's reverse GD step (sr_gd_step_vjp), which
recomputes A x and the residual of each step, so no measurement-sized tensor
is kept per step.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (Plan, sr_adjoint, sr_adjoint_vjp, sr_forward, sr_forward_vjp, sr_gd_solve, sr_gd_step_vjp,
               sr_intensity_vjp, sr_plan_set_theta)


def _use_theta(plan: Plan, theta: torch.Tensor) -> torch.Tensor:
    """Make `theta` the plan's phases; a no-op when it already is."""
    theta = theta.detach()
    if not theta.is_contiguous():
        theta = theta.contiguous()
    key = (theta.data_ptr(), theta._version, theta.numel())
    if getattr(plan, "_theta_key", None) != key:
        sr_plan_set_theta(plan, theta)
        plan._theta_key = key
    return theta


class StructuredA(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, theta, plan: Plan):
        theta = _use_theta(plan, theta)
        x = x.detach().contiguous()
        z = torch.empty(plan.m_total, dtype=torch.complex64, device=x.device)
        sr_forward(plan, x, z, None)
        ctx.save_for_backward(x, theta)
        ctx.plan = plan
        return z

    @staticmethod
    def backward(ctx, gz):
        x, theta = ctx.saved_tensors
        plan = ctx.plan
        _use_theta(plan, theta)
        gx = torch.empty_like(x) if ctx.needs_input_grad[0] else None
        gth = torch.zeros_like(theta)
        sr_forward_vjp(plan, x, gz.contiguous(), gx, gth)
        return gx, (gth if ctx.needs_input_grad[1] else None), None


class StructuredAH(torch.autograd.Function):
    @staticmethod
    def forward(ctx, r, theta, plan: Plan):
        theta = _use_theta(plan, theta)
        r = r.detach().contiguous()
        v = torch.empty(plan.n_total, dtype=torch.complex64, device=r.device)
        sr_adjoint(plan, r, v)
        ctx.save_for_backward(r, theta)
        ctx.plan = plan
        return v

    @staticmethod
    def backward(ctx, gv):
        r, theta = ctx.saved_tensors
        plan = ctx.plan
        _use_theta(plan, theta)
        gr = torch.empty_like(r) if ctx.needs_input_grad[0] else None
        gth = torch.zeros_like(theta)
        sr_adjoint_vjp(plan, r, gv.contiguous(), gr, gth)
        return gr, (gth if ctx.needs_input_grad[1] else None), None


class Intensity(torch.autograd.Function):
    """y = |A(theta) x|^2 (Eq. (1)); the backward recomputes A x."""

    @staticmethod
    def forward(ctx, x, theta, plan: Plan):
        theta = _use_theta(plan, theta)
        x = x.detach().contiguous()
        y = torch.empty(plan.m_total, dtype=torch.float32, device=x.device)
        sr_forward(plan, x, None, y)
        ctx.save_for_backward(x, theta)
        ctx.plan = plan
        return y

    @staticmethod
    def backward(ctx, gy):
        x, theta = ctx.saved_tensors
        plan = ctx.plan
        _use_theta(plan, theta)
        gx = torch.empty_like(x) if ctx.needs_input_grad[0] else None
        gth = torch.zeros_like(theta)
        sr_intensity_vjp(plan, x, gy.contiguous(), gx, gth)
        return gx, (gth if ctx.needs_input_grad[1] else None), None


class UnrolledGD(torch.autograd.Function):
    """x_T after `steps` GD steps x <- x - (eta/m) A^H((|Ax|^2 - y) . Ax)
    (Eq. (2)) from x0, differentiable in x0, y and theta.  eta: host array of
    raw steps, one per problem.  Keeps x_0 .. x_{T-1} (signal-sized)."""

    @staticmethod
    def forward(ctx, x0, y, theta, plan: Plan, eta, steps: int):
        theta = _use_theta(plan, theta)
        y = y.detach().contiguous()
        x = x0.detach().contiguous().clone()
        hist = torch.empty((steps, plan.n_total), dtype=torch.complex64, device=x.device)
        for t in range(steps):
            hist[t].copy_(x)
            sr_gd_solve(plan, y, x, 1, eta)
        ctx.save_for_backward(hist, y, theta)
        ctx.plan, ctx.eta, ctx.steps = plan, np.asarray(eta, np.float32), steps
        return x

    @staticmethod
    def backward(ctx, gxT):
        hist, y, theta = ctx.saved_tensors
        plan = ctx.plan
        _use_theta(plan, theta)
        g = gxT.contiguous().clone()
        g2 = torch.empty_like(g)
        gy = torch.zeros_like(y)
        gth = torch.zeros_like(theta)
        for t in range(ctx.steps - 1, -1, -1):
            sr_gd_step_vjp(plan, y, hist[t], ctx.eta, g, g2, gy, gth)
            g, g2 = g2, g
        return g, gy, gth, None, None, None


def unrolled_gd_loss(plan: Plan, theta, x_star, x0, steps: int, mu: float):
    """Mean over the batch of (||x_T||^2 + ||x*||^2 - 2|x_T^H x*|)/||x*||^2.

    plan: B problems of one shape sharing the phase block `theta`;
    x_star, x0: (B, n) complex64 device tensors (x0 independent of theta).
    Step size per problem eta_b = mu m^2 / ||x*_b||^2 (= mu / (c mean(y_b))
    with c = 1/m, since mean(y_b) = ||x*_b||^2 / m for these operators).
    """
    B = x_star.shape[0]
    m = plan.problems[0].m
    ns2 = (x_star.abs() ** 2).sum(dim=1).to(torch.float32)
    eta = (mu * float(m) ** 2 / ns2.detach().cpu().numpy().astype(np.float64)).astype(np.float32)
    y = Intensity.apply(x_star.reshape(-1), theta, plan)
    x = UnrolledGD.apply(x0.reshape(-1), y, theta, plan, eta, steps).reshape(B, -1)
    inner = (x.conj() * x_star).sum(dim=1)
    per = ((x.abs() ** 2).sum(dim=1) + ns2 - 2.0 * inner.abs()) / ns2
    return per.mean()
