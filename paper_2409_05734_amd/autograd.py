"""torch.autograd Functions over the library's structured operator.

StructuredA(x, theta) = A(theta) x and StructuredAH(r, theta) = A(theta)^H r
(section III, Eq. (5)) with gradients with respect to both the signal and the
phase masks, computed by the library's reverse-mode kernels
(sr_forward_vjp / sr_adjoint_vjp, intermediates recomputed per call).
Gradients follow PyTorch's complex convention (dL/dRe + i dL/dIm).

`theta` is the plan's whole phase buffer as a float32 device tensor (for a
batch of problems sharing one set of masks: shape (L * m,)).

unrolled_gd_loss() builds the mask-design objective: the mean phase-aligned
relative squared error after T unrolled gradient-descent steps (Eq. (2)) on
intensities y = |A(theta) x*|^2 (Eq. (1)).
"""
from __future__ import annotations

import torch

from . import Plan, sr_adjoint_vjp, sr_forward, sr_forward_vjp, sr_adjoint, sr_plan_set_theta


class StructuredA(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, theta, plan: Plan):
        theta = theta.detach().contiguous()
        x = x.detach().contiguous()
        sr_plan_set_theta(plan, theta)
        z = torch.empty(plan.m_total, dtype=torch.complex64, device=x.device)
        sr_forward(plan, x, z, None)
        ctx.save_for_backward(x, theta)
        ctx.plan = plan
        return z

    @staticmethod
    def backward(ctx, gz):
        x, theta = ctx.saved_tensors
        plan = ctx.plan
        sr_plan_set_theta(plan, theta)
        gx = torch.empty_like(x) if ctx.needs_input_grad[0] else None
        gth = torch.zeros_like(theta)
        sr_forward_vjp(plan, x, gz.contiguous(), gx, gth)
        return gx, (gth if ctx.needs_input_grad[1] else None), None


class StructuredAH(torch.autograd.Function):
    @staticmethod
    def forward(ctx, r, theta, plan: Plan):
        theta = theta.detach().contiguous()
        r = r.detach().contiguous()
        sr_plan_set_theta(plan, theta)
        v = torch.empty(plan.n_total, dtype=torch.complex64, device=r.device)
        sr_adjoint(plan, r, v)
        ctx.save_for_backward(r, theta)
        ctx.plan = plan
        return v

    @staticmethod
    def backward(ctx, gv):
        r, theta = ctx.saved_tensors
        plan = ctx.plan
        sr_plan_set_theta(plan, theta)
        gr = torch.empty_like(r) if ctx.needs_input_grad[0] else None
        gth = torch.zeros_like(theta)
        sr_adjoint_vjp(plan, r, gv.contiguous(), gr, gth)
        return gr, (gth if ctx.needs_input_grad[1] else None), None


def unrolled_gd_loss(plan: Plan, theta, x_star, x0, steps: int, mu: float):
    """Mean over the batch of (||x_T||^2 + ||x*||^2 - 2|x_T^H x*|)/||x*||^2.

    plan: B problems of one shape sharing the phase block `theta`;
    x_star, x0: (B, n) complex64 device tensors (x0 independent of theta).
    Step size per problem eta_b = mu m^2 / ||x*_b||^2 (= mu / (c mean(y_b))
    with c = 1/m, since mean(y_b) = ||x*_b||^2 / m for these operators).
    """
    B = x_star.shape[0]
    m = plan.problems[0].m
    xs = x_star.reshape(-1)
    ns2 = (x_star.abs() ** 2).sum(dim=1).to(torch.float32)
    eta = (mu * float(m) ** 2 / ns2).to(torch.float32)
    zs = StructuredA.apply(xs, theta, plan)
    y = (zs.abs() ** 2).reshape(B, m)
    x = x0.reshape(B, -1)
    for _ in range(steps):
        z = StructuredA.apply(x.reshape(-1), theta, plan).reshape(B, m)
        r = ((z.abs() ** 2 - y) * z).reshape(-1)
        g = StructuredAH.apply(r, theta, plan).reshape(B, -1) / m
        x = x - eta[:, None] * g
    inner = (x.conj() * x_star).sum(dim=1)
    per = ((x.abs() ** 2).sum(dim=1) + ns2 - 2.0 * inner.abs()) / ns2
    return per.mean()
