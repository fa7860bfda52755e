"""Structured random phase retrieval on MI355X (gfx950).

Python binding of libsrpr (include/sr.h).  Functions carry the names of the
C entry points and only marshal torch tensors (device memory) and the current
HIP stream into them; all computation happens in the library's HIP kernels.

    plan = Plan([Problem((256, 256), (512, 512), layers=2)], theta)
    sr_forward(plan, x, y=y)          # y = |A x|^2          (Eq. (1), Eq. (5))
    sr_spectral_init(plan, y, v0, 100, -1.0, x0)              (Eq. (3)-(4))
    sr_gd_solve(plan, y, x0, 500, [eta])                       (Eq. (2))

Several problems go into one plan (arrays concatenated, offsets from
sr_plan_offsets).  Problems of one shape whose phase blocks are shared or
evenly spaced run as a stack (one launch per pass for all of them, results
bitwise equal to one-by-one runs); plans of many uneven problems run one
launch per pass level (sr_plan_set_schedule picks explicitly).
StructuredA / StructuredAH (autograd.py) make A and A^H differentiable with
respect to the signal and the phases.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import (SR_DENSE, SR_E_NONFINITE, SR_LOSS_L2, SR_LOSS_POISSON, SR_SCHED_AUTO, SR_SCHED_BATCHED,
                   SR_SCHED_LOOP, SR_STRUCTURED, SrError)

__all__ = [
    "Problem", "Plan", "SrError",
    "sr_plan_set_theta", "sr_plan_workspace_size", "sr_plan_set_workspace", "sr_plan_offsets", "sr_plan_set_schedule", "sr_plan_set_loss",
    "sr_plan_sync",
    "sr_forward", "sr_adjoint", "sr_spectral_init", "sr_gd_solve", "sr_gd_solve_noalloc", "sr_forward_vjp",
    "sr_adjoint_vjp", "sr_gd_step_vjp", "sr_intensity_vjp",
    "SR_STRUCTURED", "SR_DENSE", "SR_SCHED_AUTO", "SR_SCHED_LOOP", "SR_SCHED_BATCHED", "SR_LOSS_L2", "SR_LOSS_POISSON",
    "SR_E_NONFINITE",
]


@dataclass
class Problem:
    """Signal shape n_shape, measurement shape m_shape, L layers.

    The transforms run on a grid of max(n, m) points per axis: the signal is
    zero-padded into it where m > n, the measurements are its centred window
    where m < n.  theta_offset: float offset of this problem's L phase grids
    in the plan's theta buffer (None: packed after the previous problem's
    block)."""
    n_shape: tuple
    m_shape: tuple
    layers: int = 2
    theta_offset: int | None = None
    kind: int = SR_STRUCTURED

    @property
    def n(self) -> int:
        return int(np.prod(self.n_shape))

    @property
    def m(self) -> int:
        return int(np.prod(self.m_shape))

    @property
    def grid_shape(self) -> tuple:
        return tuple(max(a, b) for a, b in zip(self.n_shape, self.m_shape))

    @property
    def grid(self) -> int:
        return int(np.prod(self.grid_shape))


def _torch():
    import torch
    return torch


def _ptr(t, dtype, numel: int, name: str, allow_none: bool = False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live in GPU memory")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A set of problems sharing one device workspace and one HIP stream.

    theta: host float32 array (any shape) holding every problem's phases, or
    None for dense plans.  dense_A: device complex64 (m, n) matrix for dense
    plans (kept referenced by the plan).  stream: torch.cuda.Stream or None
    (current stream)."""

    def __init__(self, problems, theta=None, dense_A=None, stream=None):
        torch = _torch()
        self.problems = list(problems)
        kind = self.problems[0].kind
        arr = (_lib.SrProblem * len(self.problems))()
        off = 0
        for i, p in enumerate(self.problems):
            q = arr[i]
            q.ndim = len(p.n_shape)
            n2 = list(p.n_shape) + [1]
            m2 = list(p.m_shape) + [1]
            q.n[0], q.n[1] = int(n2[0]), int(n2[1])
            q.m[0], q.m[1] = int(m2[0]), int(m2[1])
            q.layers = int(p.layers)
            q.kind = int(p.kind)
            if kind == SR_STRUCTURED:
                q.theta_offset = int(off if p.theta_offset is None else p.theta_offset)
                off = q.theta_offset + p.layers * p.grid
            else:
                q.theta_offset = 0
        self._theta_host = None
        theta_ptr, theta_len = None, 0
        if theta is not None:
            th = np.ascontiguousarray(np.asarray(theta, dtype=np.float32).ravel())
            self._theta_host = th
            theta_ptr, theta_len = th.ctypes.data_as(ctypes.c_void_p), th.size
        self.dense_A = dense_A
        a_ptr = None
        if dense_A is not None:
            p0 = self.problems[0]
            a_ptr = _ptr(dense_A, torch.complex64, p0.m * p0.n, "dense_A")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.handle = ctypes.c_void_p()
        _lib.call("sr_plan_create", ctypes.byref(self.handle), arr, len(self.problems), theta_ptr, theta_len,
                  a_ptr, ctypes.c_void_p(self.stream.cuda_stream))
        self.theta_len = theta_len
        xo = (ctypes.c_int64 * (len(self.problems) + 1))()
        yo = (ctypes.c_int64 * (len(self.problems) + 1))()
        _lib.call("sr_plan_offsets", self.handle, xo, yo)
        self.x_off = list(xo)
        self.y_off = list(yo)
        _track(self)

    @property
    def nprob(self) -> int:
        return len(self.problems)

    @property
    def n_total(self) -> int:
        return self.x_off[-1]

    @property
    def m_total(self) -> int:
        return self.y_off[-1]

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.load().sr_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Plans still alive at interpreter exit are destroyed from an exit handler.
# It is registered when the first plan is made, after torch (imported by
# Plan.__init__) has registered its own, so it runs before them (exit
# handlers run last-registered first): every plan's graphs, streams and
# device memory go back while the HIP runtime and any profiler attached to it
# are fully up, rather than from finalizers that may run during their teardown.
_live_plans: "weakref.WeakSet[Plan]" = weakref.WeakSet()
_exit_hook = False


def _destroy_live_plans() -> None:
    for plan in list(_live_plans):
        try:
            plan.close()
        except Exception:
            pass


def _track(plan: Plan) -> None:
    global _exit_hook
    if not _exit_hook:
        atexit.register(_destroy_live_plans)
        _exit_hook = True
    _live_plans.add(plan)


def sr_plan_set_theta(plan: Plan, theta_dev) -> None:
    torch = _torch()
    _lib.call("sr_plan_set_theta", plan.handle, _ptr(theta_dev, torch.float32, plan.theta_len, "theta"),
              plan.theta_len)


def sr_plan_workspace_size(plan: Plan) -> int:
    v = ctypes.c_size_t()
    _lib.call("sr_plan_workspace_size", plan.handle, ctypes.byref(v))
    return v.value


def sr_plan_set_workspace(plan: Plan, workspace) -> None:
    """Move the plan's workspace into `workspace`, a contiguous uint8 GPU
    tensor of at least sr_plan_workspace_size bytes, 256-byte aligned; the
    plan keeps a reference to it."""
    torch = _torch()
    if not isinstance(workspace, torch.Tensor) or workspace.device.type != "cuda":
        raise TypeError("workspace must be a GPU tensor")
    if workspace.dtype != torch.uint8 or not workspace.is_contiguous():
        raise TypeError("workspace must be a contiguous uint8 tensor")
    _lib.call("sr_plan_set_workspace", plan.handle, ctypes.c_void_p(workspace.data_ptr()), workspace.numel())
    plan._workspace = workspace


def sr_plan_offsets(plan: Plan):
    return list(plan.x_off), list(plan.y_off)


def sr_plan_set_schedule(plan: Plan, schedule: int) -> None:
    _lib.call("sr_plan_set_schedule", plan.handle, int(schedule))


def sr_plan_set_loss(plan: Plan, loss: int, eps: float = 0.0) -> None:
    """GD loss of the plan: SR_LOSS_L2 (default) or SR_LOSS_POISSON with guard eps > 0."""
    _lib.call("sr_plan_set_loss", plan.handle, int(loss), float(eps))


def sr_plan_sync(plan: Plan) -> None:
    _lib.call("sr_plan_sync", plan.handle)


def sr_forward(plan: Plan, x, z=None, y=None) -> None:
    torch = _torch()
    _lib.call("sr_forward", plan.handle, _ptr(x, torch.complex64, plan.n_total, "x"),
              _ptr(z, torch.complex64, plan.m_total, "z", True), _ptr(y, torch.float32, plan.m_total, "y", True))


def sr_adjoint(plan: Plan, r, x_out) -> None:
    torch = _torch()
    _lib.call("sr_adjoint", plan.handle, _ptr(r, torch.complex64, plan.m_total, "r"),
              _ptr(x_out, torch.complex64, plan.n_total, "x_out"))


def sr_spectral_init(plan: Plan, y, v0, iters: int, lam: float, x0_out) -> None:
    torch = _torch()
    _lib.call("sr_spectral_init", plan.handle, _ptr(y, torch.float32, plan.m_total, "y"),
              _ptr(v0, torch.complex64, plan.n_total, "v0"), int(iters), float(lam),
              _ptr(x0_out, torch.complex64, plan.n_total, "x0_out"))


def sr_gd_solve(plan: Plan, y, x_inout, iters: int, eta, loss_trace=None) -> None:
    torch = _torch()
    eta_h = np.ascontiguousarray(np.broadcast_to(np.asarray(eta, dtype=np.float32), (plan.nprob,)))
    _lib.call("sr_gd_solve", plan.handle, _ptr(y, torch.float32, plan.m_total, "y"),
              _ptr(x_inout, torch.complex64, plan.n_total, "x_inout"), int(iters),
              eta_h.ctypes.data_as(ctypes.c_void_p),
              _ptr(loss_trace, torch.float32, int(iters) * plan.nprob, "loss_trace", True))


def sr_gd_solve_noalloc(plan: Plan, y, x_inout, iters: int, eta) -> None:
    """sr_gd_solve that allocates no device memory (2D grids up to 2^20 points)."""
    torch = _torch()
    eta_h = np.ascontiguousarray(np.broadcast_to(np.asarray(eta, dtype=np.float32), (plan.nprob,)))
    _lib.call("sr_gd_solve_noalloc", plan.handle, _ptr(y, torch.float32, plan.m_total, "y"),
              _ptr(x_inout, torch.complex64, plan.n_total, "x_inout"), int(iters),
              eta_h.ctypes.data_as(ctypes.c_void_p))


def sr_forward_vjp(plan: Plan, x, gz, gx_out, gtheta_accum) -> None:
    torch = _torch()
    _lib.call("sr_forward_vjp", plan.handle, _ptr(x, torch.complex64, plan.n_total, "x"),
              _ptr(gz, torch.complex64, plan.m_total, "gz"),
              _ptr(gx_out, torch.complex64, plan.n_total, "gx_out", True),
              _ptr(gtheta_accum, torch.float32, plan.theta_len, "gtheta_accum"))


def sr_adjoint_vjp(plan: Plan, r, gv, gr_out, gtheta_accum) -> None:
    torch = _torch()
    _lib.call("sr_adjoint_vjp", plan.handle, _ptr(r, torch.complex64, plan.m_total, "r"),
              _ptr(gv, torch.complex64, plan.n_total, "gv"),
              _ptr(gr_out, torch.complex64, plan.m_total, "gr_out", True),
              _ptr(gtheta_accum, torch.float32, plan.theta_len, "gtheta_accum"))


def sr_gd_step_vjp(plan: Plan, y, x, eta, gx_next, gx_out, gy_accum, gtheta_accum) -> None:
    torch = _torch()
    eta_h = np.ascontiguousarray(np.broadcast_to(np.asarray(eta, dtype=np.float32), (plan.nprob,)))
    _lib.call("sr_gd_step_vjp", plan.handle, _ptr(y, torch.float32, plan.m_total, "y"),
              _ptr(x, torch.complex64, plan.n_total, "x"), eta_h.ctypes.data_as(ctypes.c_void_p),
              _ptr(gx_next, torch.complex64, plan.n_total, "gx_next"),
              _ptr(gx_out, torch.complex64, plan.n_total, "gx_out"),
              _ptr(gy_accum, torch.float32, plan.m_total, "gy_accum", True),
              _ptr(gtheta_accum, torch.float32, plan.theta_len, "gtheta_accum"))


def sr_intensity_vjp(plan: Plan, x, gy, gx_out, gtheta_accum) -> None:
    torch = _torch()
    _lib.call("sr_intensity_vjp", plan.handle, _ptr(x, torch.complex64, plan.n_total, "x"),
              _ptr(gy, torch.float32, plan.m_total, "gy"),
              _ptr(gx_out, torch.complex64, plan.n_total, "gx_out", True),
              _ptr(gtheta_accum, torch.float32, plan.theta_len, "gtheta_accum"))
