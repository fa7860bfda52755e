"""ctypes binding of libsrpr.so (include/sr.h).

Argument marshalling only: every step of every call runs in the HIP library.
Importing this module does not load the library; the first call does, and it
raises if libsrpr.so has not been built.  There is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsrpr.so")

SR_OK = 0
SR_STRUCTURED = 0
SR_DENSE = 1
SR_SCHED_AUTO = 0
SR_SCHED_LOOP = 1
SR_SCHED_BATCHED = 2
SR_LOSS_L2 = 0
SR_LOSS_POISSON = 1
SR_E_NONFINITE = -5

STATUS_NAMES = {
    0: "SR_OK", -1: "SR_E_ARG", -2: "SR_E_SHAPE", -3: "SR_E_UNSUPPORTED", -4: "SR_E_HIP",
    -5: "SR_E_NONFINITE", -6: "SR_E_STATE", -7: "SR_E_NOMEM",
}

# Every symbol include/sr.h declares, with (restype, argtypes).
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f32 = ctypes.c_float


class SrProblem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 2),
        ("m", ctypes.c_int32 * 2),
        ("layers", ctypes.c_int32),
        ("kind", ctypes.c_int32),
        ("theta_offset", ctypes.c_int64),
    ]


SIGNATURES = {
    "sr_plan_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(SrProblem), _i32, _vp, _i64, _vp, _vp]),
    "sr_plan_set_theta": (ctypes.c_int, [_vp, _vp, _i64]),
    "sr_plan_workspace_size": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "sr_plan_set_workspace": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "sr_plan_offsets": (ctypes.c_int, [_vp, _vp, _vp]),
    "sr_plan_set_schedule": (ctypes.c_int, [_vp, _i32]),
    "sr_plan_set_loss": (ctypes.c_int, [_vp, _i32, _f32]),
    "sr_plan_sync": (ctypes.c_int, [_vp]),
    "sr_plan_destroy": (ctypes.c_int, [_vp]),
    "sr_forward": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "sr_adjoint": (ctypes.c_int, [_vp, _vp, _vp]),
    "sr_spectral_init": (ctypes.c_int, [_vp, _vp, _vp, _i32, _f32, _vp]),
    "sr_gd_solve": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp]),
    "sr_gd_solve_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp]),
    "sr_forward_vjp": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "sr_adjoint_vjp": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "sr_gd_step_vjp": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "sr_intensity_vjp": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "sr_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sr_last_error": (ctypes.c_char_p, []),
}

_lib = None


class SrError(RuntimeError):
    def __init__(self, status: int, func: str, message: str):
        self.status = status
        super().__init__(f"{func} failed: {STATUS_NAMES.get(status, status)}: {message}")


def load(path: str | None = None):
    """Load libsrpr.so once and declare every exported signature."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            f"{p} is missing: build it with `python paper_2409_05734_amd/build.py` "
            "(the library has no CPU fallback)")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def check(status: int, func: str) -> None:
    if status != SR_OK:
        msg = load().sr_last_error().decode(errors="replace")
        raise SrError(status, func, msg)


def call(name: str, *args) -> None:
    """Call an sr_* function that returns a status, raising SrError on failure."""
    check(getattr(load(), name)(*args), name)
