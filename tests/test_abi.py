"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid plans synchronously (before any device
work) with the documented status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sr.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sr_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2409_05734_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsrpr.so is not built (run paper_2409_05734_amd/build.py)")
    return _lib.load()


def test_header_and_binding_agree():
    from paper_2409_05734_amd import _lib
    declared = _declared_functions()
    assert declared, "no declarations found"
    assert sorted(_lib.SIGNATURES) == declared


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def _problem(n, m, L=2, off=0, kind=0):
    from paper_2409_05734_amd import _lib
    q = _lib.SrProblem()
    q.ndim = len(n)
    nn = list(n) + [1]
    mm = list(m) + [1]
    q.n[0], q.n[1] = nn[0], nn[1]
    q.m[0], q.m[1] = mm[0], mm[1]
    q.layers = L
    q.kind = kind
    q.theta_offset = off
    return q


def _create(lib, probs, theta_len, theta=True, dense=None):
    from paper_2409_05734_amd import _lib
    arr = (_lib.SrProblem * len(probs))(*probs)
    th = np.zeros(max(theta_len, 1), np.float32)
    h = ctypes.c_void_p()
    st = lib.sr_plan_create(ctypes.byref(h), arr, len(probs),
                            th.ctypes.data_as(ctypes.c_void_p) if theta else None,
                            theta_len, dense, None)
    return st, lib.sr_last_error().decode()


@pytest.mark.parametrize("n,m,L,tlen,status", [
    ((64,), (32,), 2, 64, -2),            # trimmed: theta must cover L x 64 grid points
    ((16, 16), (32, 30), 2, 2 * 960, -3),  # 30 has a prime factor 5
    ((16, 16), (32, 32), 0, 2048, -1),     # L = 0
    ((16, 16), (32, 32), 2, 1000, -2),     # theta block out of range
    ((0, 16), (32, 32), 2, 2048, -2),      # empty signal
    ((40,), (100,), 1, 100, -3),           # 1D length 100 unsupported
    ((4, 4), (8, 8), 1, 64, -3),           # 2D length 8 unsupported
    ((256,), (2048,), 4, 8192, -3),        # 1D needs L*m <= 4096
])
def test_invalid_plans_are_rejected(lib, n, m, L, tlen, status):
    st, msg = _create(lib, [_problem(n, m, L)], tlen)
    assert st == status, msg
    assert msg


def test_null_and_kind_errors(lib):
    from paper_2409_05734_amd import _lib
    assert lib.sr_plan_create(None, None, 0, None, 0, None, None) == -1
    st, _ = _create(lib, [_problem((8,), (32,), 1)], 32, theta=False)
    assert st == -1  # structured plan without phases
    st, _ = _create(lib, [_problem((8,), (32,), 1, kind=1)], 0, theta=False, dense=None)
    assert st == -1  # dense plan without a matrix
    st, _ = _create(lib, [_problem((8,), (32,), 1), _problem((8,), (32,), 1, kind=1)], 64)
    assert st == -1  # mixed kinds
    assert lib.sr_forward(None, None, None, None) == -1
    assert lib.sr_plan_set_loss(None, 0, 0.0) == -1
    assert lib.sr_plan_set_workspace(None, None, 0) == -1
    assert lib.sr_plan_destroy(None) == 0
    assert lib.sr_status_string(-3).decode() == "unsupported configuration"
