"""The C ABI library without a GPU: it loads, exports every declared symbol,
and rejects malformed arguments in host code before touching a device."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import pytest

import paper_2512_07057_amd as bsd

pytestmark = pytest.mark.skipif(not os.path.exists(bsd.LIB_PATH), reason="libbsd.so not built")


def test_exports_every_declared_symbol():
    names = bsd.exported_symbols_from_header()
    assert {"bsd_code_create", "bsd_code_destroy", "bsd_decode", "bsd_decode_ex", "bsd_bp_run",
            "bsd_code_info", "bsd_last_error", "bsd_version"} <= set(names)
    lib = bsd.load()
    for n in names:
        assert hasattr(lib, n), n


def test_version_string():
    assert "gfx950" in bsd.version()


def _create(m, n, k, colptr, rowidx, p, lptr=None, lidx=None):
    lib = bsd.load()
    i32p = C.POINTER(C.c_int32)
    colptr = np.ascontiguousarray(colptr, np.int32)
    rowidx = np.ascontiguousarray(rowidx, np.int32)
    p = np.ascontiguousarray(p, np.float64)
    h = C.c_void_p()
    lp = np.ascontiguousarray(lptr, np.int32).ctypes.data_as(i32p) if lptr is not None else None
    li = np.ascontiguousarray(lidx, np.int32).ctypes.data_as(i32p) if lidx is not None else None
    rc = lib.bsd_code_create(m, n, k, colptr.ctypes.data_as(i32p), rowidx.ctypes.data_as(i32p),
                             p.ctypes.data_as(C.POINTER(C.c_double)), lp, li, C.byref(h))
    return rc, lib.bsd_last_error().decode()


@pytest.mark.parametrize("case,fragment", [
    ("neg_m", "m, n must be"),
    ("bad_ptr0", "h_colptr[0]"),
    ("descending", "strictly ascending"),
    ("row_range", "row index out of range"),
    ("p_zero", "is not in (0,1)"),
    ("p_nan", "is not in (0,1)"),
    ("deg9", "degree 9"),
    ("k_big", "k must be"),
])
def test_create_rejects_malformed_input(case, fragment):
    colptr, rowidx, p = [0, 2, 3], [0, 1, 1], [0.1, 0.2]
    m, n, k = 2, 2, 0
    if case == "neg_m":
        m = -1
    elif case == "bad_ptr0":
        colptr = [1, 2, 3]
    elif case == "descending":
        rowidx = [1, 0, 1]
    elif case == "row_range":
        rowidx = [0, 5, 1]
    elif case == "p_zero":
        p = [0.0, 0.2]
    elif case == "p_nan":
        p = [float("nan"), 0.2]
    elif case == "deg9":
        m, n = 9, 1
        colptr, rowidx, p = [0, 9], list(range(9)), [0.1]
    elif case == "k_big":
        k = 65
        return _assert(_create(m, n, k, colptr, rowidx, p, [0, 0, 0], [0]), fragment)
    _assert(_create(m, n, k, colptr, rowidx, p), fragment)


def _assert(res, fragment):
    rc, msg = res
    assert rc == bsd.BSD_EINVAL
    assert fragment in msg, msg


def test_decode_rejects_bad_params_before_device_work():
    lib = bsd.load()
    prm = bsd.make_params(10, 0, 20, 8)
    rc = lib.bsd_decode(None, C.byref(prm), 1, None, None, None, None, None)
    assert rc == bsd.BSD_EINVAL and "code is NULL" in lib.bsd_last_error().decode()


def test_server_needs_a_hardware_queue_per_code(monkeypatch):
    """bsd_server_create_ex refuses more codes than the process has hardware
    queues (checked before any device call)."""
    lib = bsd.load()
    monkeypatch.setenv("GPU_MAX_HW_QUEUES", "4")
    codes = (C.c_void_p * 5)(*[C.c_void_p(16 * (i + 1)) for i in range(5)])
    prm = (bsd.Params * 5)()
    out = C.c_void_p()
    rc = lib.bsd_server_create_ex(5, codes, prm, None, None, C.byref(out))
    assert rc == bsd.BSD_EINVAL
    assert b"hardware queues" in lib.bsd_last_error()
