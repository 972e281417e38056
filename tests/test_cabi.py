"""C-ABI host checks that need no GPU: the library loads, exports every
function the header declares, and rejects malformed input with a status code
before touching the device."""
import ctypes

import numpy as np
import pytest

from paper_2604_11920_amd import lsqr as L


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_exports_every_declared_function(lib):
    names = L.header_functions()
    assert {"lsqr_create", "lsqr_solve", "lsqr_destroy", "lsqr_apply", "lsqr_apply_t"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for s in range(0, -7, -1):
        assert lib.lsqr_status_string(s).decode() not in ("", "unknown status")


def _create(lib, row_ptr, col, val, grid=(2, 2, 2), damp=0.1, smooth=0.5, n=None):
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.float64)
    nn = grid[0] * grid[1] * grid[2] if n is None else n
    csr = L.CSR(len(row_ptr) - 1, nn, len(col), *grid,
                row_ptr.ctypes.data, col.ctypes.data, val.ctypes.data, L.MEM_HOST)
    ctx = ctypes.c_void_p()
    rc = lib.lsqr_create(ctypes.byref(csr), damp, smooth, None, ctypes.byref(ctx))
    return rc, lib.lsqr_last_error(None).decode()


@pytest.mark.parametrize("case,expect", [
    ("decreasing_row_ptr", L.LSQR_E_BAD_CSR),
    ("col_out_of_range", L.LSQR_E_BAD_CSR),
    ("negative_col", L.LSQR_E_BAD_CSR),
    ("unsorted_cols", L.LSQR_E_BAD_CSR),
    ("duplicate_cols", L.LSQR_E_BAD_CSR),
    ("nan_value", L.LSQR_E_NONFINITE),
    ("inf_value", L.LSQR_E_NONFINITE),
    ("row_ptr_end", L.LSQR_E_BAD_CSR),
    ("grid_mismatch", L.LSQR_E_INVALID_ARG),
    ("negative_damp", L.LSQR_E_INVALID_ARG),
    ("nan_smooth", L.LSQR_E_INVALID_ARG),
])
def test_create_rejects(lib, case, expect):
    rp, ci, va = [0, 2, 3, 5], [0, 3, 1, 2, 7], [1.0, 2.0, 3.0, 4.0, 5.0]
    kw = {}
    if case == "decreasing_row_ptr":
        rp = [0, 3, 2, 5]
    elif case == "col_out_of_range":
        ci = [0, 3, 1, 2, 8]
    elif case == "negative_col":
        ci = [-1, 3, 1, 2, 7]
    elif case == "unsorted_cols":
        ci = [3, 0, 1, 2, 7]
    elif case == "duplicate_cols":
        ci = [0, 0, 1, 2, 7]
    elif case == "nan_value":
        va = [1.0, np.nan, 3.0, 4.0, 5.0]
    elif case == "inf_value":
        va = [1.0, 2.0, 3.0, 4.0, np.inf]
    elif case == "row_ptr_end":
        rp = [0, 2, 3, 4]
    elif case == "grid_mismatch":
        kw["n"] = 9
    elif case == "negative_damp":
        kw["damp"] = -0.1
    elif case == "nan_smooth":
        kw["smooth"] = float("nan")
    rc, msg = _create(lib, rp, ci, va, **kw)
    assert rc == expect, (rc, msg)
    assert msg


def test_null_arguments(lib):
    ctx = ctypes.c_void_p()
    assert lib.lsqr_create(None, 0.1, 0.5, None, ctypes.byref(ctx)) == L.LSQR_E_INVALID_ARG
    assert lib.lsqr_solve(None, None, 0, 1, 0.0, None, None, None) == L.LSQR_E_INVALID_ARG
    assert lib.lsqr_apply(None, None, None) == L.LSQR_E_INVALID_ARG
    lib.lsqr_destroy(None)


@pytest.mark.parametrize("field,value", [("row_format", 2), ("row_format", 3), ("row_format", 5),
                                         ("col_format", 3), ("col_format", 5), ("flags", 4),
                                         ("refine_stall_ratio", -0.5),
                                         ("refine_stall_ratio", 1.5),
                                         ("refine_stall_ratio", float("nan"))])
def test_create_rejects_unknown_formats_and_flags(lib, field, value):
    """Only the built formats and flags are accepted (row 0/1/4, column
    0/1/2/4, flags TIMING and NO_GRAPH), and a stall ratio in [0, 1]; the
    check comes before any device call."""
    rp = np.array([0, 2, 3], np.int64)
    ci = np.array([0, 3, 1], np.int32)
    va = np.array([1.0, 2.0, 3.0])
    csr = L.CSR(2, 4, 3, 2, 2, 1, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, L.MEM_HOST)
    opts = L.Opts()                     # zeros: FP64, no scaling, auto formats
    setattr(opts, field, value)
    ctx = ctypes.c_void_p()
    rc = lib.lsqr_create(ctypes.byref(csr), 0.1, 0.5, ctypes.byref(opts), ctypes.byref(ctx))
    assert rc == L.LSQR_E_INVALID_ARG, (rc, lib.lsqr_last_error(None).decode())
