"""The C-ABI library loads and exports every entry point its header declares (CPU only)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pipesafe.h")
LIB = os.path.join(ROOT, "paper_2108_10591_amd", "libpipesafe.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ps_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2108_10591_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["ps_create", "ps_solve", "ps_solve_dev", "ps_destroy", "ps_strerror",
                     "ps_default_options", "ps_spmv_dev", "ps_create_batch", "ps_solve_batch",
                     "ps_solve_batch_dev", "ps_matrix_info"]:
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (ps_[a-z_]+)\b", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    for f in declared_functions():
        getattr(lib, f)


def test_options_defaults_and_strerror(lib):
    from paper_2108_10591_amd import pipesafe
    o = pipesafe.options()
    assert (o.rr_m, o.rr_M, o.norm_ref, o.batch_iters, o.overlap, o.profile, o.resume, o.graph,
            o.schedule, o.x0_fallback) == (100, 0, 0, 0, -1, 0, 0, 1, -1, 0)
    assert ctypes.sizeof(pipesafe.Options) == 56
    assert ctypes.sizeof(pipesafe.Info) == 80
    pipesafe.library().ps_strerror.restype = ctypes.c_char_p
    for code in (0, 1, 2, 3, -1, -2, -3, -4, -5, -6):
        assert pipesafe.library().ps_strerror(code)


def _create(n, rowptr, col, val):
    from paper_2108_10591_amd import pipesafe
    L = pipesafe.library()
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    rc = L.ps_create(ctypes.byref(h), n, int(rp[-1]) if rp.size else 0, rp.ctypes.data, c.ctypes.data,
                     v.ctypes.data)
    return rc, h


@pytest.mark.parametrize("case", ["bad_rowptr0", "decreasing", "col_range", "nan_value", "n_zero",
                                  "nnz_mismatch"])
def test_create_rejects_invalid_csr_before_touching_the_device(lib, case):
    rowptr, col, val, n = [0, 1, 2], [0, 1], [1.0, 2.0], 2
    if case == "bad_rowptr0":
        rowptr = [1, 1, 2]
    elif case == "decreasing":
        rowptr, col, val = [0, 2, 1], [0, 1], [1.0, 2.0]
    elif case == "col_range":
        col = [0, 2]
    elif case == "nan_value":
        val = [1.0, float("nan")]
    elif case == "n_zero":
        n, rowptr, col, val = 0, [0], [], []
    if case == "nnz_mismatch":
        from paper_2108_10591_amd import pipesafe
        L = pipesafe.library()
        h = ctypes.c_void_p()
        rp = np.array([0, 1, 2], dtype=np.int64)
        c = np.array([0, 1], dtype=np.int32)
        v = np.array([1.0, 2.0])
        assert L.ps_create(ctypes.byref(h), 2, 3, rp.ctypes.data, c.ctypes.data, v.ctypes.data) == -1
        return
    rc, h = _create(n, rowptr, col, val)
    assert rc == -1 and not h.value


def test_solve_rejects_null_handle(lib):
    from paper_2108_10591_amd import pipesafe
    L = pipesafe.library()
    x = np.zeros(2)
    it, st = ctypes.c_int32(), ctypes.c_int32()
    rc = L.ps_solve(None, x.ctypes.data, None, 1e-8, 10, 1, None, x.ctypes.data, ctypes.byref(it),
                    None, ctypes.byref(st))
    assert rc == -1
    assert L.ps_destroy(None) == 0


@pytest.mark.parametrize("case", ["sys_ptr_start", "sys_ptr_end", "empty_system", "cross_system_col",
                                  "no_systems"])
def test_create_batch_rejects_invalid_layout_before_touching_the_device(lib, case):
    from paper_2108_10591_amd import pipesafe
    L = pipesafe.library()
    # two 2x2 diagonal systems
    rowptr = np.array([0, 1, 2, 3, 4], dtype=np.int64)
    col = np.array([0, 1, 2, 3], dtype=np.int32)
    val = np.ones(4)
    sys_ptr = np.array([0, 2, 4], dtype=np.int64)
    nsys = 2
    if case == "sys_ptr_start":
        sys_ptr = np.array([1, 2, 4], dtype=np.int64)
    elif case == "sys_ptr_end":
        sys_ptr = np.array([0, 2, 3], dtype=np.int64)
    elif case == "empty_system":
        sys_ptr = np.array([0, 2, 2, 4], dtype=np.int64)
        nsys = 3
    elif case == "cross_system_col":
        col = np.array([0, 2, 2, 3], dtype=np.int32)  # row 1 (system 0) references column 2
    elif case == "no_systems":
        nsys = 0
    h = ctypes.c_void_p()
    rc = L.ps_create_batch(ctypes.byref(h), nsys, sys_ptr.ctypes.data, 4, 4, rowptr.ctypes.data,
                           col.ctypes.data, val.ctypes.data)
    assert rc == -1 and not h.value


@pytest.mark.parametrize("field,value", [("format", 2), ("format", -2), ("sell_rows_per_lane", 3),
                                         ("sell_rows_per_lane", 0), ("spmv_shape", 5),
                                         ("index_bits", 8), ("index_bits", 64),
                                         ("gather_sort", 2), ("gather_sort", -2)])
def test_create_ex_rejects_invalid_layout_before_touching_the_device(lib, field, value):
    from paper_2108_10591_amd import pipesafe
    L = pipesafe.library()
    lay = pipesafe.layout()
    setattr(lay, field, value)
    rp = np.array([0, 1, 2], dtype=np.int64)
    c = np.array([0, 1], dtype=np.int32)
    v = np.array([1.0, 2.0])
    h = ctypes.c_void_p()
    assert L.ps_create_ex(ctypes.byref(h), 2, 2, rp.ctypes.data, c.ctypes.data, v.ctypes.data,
                          ctypes.byref(lay)) == -1 and not h.value
    sp = np.array([0, 2], dtype=np.int64)
    assert L.ps_create_batch_ex(ctypes.byref(h), 1, sp.ctypes.data, 2, 2, rp.ctypes.data,
                                c.ctypes.data, v.ctypes.data, ctypes.byref(lay)) == -1


def test_tuner_structs_and_argument_checks(lib):
    from paper_2108_10591_amd import pipesafe
    L = pipesafe.library()
    assert ctypes.sizeof(pipesafe.Layout) == 20
    assert ctypes.sizeof(pipesafe.TuneEntry) == 48
    assert ctypes.sizeof(pipesafe.TuneReport) == 8 + 48 * 48
    rp = np.array([0, 1, 2], dtype=np.int64)
    c = np.array([0, 1], dtype=np.int32)
    v = np.array([1.0, 2.0])
    h = ctypes.c_void_p()
    rep = pipesafe.TuneReport()
    # reps out of range, or a batch without row ranges: rejected before any device work
    assert L.ps_autotune_layout(ctypes.byref(h), 1, None, 2, 2, rp.ctypes.data, c.ctypes.data,
                                v.ctypes.data, 0, ctypes.byref(rep)) == -1
    assert L.ps_autotune_layout(ctypes.byref(h), 2, None, 2, 2, rp.ctypes.data, c.ctypes.data,
                                v.ctypes.data, 5, ctypes.byref(rep)) == -1
    o = pipesafe.options()
    assert L.ps_tune_options(None, None, 1, 10, ctypes.byref(o), None) == -1
