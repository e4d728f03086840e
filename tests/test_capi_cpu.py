"""C ABI checks that need no GPU: the library loads, exports every function
include/fk.h declares, and rejects malformed input with status codes before
touching the device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1410_4054_amd import fk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fk.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fk_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = header_functions()
    assert "fk_csr_create" in names and "fk_solve" in names and "fk_get_residual_history" in names
    assert sorted(fk.exported_symbols()) == names


def test_library_exports_every_declared_symbol():
    L = fk.lib()
    for name in header_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", fk.library_path()],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (fk_[a-z0-9_]+)$", out, flags=re.M))
    assert set(header_functions()) <= exported


def test_version_and_status_strings():
    assert "gfx950" in fk.version()
    assert fk.status_str(fk.OK) == "FK_OK"
    assert fk.status_str(fk.E_CSR) == "FK_E_CSR"
    assert fk.status_str(fk.BREAKDOWN) == "FK_BREAKDOWN"
    assert fk.status_str(99) == "FK_UNKNOWN"


def _create(n, nnz, rp, ci, va, kind=fk.PTR_HOST):
    L = fk.lib()
    h = ctypes.c_void_p()
    args = []
    for a, dt in ((rp, np.int32), (ci, np.int32), (va, np.float64)):
        if a is None:
            args.append(None)
        else:
            arr = np.ascontiguousarray(a, dtype=dt)
            args.append(arr)
    ptrs = [None if a is None else a.ctypes.data_as(ctypes.c_void_p) for a in args]
    st = L.fk_csr_create(n, nnz, ptrs[0], ptrs[1], ptrs[2], kind, None, ctypes.byref(h))
    return st, L.fk_last_error().decode(), h


@pytest.mark.parametrize("case,n,nnz,rp,ci,expect,msg", [
    ("n_zero", 0, 0, [0], [], fk.E_ARG, "n = 0"),
    ("n_negative", -3, 0, [0], [], fk.E_ARG, "n = -3"),
    ("nnz_negative", 2, -1, [0, 0, 0], [], fk.E_ARG, "nnz"),
    ("row_ptr0", 2, 2, [1, 1, 2], [0, 1], fk.E_CSR, "row_ptr[0]"),
    ("decreasing", 3, 2, [0, 2, 1, 2], [0, 1], fk.E_CSR, "decreases"),
    ("last_not_nnz", 2, 3, [0, 1, 2], [0, 1, 1], fk.E_CSR, "row_ptr[n]"),
    ("col_negative", 2, 2, [0, 1, 2], [0, -1], fk.E_CSR, "col_idx[1]"),
    ("col_too_large", 2, 2, [0, 1, 2], [0, 2], fk.E_CSR, "col_idx[1]"),
])
def test_csr_validation(case, n, nnz, rp, ci, expect, msg):
    va = np.ones(max(len(ci), 1))
    st, err, h = _create(n, nnz, rp, ci, va)
    assert st == expect, (case, st, err)
    assert msg in err, (case, err)
    assert not h.value


def test_csr_null_arrays_and_bad_kind():
    st, err, _ = _create(2, 2, None, [0, 1], [1.0, 1.0])
    assert st == fk.E_ARG
    st, err, _ = _create(2, 2, [0, 1, 2], None, [1.0, 1.0])
    assert st == fk.E_ARG
    st, err, _ = _create(2, 2, [0, 1, 2], [0, 1], [1.0, 1.0], kind=7)
    assert st == fk.E_ARG and "ptr_kind" in err
    L = fk.lib()
    rp = np.array([0, 0], dtype=np.int32)
    assert L.fk_csr_create(1, 0, rp.ctypes.data_as(ctypes.c_void_p), None, None, 0, None, None) == fk.E_ARG


def test_null_handles_rejected():
    L = fk.lib()
    opts = fk._Opts(0, 1e-8, 10, 1, 32, 0)
    h = ctypes.c_void_p()
    assert L.fk_solver_create(None, ctypes.byref(opts), None, ctypes.byref(h)) == fk.E_ARG
    assert L.fk_solve(None, None, None) == fk.E_ARG
    assert L.fk_csr_destroy(None) == fk.E_ARG
    assert L.fk_solver_destroy(None) == fk.E_ARG
    k = ctypes.c_int32()
    assert L.fk_get_iterations(None, ctypes.byref(k)) == fk.E_ARG
    out = ctypes.c_double()
    assert L.fk_dot(-1, None, None, ctypes.byref(out), None) == fk.E_ARG
    assert L.fk_dot(0, None, None, ctypes.byref(out), None) == fk.OK and out.value == 0.0
    assert L.fk_copy(None, None, -5, None) == fk.E_ARG
    assert L.fk_copy(None, None, 0, None) == fk.OK
    assert L.fk_spmv(None, None, None, None, None) == fk.E_ARG


def test_missing_library_fails_loudly(tmp_path):
    code = ("import os; os.environ['FK_LIBRARY'] = %r\n"
            "from paper_1410_4054_amd import fk\n"
            "try:\n    fk.lib()\nexcept OSError:\n    print('raised')\n") % str(tmp_path / "absent" / "libfk.so")
    res = subprocess.run(["python", "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert "raised" in res.stdout, res.stderr


def _batch_create(sys_ptr, rp, ci, vals):
    L = fk.lib()
    sp = np.ascontiguousarray(sys_ptr, dtype=np.int64)
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    va = np.ascontiguousarray(vals, dtype=np.float64)
    h = ctypes.c_void_p()
    return L.fk_batch_create(len(sp) - 1, sp.ctypes.data_as(ctypes.c_void_p), ci.size,
                             rp.ctypes.data_as(ctypes.c_void_p), ci.ctypes.data_as(ctypes.c_void_p),
                             va.ctypes.data_as(ctypes.c_void_p), 0, None, ctypes.byref(h))


@pytest.mark.parametrize("case,sys_ptr,rp,ci,expect", [
    ("cross_block_column", [0, 2, 3], [0, 1, 3, 4], [0, 1, 2, 2], fk.E_CSR),  # row 1 reads column 2 of system 1
    ("empty_system", [0, 2, 2, 3], [0, 1, 2, 3], [0, 1, 2], fk.E_CSR),
    ("sys_ptr_not_zero", [1, 3], [0, 1, 2, 3], [0, 1, 2], fk.E_CSR),
    ("row_ptr_end", [0, 2], [0, 1, 3], [0, 1], fk.E_CSR),
    ("row_ptr_decreasing", [0, 3], [0, 2, 1, 3], [0, 1, 2], fk.E_CSR),
])
def test_batch_validation(case, sys_ptr, rp, ci, expect):
    """Block-diagonal structure and CSR conventions are checked on the host
    before any device work."""
    assert _batch_create(sys_ptr, rp, ci, np.ones(len(ci))) == expect, case
    assert fk.lib().fk_last_error()


def test_batch_null_arguments():
    L = fk.lib()
    assert L.fk_batch_create(0, None, 0, None, None, None, 0, None, None) == fk.E_ARG
    assert L.fk_batch_destroy(None) == fk.E_ARG
    assert L.fk_batch_results(None, None, None, None, None) == fk.E_ARG


@pytest.mark.parametrize("cname,pyname", [("fk_opts", "_Opts"), ("fk_batch_opts", "_BatchOpts")])
def test_struct_layouts_match_the_header(cname, pyname, tmp_path):
    """The binding's ctypes mirrors of the option structs have the C
    layout: gcc compiles include/fk.h and reports sizeof and every field's
    offsetof, compared field by field."""
    cls = getattr(fk, pyname)
    names = [f[0] for f in cls._fields_]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "fk.h"', "int main(void) {",
             f'    printf("size %zu\\n", sizeof({cname}));']
    lines += [f'    printf("{n} %zu\\n", offsetof({cname}, {n}));' for n in names]
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                      check=True).stdout.splitlines())
    assert int(out["size"]) == ctypes.sizeof(cls)
    for n in names:
        assert int(out[n]) == getattr(cls, n).offset, n
