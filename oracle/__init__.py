"""ctypes front end of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the
benchmark's CPU-baseline leg.  The GPU library and its Python binding never
import it.  It shares no code with them; both take their inputs from the
seeded generators.

Functions take numpy arrays and a problems.Csr-like object (attributes n,
row_ptr, col_idx, vals).
"""
from __future__ import annotations

import contextlib
import ctypes
import os
from dataclasses import dataclass

import numpy as np

from .build import build as _build, library_path

METHODS = {
    "cg_classical": 0,
    "cg_pipelined": 1,
    "bicgstab_classical": 2,
    "bicgstab_pipelined": 3,
}
STATUS = {0: "converged", 1: "not_converged", 2: "breakdown", 3: "bad_arg"}
# inner products of the FP32 inner solver of solve_mixed
ACC_MODES = {"exact": 0, "f32": 1}

# Slots of one per-iteration trace record (see oracle.c).
TRACE_SLOTS = {
    "alpha": 0, "beta": 1, "omega": 2, "rr": 2, "rho": 3, "pap": 3, "apr": 4,
    "apap": 4, "rr_new": 5, "ss": 5, "ass": 6, "asas": 7, "asr": 8,
    "rr_expanded": 9, "rr_direct": 10,
}

class Oracle:
    """One loaded build of oracle.c (the default build, or a test variant)."""

    def __init__(self, path: str | None = None):
        path = path or library_path()
        if not os.path.exists(path):
            _build()
        lib = ctypes.CDLL(path)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.oracle_spmv.argtypes = [ctypes.c_int64, i32p, i32p, f64p, f64p, f64p]
        lib.oracle_spmv.restype = None
        lib.oracle_dot.argtypes = [ctypes.c_int64, f64p, f64p]
        lib.oracle_dot.restype = ctypes.c_double
        lib.oracle_set_dot_mode.argtypes = [ctypes.c_int]
        lib.oracle_set_dot_mode.restype = None
        lib.oracle_get_dot_mode.argtypes = []
        lib.oracle_get_dot_mode.restype = ctypes.c_int
        lib.oracle_trace_stride.argtypes = []
        lib.oracle_trace_stride.restype = ctypes.c_int
        lib.oracle_solve.argtypes = [
            ctypes.c_int, ctypes.c_int64, i32p, i32p, f64p, f64p, f64p, f64p,
            ctypes.c_double, ctypes.c_int32, f64p, f64p, ctypes.c_int32,
            ctypes.POINTER(ctypes.c_int32),
        ]
        lib.oracle_solve.restype = ctypes.c_int
        lib.oracle_solve_mixed.argtypes = [
            ctypes.c_int64, i32p, i32p, f64p, f64p, f64p, ctypes.c_double, ctypes.c_double,
            ctypes.c_int32, ctypes.c_int32, f64p, i32p, ctypes.c_int32,
            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
        ]
        lib.oracle_solve_mixed.restype = ctypes.c_int
        lib.oracle_solve_gmres.argtypes = [
            ctypes.c_int, ctypes.c_int32, ctypes.c_int64, i32p, i32p, f64p, f64p, f64p, f64p,
            ctypes.c_double, ctypes.c_int32, f64p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
        ]
        lib.oracle_solve_gmres.restype = ctypes.c_int
        f32p = ctypes.POINTER(ctypes.c_float)
        lib.oracle_spmv_f32.argtypes = [ctypes.c_int64, i32p, i32p, f32p, f32p, f32p]
        lib.oracle_spmv_f32.restype = None
        lib.oracle_dot_f32.argtypes = [ctypes.c_int64, f32p, f32p]
        lib.oracle_dot_f32.restype = ctypes.c_double
        lib.oracle_dot_f32acc.argtypes = [ctypes.c_int64, f32p, f32p]
        lib.oracle_dot_f32acc.restype = ctypes.c_float
        self.lib = lib
        self.path = path

    def spmv(self, A, p) -> np.ndarray:
        """q = A p, rows summed left to right in CSR order."""
        rp, rpp = _i32(A.row_ptr)
        ci, cip = _i32(A.col_idx)
        v, vp = _f64(A.vals)
        p, pp = _f64(p)
        q = np.empty(A.n)
        _, qp = _f64(q)
        self.lib.oracle_spmv(A.n, rpp, cip, vp, pp, qp)
        return q

    def spmv_f32(self, A, p) -> np.ndarray:
        """q = A p in FP32 (values rounded to FP32, one rounding per operation)."""
        rp, rpp = _i32(A.row_ptr)
        ci, cip = _i32(A.col_idx)
        v, vp = _f32(A.vals)
        p, pp = _f32(p)
        q = np.empty(A.n, dtype=np.float32)
        _, qp = _f32(q)
        self.lib.oracle_spmv_f32(A.n, rpp, cip, vp, pp, qp)
        return q

    def dot_f32(self, a, b) -> float:
        """<a, b> of two FP32 vectors, as if in twice FP64 precision, rounded to FP64."""
        a, ap = _f32(a)
        b, bp = _f32(b)
        if a.shape != b.shape:
            raise ValueError("shape mismatch")
        return float(self.lib.oracle_dot_f32(a.size, ap, bp))

    def dot_f32acc(self, a, b) -> np.float32:
        """<a, b> of two FP32 vectors accumulated in FP32, left to right."""
        a, ap = _f32(a)
        b, bp = _f32(b)
        if a.shape != b.shape:
            raise ValueError("shape mismatch")
        return np.float32(self.lib.oracle_dot_f32acc(a.size, ap, bp))

    def dot(self, a, b) -> float:
        """<a, b> by the compensated dot (twice working precision, one rounding)."""
        a, ap = _f64(a)
        b, bp = _f64(b)
        if a.shape != b.shape:
            raise ValueError("shape mismatch")
        return float(self.lib.oracle_dot(a.size, ap, bp))

    @contextlib.contextmanager
    def dot_mode(self, mode: int):
        """Temporarily switch the summation order of every oracle dot.

        0 = compensated (the oracle), 1 = plain left-to-right, 2 = plain
        pairwise.  Only for measuring how sensitive a trajectory is to
        summation order.
        """
        old = self.lib.oracle_get_dot_mode()
        self.lib.oracle_set_dot_mode(int(mode))
        try:
            yield
        finally:
            self.lib.oracle_set_dot_mode(old)

    def solve(self, A, b, x0=None, method: str = "cg_pipelined", rtol: float = 1e-8,
              max_iter: int | None = None, trace: bool = False) -> "Result":
        """Run one of Algorithms 1-4 on the CPU in FP64."""
        n = A.n
        if max_iter is None:
            max_iter = 10 * n
        rp, rpp = _i32(A.row_ptr)
        ci, cip = _i32(A.col_idx)
        v, vp = _f64(A.vals)
        b, bp = _f64(b)
        x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        _, xp = _f64(x)
        r = np.empty(n)
        _, rptr = _f64(r)
        cap = max_iter + 1
        hist = np.full(cap, np.nan)
        _, hp = _f64(hist)
        stride = self.lib.oracle_trace_stride()
        tr = np.full((cap, stride), np.nan) if trace else None
        trp = _f64(tr)[1] if trace else None
        k = ctypes.c_int32(0)
        st = self.lib.oracle_solve(METHODS[method], n, rpp, cip, vp, bp, xp, rptr, float(rtol),
                                   int(max_iter), hp, trp, cap, ctypes.byref(k))
        kk = int(k.value)
        return Result(x=x, r=r, k=kk, status=STATUS[st], hist=hist[: kk + 1].copy(),
                      trace=None if tr is None else tr[:kk].copy())

    def solve_gmres(self, A, b, x0=None, m: int = 30, pipelined: bool = True, rtol: float = 1e-8,
                    max_iter: int | None = None) -> "Result":
        """Restarted simpler GMRES(m): Algorithm 6 (pipelined) or 5 (classical)."""
        n = A.n
        if max_iter is None:
            max_iter = 10 * n
        rp, rpp = _i32(A.row_ptr)
        ci, cip = _i32(A.col_idx)
        v, vp = _f64(A.vals)
        b, bp = _f64(b)
        x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        _, xp = _f64(x)
        r = np.empty(n)
        _, rptr = _f64(r)
        cap = max_iter + 1
        hist = np.full(cap, np.nan)
        _, hp = _f64(hist)
        k = ctypes.c_int32(0)
        st = self.lib.oracle_solve_gmres(1 if pipelined else 0, int(m), n, rpp, cip, vp, bp, xp, rptr,
                                         float(rtol), int(max_iter), hp, cap, ctypes.byref(k))
        kk = int(k.value)
        return Result(x=x, r=r, k=kk, status=STATUS[st], hist=hist[: kk + 1].copy(), trace=None)

    def solve_mixed(self, A, b, x0=None, rtol: float = 1e-10, inner_rtol: float = 1e-4,
                    max_iter: int | None = None, max_outer: int = 50,
                    acc: str = "exact") -> "MixedResult":
        """Iterative refinement in FP64 around FP32 pipelined CG (oracle.c).
        acc: "exact" (inner products exact sums of the FP32 operands, scalars
        in FP64) or "f32" (inner products accumulated in FP32, scalars in FP32)."""
        n = A.n
        if max_iter is None:
            max_iter = 10 * n
        rp, rpp = _i32(A.row_ptr)
        ci, cip = _i32(A.col_idx)
        v, vp = _f64(A.vals)
        b, bp = _f64(b)
        x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        _, xp = _f64(x)
        cap = max_outer + 1
        hist = np.full(cap, np.nan)
        _, hp = _f64(hist)
        inner = np.zeros(cap, dtype=np.int32)
        _, ip = _i32(inner)
        k = ctypes.c_int32(0)
        sw = ctypes.c_int32(0)
        st = self.lib.oracle_solve_mixed(n, rpp, cip, vp, bp, xp, float(rtol), float(inner_rtol),
                                         int(max_iter), int(max_outer), hp, ip, cap,
                                         ctypes.byref(k), ctypes.byref(sw), ACC_MODES[acc])
        J = int(sw.value)
        return MixedResult(x=x, k=int(k.value), sweeps=J, status=STATUS[st],
                           hist=hist[: J + 1].copy(), inner_k=inner[:J].copy())

    def true_residual(self, A, b, x) -> float:
        """||b - A x|| / ||b|| with the oracle's product and compensated dots."""
        ax = self.spmv(A, x)
        r = np.asarray(b, dtype=np.float64) - ax
        bb = self.dot(b, b)
        rr = self.dot(r, r)
        return float(np.sqrt(rr) / np.sqrt(bb)) if bb > 0 else float(np.sqrt(rr))


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def spmv(A, p) -> np.ndarray:
    return default().spmv(A, p)


def dot(a, b) -> float:
    return default().dot(a, b)


def dot_mode(mode: int):
    return default().dot_mode(mode)


def solve(A, b, x0=None, method: str = "cg_pipelined", rtol: float = 1e-8,
          max_iter: int | None = None, trace: bool = False) -> "Result":
    return default().solve(A, b, x0=x0, method=method, rtol=rtol, max_iter=max_iter, trace=trace)


def solve_mixed(A, b, x0=None, rtol: float = 1e-10, inner_rtol: float = 1e-4,
                max_iter: int | None = None, max_outer: int = 50, acc: str = "exact") -> "MixedResult":
    return default().solve_mixed(A, b, x0=x0, rtol=rtol, inner_rtol=inner_rtol,
                                 max_iter=max_iter, max_outer=max_outer, acc=acc)


def solve_gmres(A, b, x0=None, m: int = 30, pipelined: bool = True, rtol: float = 1e-8,
                max_iter: int | None = None) -> "Result":
    return default().solve_gmres(A, b, x0=x0, m=m, pipelined=pipelined, rtol=rtol, max_iter=max_iter)


def true_residual(A, b, x) -> float:
    return default().true_residual(A, b, x)


@dataclass
class Result:
    x: np.ndarray
    r: np.ndarray
    k: int
    status: str
    hist: np.ndarray  # ||r_i||/||b||, i = 0..k
    trace: np.ndarray | None  # (k, stride) per-iteration scalars

    def t(self, name: str) -> np.ndarray:
        return self.trace[:, TRACE_SLOTS[name]]


@dataclass
class MixedResult:
    x: np.ndarray
    k: int              # inner iterations over all sweeps
    sweeps: int         # corrections applied
    status: str
    hist: np.ndarray    # ||b - A x_j||/||b||, j = 0..sweeps
    inner_k: np.ndarray  # inner iterations of each sweep


class TimingOracle:
    """The OpenMP timing build of oracle.c (oracle.build.build_timing): only
    oracle_cg_classical_omp, Algorithm 1 over `threads` threads in static row
    chunks.  Used to time the oracle on the host's cores, never for parity."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.oracle_cg_classical_omp.argtypes = [
            ctypes.c_int32, ctypes.c_int64, i32p, i32p, f64p, f64p, f64p, ctypes.c_double,
            ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        lib.oracle_cg_classical_omp.restype = ctypes.c_int
        self.lib = lib

    def cg_classical(self, A, b, threads: int, x0=None, rtol: float = 1e-8, max_iter: int | None = None):
        """Returns (status, k, x)."""
        rp, rpp = _i32(A.row_ptr)
        ci, cip = _i32(A.col_idx)
        v, vp = _f64(A.vals)
        b, bp = _f64(b)
        x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        _, xp = _f64(x)
        k = ctypes.c_int32(0)
        st = self.lib.oracle_cg_classical_omp(int(threads), A.n, rpp, cip, vp, bp, xp, float(rtol),
                                              int(10 * A.n if max_iter is None else max_iter),
                                              ctypes.byref(k))
        return STATUS[st], int(k.value), x
