"""Python binding of libfk.so (include/fk.h): argument marshalling only.

Every function here forwards to the C ABI function of the same name (without
the ``fk_`` prefix).  Device buffers are torch tensors on the current HIP
device (float64 vectors, int32 index arrays); streams are torch streams.
There is no fallback: if libfk.so cannot be loaded or built, every call
raises.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import numpy as np

from . import build as _build

# fk_status
OK, E_ARG, E_CSR, E_HIP, E_OOM, NOT_CONVERGED, BREAKDOWN, E_STATE = range(8)
STATUS_NAMES = {
    OK: "converged", NOT_CONVERGED: "not_converged", BREAKDOWN: "breakdown",
}
# fk_method
METHODS = {"cg_pipelined": 0, "cg_classical": 1, "bicgstab_pipelined": 2, "bicgstab_classical": 3,
           "cg_mixed": 4, "gmres_pipelined": 5, "gmres_classical": 6, "cg_mixed_f32": 7,
           "cg_pipelined_split": 8, "bicgstab_pipelined_split": 9, "bicgstab_pipelined_2k": 10,
           "cg_pipelined_1k": 11}
# methods that record per-iteration scalars (alpha, beta, omega, <r,r>)
SCALAR_METHODS = ("cg_pipelined", "cg_classical", "bicgstab_pipelined", "bicgstab_classical",
                  "cg_pipelined_split", "bicgstab_pipelined_split", "bicgstab_pipelined_2k", "cg_pipelined_1k")
FLAG_GRAPH = 1
FLAG_PROFILE = 2
FLAG_NO_SMALL = 4
FLAG_SCALARS = 8
PTR_HOST, PTR_DEVICE = 0, 1
KERNEL_KINDS = ("setup", "spmv_dot", "update_dot", "spmv", "dot", "axpy", "small", "residual")
LONG_ROW = 2048


class FkError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


class _Opts(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int32),
        ("rtol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("record_history", ctypes.c_int32),
        ("unroll", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("inner_rtol", ctypes.c_double),
        ("max_outer", ctypes.c_int32),
        ("restart", ctypes.c_int32),
    ]


class _BatchOpts(ctypes.Structure):
    _fields_ = [
        ("rtol", ctypes.c_double),
        ("inner_rtol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("max_outer", ctypes.c_int32),
        ("workgroup", ctypes.c_int32),
        ("lds_rows", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("team", ctypes.c_int32),
        ("teams", ctypes.c_int32),
        ("spin_limit", ctypes.c_int32),
    ]


_lib = None
_lock = threading.Lock()


def library_path() -> str:
    """libfk.so next to this file, or the path in FK_LIBRARY (alternate builds)."""
    return os.environ.get("FK_LIBRARY") or _build.library_path()


def lib():
    """Load libfk.so (building it first if it is absent); raise on failure."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        path = library_path()
        if not os.path.exists(path) and path == _build.library_path():
            _build.build()
        L = ctypes.CDLL(path)  # raises OSError if it cannot be loaded
        vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER
        sig = {
            "fk_csr_create": [i64, i64, vp, vp, vp, i32, vp, P(vp)],
            "fk_csr_destroy": [vp],
            "fk_csr_shape": [vp, P(i64), P(i64)],
            "fk_csr_blocks": [vp, P(i32), P(i32)],
            "fk_csr_layout": [vp, P(i32), P(i64), P(i64)],
            "fk_csr_set_layout": [vp, i32, vp],
            "fk_csr_set_stream": [vp, i32],
            "fk_csr_stream": [vp, P(i32), P(i32)],
            "fk_solver_create": [vp, P(_Opts), vp, P(vp)],
            "fk_solve": [vp, vp, vp],
            "fk_get_iterations": [vp, P(i32)],
            "fk_get_residual": [vp, P(f64)],
            "fk_get_residual_history": [vp, P(f64), i32, P(i32)],
            "fk_get_scalars": [vp, P(f64), i32, P(i32)],
            "fk_get_kernel_times": [vp, P(f64), P(i32), i32],
            "fk_solver_destroy": [vp],
            "fk_solver_uses_small": [vp, P(i32)],
            "fk_get_refinements": [vp, P(i32)],
            "fk_spmv": [vp, vp, vp, P(f64), vp],
            "fk_spmv_time": [vp, vp, vp, i32, i32, P(f64), vp],
            "fk_spmv32": [vp, vp, vp, i32, P(f64), vp],
            "fk_dot": [i64, vp, vp, P(f64), vp],
            "fk_copy": [vp, vp, i64, vp],
            "fk_axpby": [i64, f64, vp, f64, vp, vp, vp],
            "fk_net_num_weights": [i32, i32, P(i64)],
            "fk_net_create": [i32, i32, i32, vp, i64, P(vp)],
            "fk_net_destroy": [vp],
            "fk_net_get_weights": [vp, vp, i64],
            "fk_net_set_weights": [vp, vp, i64],
            "fk_net_forward": [vp, vp, i32, i32, vp, vp, vp, vp, vp],
            "fk_net_guess": [vp, vp, i32, i32, vp, vp, vp, i32, vp, P(i32), vp],
            "fk_net_gradient": [vp, vp, i32, i32, vp, vp, vp, vp, vp, P(f64), vp],
            "fk_net_train_step": [vp, vp, i32, i32, vp, vp, vp, vp, ctypes.c_float, P(f64), vp],
            "fk_batch_create": [i32, vp, i64, vp, vp, vp, i32, vp, P(vp)],
            "fk_batch_destroy": [vp],
            "fk_batch_shape": [vp, P(i32), P(i64), P(i64)],
            "fk_batch_solve": [vp, P(_BatchOpts), vp, vp, vp],
            "fk_batch_results": [vp, vp, vp, vp, vp],
            "fk_solve_noalloc": [vp, P(_Opts), vp, vp, vp, P(i32), P(f64)],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        for name in ("fk_status_str", "fk_last_error", "fk_version"):
            getattr(L, name).restype = ctypes.c_char_p
        L.fk_status_str.argtypes = [ctypes.c_int]
        L.fk_last_error.argtypes = []
        L.fk_version.argtypes = []
        _lib = L
        return L


def exported_symbols() -> list[str]:
    """Names every caller may rely on (the declarations of include/fk.h)."""
    return [
        "fk_csr_create", "fk_csr_destroy", "fk_csr_shape", "fk_csr_blocks", "fk_csr_layout",
        "fk_csr_set_layout", "fk_csr_set_stream", "fk_csr_stream",
        "fk_solver_create", "fk_solve", "fk_get_iterations", "fk_get_residual",
        "fk_get_residual_history", "fk_get_scalars", "fk_get_kernel_times",
        "fk_solver_destroy", "fk_solver_uses_small", "fk_get_refinements", "fk_spmv", "fk_spmv_time",
        "fk_spmv32", "fk_dot",
        "fk_copy",
        "fk_axpby", "fk_net_num_weights", "fk_net_create", "fk_net_destroy", "fk_net_get_weights",
        "fk_net_set_weights", "fk_net_forward", "fk_net_guess", "fk_net_gradient", "fk_net_train_step",
        "fk_batch_create", "fk_batch_destroy", "fk_batch_shape", "fk_batch_solve", "fk_batch_results",
        "fk_solve_noalloc", "fk_status_str", "fk_last_error", "fk_version",
    ]


def _check(status: int, where: str, allowed=(OK,)):
    if status not in allowed:
        msg = lib().fk_last_error().decode(errors="replace")
        raise FkError(status, where, msg)
    return status


def _stream_ptr(stream=None) -> int:
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _dev_f64(t, n=None, name="vector"):
    import torch

    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a torch tensor on a HIP device")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def version() -> str:
    return lib().fk_version().decode()


def status_str(status: int) -> str:
    return lib().fk_status_str(int(status)).decode()


# ------------------------------------------------------------------ matrix

LAYOUTS = {"auto": 0, "row_blocks": 1, "sliced": 2, "sliced16": 3, "slots": 4}


class Matrix:
    """A device-resident CSR matrix (fk_csr handle)."""

    def __init__(self, csr, stream=None, layout: str | None = None):
        """`csr`: object with n, row_ptr, col_idx, vals (numpy host arrays).
        `layout`: None keeps the library's choice; else one of LAYOUTS."""
        L = lib()
        rp = np.ascontiguousarray(csr.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(csr.col_idx, dtype=np.int32)
        va = np.ascontiguousarray(csr.vals, dtype=np.float64)
        h = ctypes.c_void_p()
        st = L.fk_csr_create(int(csr.n), int(ci.size), rp.ctypes.data_as(ctypes.c_void_p),
                             ci.ctypes.data_as(ctypes.c_void_p), va.ctypes.data_as(ctypes.c_void_p),
                             PTR_HOST, ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(h))
        _check(st, "fk_csr_create")
        self._h = h
        self.n = int(csr.n)
        self.nnz = int(ci.size)
        if layout is not None:
            self.set_layout(layout, stream)

    @property
    def handle(self):
        return self._h

    def blocks(self) -> tuple[int, int]:
        nb, lr = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fk_csr_blocks(self._h, ctypes.byref(nb), ctypes.byref(lr)), "fk_csr_blocks")
        return nb.value, lr.value

    def layout(self) -> tuple[str, int]:
        """(layout the products read, entries they read per product)."""
        lay, ent = ctypes.c_int32(), ctypes.c_int64()
        _check(lib().fk_csr_layout(self._h, ctypes.byref(lay), ctypes.byref(ent), None), "fk_csr_layout")
        name = {v: k for k, v in LAYOUTS.items()}[lay.value]
        return name, ent.value

    def matrix_bytes(self) -> int:
        """Bytes of matrix data one FP64 product reads in the current layout."""
        lay, ent, nb = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().fk_csr_layout(self._h, ctypes.byref(lay), ctypes.byref(ent), ctypes.byref(nb)),
               "fk_csr_layout")
        return nb.value

    def set_layout(self, layout: str, stream=None):
        if layout not in LAYOUTS:
            raise ValueError(f"layout must be one of {sorted(LAYOUTS)}")
        st = lib().fk_csr_set_layout(self._h, LAYOUTS[layout], ctypes.c_void_p(_stream_ptr(stream)))
        _check(st, "fk_csr_set_layout")

    def set_stream(self, mode: int):
        """Streaming mode of the sliced products: -1 by size, 0 off, 1 on."""
        _check(lib().fk_csr_set_stream(self._h, int(mode)), "fk_csr_set_stream")

    def stream(self) -> tuple[bool, bool]:
        """(streaming mode on, products in sweep order)."""
        on, sw = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fk_csr_stream(self._h, ctypes.byref(on), ctypes.byref(sw)), "fk_csr_stream")
        return bool(on.value), bool(sw.value)

    def close(self):
        if self._h:
            _check(lib().fk_csr_destroy(self._h), "fk_csr_destroy")
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().fk_csr_destroy(self._h)
        except Exception:
            pass


def spmv(A: Matrix, p, q, dots: bool = False, stream=None):
    """q = A p; with dots=True also returns (<p,q>, <q,q>) from the fused reduction."""
    out = (ctypes.c_double * 2)()
    st = lib().fk_spmv(A.handle, _dev_f64(p, A.n, "p"), _dev_f64(q, A.n, "q"),
                       out if dots else None, ctypes.c_void_p(_stream_ptr(stream)))
    _check(st, "fk_spmv")
    return (out[0], out[1]) if dots else None


SPMV_TIME_MODES = {"product": 0, "fused": 1, "split": 2}


def spmv_time(A: Matrix, p, q, mode: str = "fused", reps: int = 50, stream=None) -> float:
    """Average kernel time in microseconds of q = A p over `reps` launches:
    "product" alone, "fused" with <p,q>, <q,q>, or "split" (product, then a
    separate dot kernel; the pair's time)."""
    n = A.n
    us = ctypes.c_double()
    _check(lib().fk_spmv_time(A.handle, _dev_f64(p, n, "p"), _dev_f64(q, n, "q"), SPMV_TIME_MODES[mode],
                              int(reps), ctypes.byref(us), ctypes.c_void_p(_stream_ptr(stream))),
           "fk_spmv_time")
    return us.value


def spmv32(A: Matrix, p, q, f32acc: bool = False, stream=None) -> tuple[float, float]:
    """q = A p in FP32 (float32 tensors); returns (<p,q>, <q,q>), exact sums of
    the FP32 operands (f32acc False) or FP32 accumulations (f32acc True)."""
    import torch

    for t, nm in ((p, "p"), (q, "q")):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == A.n):
            raise ValueError(f"{nm} must be a contiguous float32 CUDA tensor of {A.n} elements")
    out = (ctypes.c_double * 2)()
    st = lib().fk_spmv32(A.handle, ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                         1 if f32acc else 0, out, ctypes.c_void_p(_stream_ptr(stream)))
    _check(st, "fk_spmv32")
    return out[0], out[1]


def dot(a, b, stream=None) -> float:
    n = a.numel()
    out = ctypes.c_double()
    st = lib().fk_dot(n, _dev_f64(a, n, "a"), _dev_f64(b, n, "b"), ctypes.byref(out),
                      ctypes.c_void_p(_stream_ptr(stream)))
    _check(st, "fk_dot")
    return out.value


def axpby(alpha: float, x, beta: float, y, out, stream=None):
    """out = alpha x + beta y on the device (enqueued, not waited for)."""
    n = out.numel()
    st = lib().fk_axpby(n, float(alpha), _dev_f64(x, n, "x"), float(beta), _dev_f64(y, n, "y"),
                        _dev_f64(out, n, "out"), ctypes.c_void_p(_stream_ptr(stream)))
    _check(st, "fk_axpby")


def copy(dst, src, n_bytes: int, stream=None):
    st = lib().fk_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                       int(n_bytes), ctypes.c_void_p(_stream_ptr(stream)))
    _check(st, "fk_copy")


# ------------------------------------------------------------------ solver

@dataclass
class SolveResult:
    status: str
    k: int
    rel_res: float
    history: np.ndarray | None
    scalars: np.ndarray | None  # (k, 4): alpha, beta, omega, <r,r> tested
    sweeps: int = 0             # cg_mixed: refinement sweeps


class Solver:
    """fk_solver handle: workspace for one matrix, method and option set."""

    def __init__(self, A: Matrix, method: str = "cg_pipelined", rtol: float = 1e-8,
                 max_iter: int | None = None, record_history: bool | int = True, unroll: int = 32,
                 graph: bool = False, profile: bool = False, small: bool = True,
                 inner_rtol: float = 0.0, max_outer: int = 0, restart: int = 0, stream=None,
                 record_scalars: bool = False):
        """small=False forces the multi-kernel path even where the
        single-workgroup solver applies.  inner_rtol, max_outer: options of
        method "cg_mixed" (0 = library defaults 1e-4 and 50); restart: the
        GMRES restart length m (0 = 30).  record_history: True keeps up to
        FK_HISTORY_DEFAULT entries, an int > 1 that many; record_scalars
        also keeps alpha, beta, omega and <r,r> per iteration."""
        import torch

        self.A = A
        if max_iter is None:
            max_iter = min(10 * A.n, 2**31 - 2)
        if graph and stream is None:
            # Stream capture needs a stream other than the legacy default one.
            stream = torch.cuda.Stream()
        self.stream = stream
        flags = ((FLAG_GRAPH if graph else 0) | (FLAG_PROFILE if profile else 0)
                 | (0 if small else FLAG_NO_SMALL) | (FLAG_SCALARS if record_scalars else 0))
        rh = int(record_history) if not isinstance(record_history, bool) else int(record_history)
        o = _Opts(METHODS[method], float(rtol), int(max_iter), rh,
                  int(unroll), flags, float(inner_rtol), int(max_outer), int(restart))
        h = ctypes.c_void_p()
        st = lib().fk_solver_create(A.handle, ctypes.byref(o), ctypes.c_void_p(_stream_ptr(stream)),
                                    ctypes.byref(h))
        _check(st, "fk_solver_create")
        self._h = h
        self.method = method
        self.max_iter = int(max_iter)
        self.record_history = bool(record_history)

    def solve(self, b, x) -> int:
        """Run fk_solve; returns the fk_status (OK, NOT_CONVERGED or BREAKDOWN)."""
        if self.stream is not None:
            import torch

            # b and x were produced on the caller's stream.
            self.stream.wait_stream(torch.cuda.current_stream())
        st = lib().fk_solve(self._h, _dev_f64(b, self.A.n, "b"), _dev_f64(x, self.A.n, "x"))
        return _check(st, "fk_solve", allowed=(OK, NOT_CONVERGED, BREAKDOWN))

    def uses_small(self) -> bool:
        v = ctypes.c_int32()
        _check(lib().fk_solver_uses_small(self._h, ctypes.byref(v)), "fk_solver_uses_small")
        return bool(v.value)

    def iterations(self) -> int:
        k = ctypes.c_int32()
        _check(lib().fk_get_iterations(self._h, ctypes.byref(k)), "fk_get_iterations")
        return k.value

    def residual(self) -> float:
        r = ctypes.c_double()
        _check(lib().fk_get_residual(self._h, ctypes.byref(r)), "fk_get_residual")
        return r.value

    def refinements(self) -> int:
        v = ctypes.c_int32()
        _check(lib().fk_get_refinements(self._h, ctypes.byref(v)), "fk_get_refinements")
        return v.value

    def history(self) -> np.ndarray:
        k = self.refinements() if self.method in ("cg_mixed", "cg_mixed_f32") else self.iterations()
        buf = np.empty(k + 1)
        ln = ctypes.c_int32()
        _check(lib().fk_get_residual_history(self._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             k + 1, ctypes.byref(ln)), "fk_get_residual_history")
        return buf[: ln.value]

    def scalars(self) -> np.ndarray:
        k = self.iterations()
        buf = np.empty((max(k, 1), 4))
        ln = ctypes.c_int32()
        _check(lib().fk_get_scalars(self._h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    k, ctypes.byref(ln)), "fk_get_scalars")
        return buf[: ln.value]

    def kernel_times(self) -> dict[str, tuple[float, int]]:
        n = len(KERNEL_KINDS)
        us = (ctypes.c_double * n)()
        cnt = (ctypes.c_int32 * n)()
        _check(lib().fk_get_kernel_times(self._h, us, cnt, n), "fk_get_kernel_times")
        return {name: (us[i], cnt[i]) for i, name in enumerate(KERNEL_KINDS)}

    def close(self):
        if self._h:
            _check(lib().fk_solver_destroy(self._h), "fk_solver_destroy")
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().fk_solver_destroy(self._h)
        except Exception:
            pass


def solve(A: Matrix, b, x, method: str = "cg_pipelined", rtol: float = 1e-8,
          max_iter: int | None = None, record_history: bool = True, **kw) -> SolveResult:
    """One-shot solve of A x = b on the device (x holds x0 on entry)."""
    want_scal = bool(record_history) and method in SCALAR_METHODS
    S = Solver(A, method=method, rtol=rtol, max_iter=max_iter, record_history=record_history,
               record_scalars=want_scal, **kw)
    try:
        st = S.solve(b, x)
        hist = S.history() if record_history else None
        scal = S.scalars() if want_scal else None
        return SolveResult(STATUS_NAMES[st], S.iterations(), S.residual(), hist, scal,
                           S.refinements())
    finally:
        S.close()


NOALLOC_MAX_N = 1048576  # FK_NOALLOC_MAX_N


def solve_noalloc(A: Matrix, b, x, rtol: float = 1e-8, max_iter: int | None = None, unroll: int = 32,
                  small: bool = True, stream=None) -> SolveResult:
    """fk_solve_noalloc: pipelined CG without a solver handle, its work
    memory in the library's static per-device array (nothing allocated).
    x holds x0 on entry.  Returns status, k and ||r_k||/||b|| (no history)."""
    if max_iter is None:
        max_iter = min(10 * A.n, 2**31 - 2)
    o = _Opts(METHODS["cg_pipelined"], float(rtol), int(max_iter), 0, int(unroll),
              0 if small else FLAG_NO_SMALL, 0.0, 0, 0)
    k = ctypes.c_int32()
    rel = ctypes.c_double()
    st = lib().fk_solve_noalloc(A.handle, ctypes.byref(o), _dev_f64(b, A.n, "b"), _dev_f64(x, A.n, "x"),
                                ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(k), ctypes.byref(rel))
    _check(st, "fk_solve_noalloc", allowed=(OK, NOT_CONVERGED, BREAKDOWN))
    return SolveResult(STATUS_NAMES[st], k.value, rel.value, None, None, 0)


# ------------------------------------------------------- warm-start network

def net_num_weights(layers: int, channels: int = 16) -> int:
    c = ctypes.c_int64()
    _check(lib().fk_net_num_weights(int(layers), int(channels), ctypes.byref(c)), "fk_net_num_weights")
    return c.value


NET_ACTIVATIONS = {"relu": 0, "linear": 1}


class Net:
    """fk_net handle: the BF16 convolutional initial-guess network."""

    def __init__(self, layers: int, weights, channels: int = 16, activation: str = "relu"):
        w = np.ascontiguousarray(weights, dtype=np.float32)
        h = ctypes.c_void_p()
        st = lib().fk_net_create(int(layers), int(channels), NET_ACTIVATIONS[activation],
                                 w.ctypes.data_as(ctypes.c_void_p), w.size, ctypes.byref(h))
        _check(st, "fk_net_create")
        self._h = h
        self.layers = int(layers)
        self.activation = activation
        self.count = int(w.size)

    def weights(self) -> np.ndarray:
        out = np.empty(self.count, dtype=np.float32)
        _check(lib().fk_net_get_weights(self._h, out.ctypes.data_as(ctypes.c_void_p), self.count),
               "fk_net_get_weights")
        return out

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(lib().fk_net_set_weights(self._h, w.ctypes.data_as(ctypes.c_void_p), w.size),
               "fk_net_set_weights")

    def forward(self, A: Matrix, nx: int, ny: int, b, um, um1, y, stream=None):
        import torch

        if not isinstance(y, torch.Tensor) or y.dtype != torch.float32 or y.numel() != A.n:
            raise TypeError("y must be a float32 device tensor of n entries")
        st = lib().fk_net_forward(self._h, A.handle, int(nx), int(ny), _dev_f64(b, A.n, "b"),
                                  _dev_f64(um, A.n, "u_m"), _dev_f64(um1, A.n, "u_m1"),
                                  ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(_stream_ptr(stream)))
        _check(st, "fk_net_forward")

    def guess(self, A: Matrix, nx: int, ny: int, b, um, um1, x0, passes: int = 1, report: bool = False,
              stream=None):
        """x0 = extrapolation corrected `passes` times by the network, with the
        fallback to u_m.  With report=True waits and returns True when it fell back."""
        fb = ctypes.c_int32(0)
        st = lib().fk_net_guess(self._h, A.handle, int(nx), int(ny), _dev_f64(b, A.n, "b"),
                                _dev_f64(um, A.n, "u_m"), _dev_f64(um1, A.n, "u_m1"), int(passes),
                                _dev_f64(x0, A.n, "x0"), ctypes.byref(fb) if report else None,
                                ctypes.c_void_p(_stream_ptr(stream)))
        _check(st, "fk_net_guess")
        return bool(fb.value) if report else None

    def gradient(self, A: Matrix, nx: int, ny: int, b, um, um1, unext, stream=None):
        g = np.empty(self.count, dtype=np.float32)
        loss = ctypes.c_double()
        st = lib().fk_net_gradient(self._h, A.handle, int(nx), int(ny), _dev_f64(b, A.n, "b"),
                                   _dev_f64(um, A.n, "u_m"), _dev_f64(um1, A.n, "u_m1"),
                                   _dev_f64(unext, A.n, "u_next"), g.ctypes.data_as(ctypes.c_void_p),
                                   ctypes.byref(loss), ctypes.c_void_p(_stream_ptr(stream)))
        _check(st, "fk_net_gradient")
        return g, loss.value

    def train_step(self, A: Matrix, nx: int, ny: int, b, um, um1, unext, lr: float,
                   report: bool = False, stream=None):
        loss = ctypes.c_double()
        st = lib().fk_net_train_step(self._h, A.handle, int(nx), int(ny), _dev_f64(b, A.n, "b"),
                                     _dev_f64(um, A.n, "u_m"), _dev_f64(um1, A.n, "u_m1"),
                                     _dev_f64(unext, A.n, "u_next"), ctypes.c_float(lr),
                                     ctypes.byref(loss) if report else None,
                                     ctypes.c_void_p(_stream_ptr(stream)))
        _check(st, "fk_net_train_step")
        return loss.value if report else None

    def close(self):
        if self._h:
            _check(lib().fk_net_destroy(self._h), "fk_net_destroy")
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().fk_net_destroy(self._h)
        except Exception:
            pass


# ------------------------------------------------------------------- batch

BATCH_STATUS = {0: "converged", 1: "not_converged", 2: "breakdown", 3: "unsolved"}


@dataclass
class BatchResult:
    status: np.ndarray      # per system: 0 converged, 1 not converged, 2 breakdown
    iterations: np.ndarray  # inner iterations over all sweeps
    sweeps: np.ndarray
    rel_res: np.ndarray     # ||b_s - A_s x_s|| / ||b_s|| of the last residual


class Batch:
    """fk_batch handle: independent systems stored as one block-diagonal CSR."""

    def __init__(self, csr, sys_ptr, stream=None):
        L = lib()
        sp = np.ascontiguousarray(sys_ptr, dtype=np.int64)
        rp = np.ascontiguousarray(csr.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(csr.col_idx, dtype=np.int32)
        va = np.ascontiguousarray(csr.vals, dtype=np.float64)
        h = ctypes.c_void_p()
        st = L.fk_batch_create(int(sp.size - 1), sp.ctypes.data_as(ctypes.c_void_p), int(ci.size),
                               rp.ctypes.data_as(ctypes.c_void_p), ci.ctypes.data_as(ctypes.c_void_p),
                               va.ctypes.data_as(ctypes.c_void_p), PTR_HOST,
                               ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(h))
        _check(st, "fk_batch_create")
        self._h = h
        self.count = int(sp.size - 1)
        self.n = int(sp[-1])
        self.sys_ptr = sp

    def solve(self, b, x, rtol: float = 1e-10, inner_rtol: float = 0.0, max_iter: int = 0,
              max_outer: int = 0, workgroup: int = 0, lds_rows: int = 0, graph: bool = False, stream=None,
              team: int = 0, teams: int = 0, spin_limit: int = 0):
        o = _BatchOpts(float(rtol), float(inner_rtol), int(max_iter), int(max_outer), int(workgroup),
                       int(lds_rows), FLAG_GRAPH if graph else 0, int(team), int(teams), int(spin_limit))
        st = lib().fk_batch_solve(self._h, ctypes.byref(o), _dev_f64(b, self.n, "b"),
                                  _dev_f64(x, self.n, "x"), ctypes.c_void_p(_stream_ptr(stream)))
        _check(st, "fk_batch_solve")

    def results(self) -> BatchResult:
        c = self.count
        st = np.empty(c, np.int32)
        it = np.empty(c, np.int32)
        sw = np.empty(c, np.int32)
        rel = np.empty(c, np.float64)
        _check(lib().fk_batch_results(self._h, st.ctypes.data_as(ctypes.c_void_p),
                                      it.ctypes.data_as(ctypes.c_void_p), sw.ctypes.data_as(ctypes.c_void_p),
                                      rel.ctypes.data_as(ctypes.c_void_p)), "fk_batch_results")
        return BatchResult(st, it, sw, rel)

    def close(self):
        if self._h:
            _check(lib().fk_batch_destroy(self._h), "fk_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().fk_batch_destroy(self._h)
        except Exception:
            pass
