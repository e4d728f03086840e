"""Helpers shared by the GPU tests (device transfer and solver calls)."""
from __future__ import annotations

import numpy as np

from paper_1410_4054_amd import fk


def dev(a, device="cuda"):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device).clone()


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def rel(a, b) -> float:
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def require_layout(A, layout):
    """Skip the test when a forced slot layout does not apply to A: the
    library refuses it with FK_E_ARG (test_gpu_kernels pins when it must)."""
    if layout != "slots":
        return
    import pytest

    M = fk.Matrix(A)
    try:
        M.set_layout("slots")
    except fk.FkError as e:
        if e.status != fk.E_ARG:
            raise
        pytest.skip("the slot layout does not apply to this matrix")
    finally:
        M.close()


def gpu_solve(A, b, x0=None, method="cg_pipelined", rtol=1e-8, max_iter=None, matrix=None, layout=None,
              **kw):
    """Solve on the device through the C ABI; returns (SolveResult, x as numpy).
    `layout` forces the layout of the products (None: the library's choice)."""
    M = matrix or fk.Matrix(A, layout=layout)
    bd = dev(b)
    xd = dev(np.zeros(A.n) if x0 is None else x0)
    res = fk.solve(M, bd, xd, method=method, rtol=rtol, max_iter=max_iter, **kw)
    return res, host(xd)
