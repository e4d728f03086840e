"""Write the stored expected values of the full-size parity tests.

Calls only the CPU oracle (oracle/) and the seeded input generators; never
the GPU library.  For each case it stores the iteration count, status, the
residual history ||r_i||/||b|| (all of it, as exact hex floats), the
SHA-256 of the whole iterate's bytes (float64, little-endian) with its
2-norm as an exact hex float (a machine-independent sum), and the iterate at 4099 evenly spaced indices
(a readable sample of the same vector).

    python tests/golden/make_golden.py            # all cases
    python tests/golden/make_golden.py NAME ...   # selected cases
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1410_4054_amd import problems as P  # noqa: E402

# name -> (workload, method, rtol, max_iter)
CASES = {
    "poisson3d_128_cg_pipelined": ("poisson3d_128", "cg_pipelined", 1e-8, None),
    "poisson3d_128_cg_classical": ("poisson3d_128", "cg_classical", 1e-8, None),
    "convdiff2d_1024_bicgstab_pipelined": ("convdiff2d_1024", "bicgstab_pipelined", 1e-8, None),
    "convdiff2d_1024_bicgstab_pipelined_30": ("convdiff2d_1024", "bicgstab_pipelined", 0.0, 30),
    "poisson3d_128_cg_pipelined_30": ("poisson3d_128", "cg_pipelined", 0.0, 30),
    # FP64 iterative refinement around FP32 pipelined CG (inner_rtol 1e-4)
    "poisson3d_128_cg_mixed": ("poisson3d_128", "cg_mixed", 1e-10, None),
}
INNER_RTOL = 1e-4
NSAMPLES = 4099


def x_norm(x) -> float:
    """||x||_2 from the correctly rounded sum of the rounded squares (math.fsum):
    the same bits on every machine, unlike a BLAS norm."""
    import math

    x = np.asarray(x, dtype=np.float64)
    return math.sqrt(math.fsum((x * x).tolist()))


def x_sha256(x) -> str:
    """SHA-256 of a float64 vector's bytes, little-endian."""
    return hashlib.sha256(np.ascontiguousarray(x, dtype="<f8").tobytes()).hexdigest()


def sample_indices(n: int) -> np.ndarray:
    return np.unique(np.linspace(0, n - 1, NSAMPLES).round().astype(np.int64))


def make(name: str) -> dict:
    workload, method, rtol, max_iter = CASES[name]
    A, b, x0 = P.workload(workload)
    t0 = time.time()
    extra = {}
    if method == "cg_mixed":
        res = oracle.solve_mixed(A, b, x0=x0, rtol=rtol, inner_rtol=INNER_RTOL, max_iter=max_iter)
        extra = {"inner_rtol": INNER_RTOL, "sweeps": res.sweeps,
                 "inner_k": [int(k) for k in res.inner_k]}
    else:
        res = oracle.solve(A, b, x0=x0, method=method, rtol=rtol, max_iter=max_iter)
    dt = time.time() - t0
    idx = sample_indices(A.n)
    return extra | {
        "case": name,
        "workload": workload,
        "method": method,
        "rtol": rtol,
        "max_iter": max_iter,
        "n": A.n,
        "nnz": A.nnz,
        "status": res.status,
        "k": res.k,
        "history_hex": [float(h).hex() for h in res.hist],
        "x_index": idx.tolist(),
        "x_sample_hex": [float(v).hex() for v in res.x[idx]],
        "x_norm": float(np.linalg.norm(res.x)),
        "x_norm_hex": x_norm(res.x).hex(),
        "x_sha256": x_sha256(res.x),
        "oracle_seconds": round(dt, 2),
        "made_by": "tests/golden/make_golden.py (CPU oracle only)",
    }


def path_for(name: str) -> str:
    return os.path.join(HERE, f"{name}.json")


def load(name: str) -> dict:
    with open(path_for(name)) as fh:
        return json.load(fh)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for nm in names:
        g = make(nm)
        with open(path_for(nm), "w") as fh:
            json.dump(g, fh)
        print(f"{nm}: k={g['k']} {g['status']} ({g['oracle_seconds']} s)", flush=True)
