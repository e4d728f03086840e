"""The benchmark workloads at full size, in the benchmark's launch
configuration, against values stored by tests/golden/make_golden.py (CPU
oracle only): iteration count, the whole residual history, the whole
iterate (SHA-256 of its bytes: the GPU reproduces the oracle's iterate bit
for bit) and its norm as an exact hex float, and the true residual of the
GPU iterate computed by the oracle's product."""
import numpy as np
import pytest

import oracle
from golden.make_golden import load, x_norm, x_sha256
from gpu_util import gpu_solve
from paper_1410_4054_amd import problems as P

pytestmark = pytest.mark.gpu

NAMES = ["poisson3d_128_cg_pipelined", "poisson3d_128_cg_classical",
         "poisson3d_128_cg_pipelined_30", "convdiff2d_1024_bicgstab_pipelined",
         "convdiff2d_1024_bicgstab_pipelined_30"]
# (stored case, GPU method): the two-kernel schedule of Algorithm 4 and the
# one-kernel schedule of Algorithm 2 must reproduce the stored iterates of
# the schedules the oracle's values were written for.
CASES = [(name, None) for name in NAMES] + \
        [("convdiff2d_1024_bicgstab_pipelined", "bicgstab_pipelined_2k"),
         ("convdiff2d_1024_bicgstab_pipelined_30", "bicgstab_pipelined_2k"),
         ("poisson3d_128_cg_pipelined", "cg_pipelined_1k"),
         ("poisson3d_128_cg_pipelined_30", "cg_pipelined_1k")]
_inputs = {}


def inputs(workload):
    if workload not in _inputs:
        _inputs.clear()
        _inputs[workload] = P.workload(workload)
    return _inputs[workload]


@pytest.mark.parametrize("name,method", CASES, ids=[f"{n}-{m or 'stored'}" for n, m in CASES])
def test_full_size_against_oracle(name, method, device):
    g = load(name)
    A, b, x0 = inputs(g["workload"])
    method = method or g["method"]
    print(f"\n[case] {name} {method} n={A.n} nnz={A.nnz}", flush=True)
    res, x = gpu_solve(A, b, x0, method=method, rtol=g["rtol"], max_iter=g["max_iter"])
    hist = np.array([float.fromhex(h) for h in g["history_hex"]])
    assert res.status == g["status"] and res.k == g["k"], (res.status, res.k, g["k"])
    assert np.array_equal(res.history, hist)
    idx = np.array(g["x_index"])
    xs = np.array([float.fromhex(h) for h in g["x_sample_hex"]])
    assert np.array_equal(x[idx], xs)
    assert x_sha256(x) == g["x_sha256"]
    assert x_norm(x).hex() == g["x_norm_hex"]
    if g["status"] == "converged":
        assert oracle.true_residual(A, b, x) <= g["rtol"] * 1.5


def test_config1_full_solve(device):
    """2D Poisson 32x32 with b from seed 0: the oracle runs live."""
    A, b, x0 = P.workload("poisson2d_32")
    ref = oracle.solve(A, b, method="cg_pipelined", rtol=1e-8)
    res, x = gpu_solve(A, b, method="cg_pipelined", rtol=1e-8)
    assert res.k == ref.k == 101
    assert np.array_equal(res.history, ref.hist)
    assert np.abs(x - ref.x).max() <= 1e-10 * np.abs(ref.x).max()
