"""First end-to-end GPU parity checks (HIP path vs the CPU oracle)."""
import numpy as np
import pytest

import oracle
from paper_1410_4054_amd import fk, problems as P

pytestmark = pytest.mark.gpu


def _t(a, device):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)


@pytest.mark.parametrize("name,method", [
    ("poisson2d_32", "cg_pipelined"), ("poisson2d_32", "cg_classical"),
    ("convdiff2d_64", "bicgstab_pipelined"), ("convdiff2d_64", "bicgstab_classical"),
    ("poisson3d_24", "cg_pipelined"),
])
def test_solve_matches_oracle(name, method, device):
    A, b, x0 = P.workload(name)
    print(f"\n[case] {name} {method}", flush=True)
    ref = oracle.solve(A, b, method=method, rtol=1e-8)
    M = fk.Matrix(A)
    bd, xd = _t(b, device), _t(x0, device)
    res = fk.solve(M, bd, xd, method=method, rtol=1e-8)
    x = xd.cpu().numpy()
    print(f"  gpu k={res.k} {res.status} oracle k={ref.k} {ref.status}", flush=True)
    assert res.status == ref.status == "converged"
    assert res.k == ref.k
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    print(f"  rel err {err:.3e}; hist identical: {np.array_equal(res.history, ref.hist)}", flush=True)
    assert err <= 1e-10
    np.testing.assert_allclose(res.history, ref.hist, rtol=1e-12, atol=0)


@pytest.mark.parametrize("nnz_row", [4, 28])
def test_spmv_bitwise(nnz_row, device):
    A = P.random_csr(5000, nnz_row, seed=nnz_row, empty_rows=17, long_rows={3: 3000, 4000: 9000})
    rng = np.random.default_rng(1)
    p = rng.uniform(-1, 1, A.n)
    M = fk.Matrix(A)
    nb, lr = M.blocks()
    assert lr == 2
    pd = _t(p, device)
    qd = _t(np.zeros(A.n), device)
    dots = fk.spmv(M, pd, qd, dots=True)
    q = qd.cpu().numpy()
    ref = oracle.spmv(A, p)
    short = np.diff(A.row_ptr) <= fk.LONG_ROW
    assert np.array_equal(q[short], ref[short])
    np.testing.assert_allclose(q[~short], ref[~short], rtol=1e-13)
    assert dots[0] == oracle.dot(p, q) and dots[1] == oracle.dot(q, q)


def test_dot(device):
    rng = np.random.default_rng(5)
    for n in [1, 7, 1000, 123457]:
        a, b = rng.standard_normal(n), rng.standard_normal(n)
        assert fk.dot(_t(a, device), _t(b, device)) == oracle.dot(a, b)
