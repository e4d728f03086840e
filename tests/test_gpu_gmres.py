"""Restarted GMRES(m) (Algorithms 5 and 6) through the C ABI against the
oracle's GMRES on the same seeded inputs.

Inner products are exact products summed almost exactly and rounded once on
both sides, the Gram-Schmidt updates and the x update are the same
expressions in the same order, and the triangular solve is the same back
substitution, so iteration counts, histories and iterates must agree
exactly."""
import numpy as np
import pytest

import oracle
from gpu_util import dev, gpu_solve, host, rel, require_layout
from paper_1410_4054_amd import fk, problems as P

pytestmark = pytest.mark.gpu


def _nonsym(n, seed):
    rng = np.random.default_rng(seed)
    return P.dense_to_csr(np.eye(n) * 4 + rng.uniform(-0.5, 0.5, (n, n)))


WORKLOADS = {
    "convdiff2d_32": lambda: P.workload("convdiff2d_32"),
    "convdiff2d_45": lambda: P.workload("convdiff2d_45"),
    "poisson2d_24": lambda: P.workload("poisson2d_24"),
    "nonsym_dense_70": lambda: (_nonsym(70, 4), P.rhs_uniform(70, 5), np.zeros(70)),
}
METHODS = {"gmres_pipelined": True, "gmres_classical": False}


def run(A, b, x0, method, m, rtol=1e-8, max_iter=None, **kw):
    res, x = gpu_solve(A, b, x0, method=method, rtol=rtol, max_iter=max_iter, restart=m, **kw)
    ref = oracle.solve_gmres(A, b, x0=x0, m=m, pipelined=METHODS[method], rtol=rtol, max_iter=max_iter)
    return res, x, ref


def assert_same(res, x, ref, label):
    assert res.status == ref.status, (label, res.status, ref.status)
    assert res.k == ref.k, (label, res.k, ref.k)
    assert np.array_equal(res.history, ref.hist), (label, np.abs(res.history - ref.hist).max())
    assert np.array_equal(x, ref.x), (label, rel(x, ref.x))


@pytest.mark.parametrize("layout", ["row_blocks", "sliced", "sliced16", "slots"])
@pytest.mark.parametrize("m", [5, 30])
@pytest.mark.parametrize("method", list(METHODS))
@pytest.mark.parametrize("wl", list(WORKLOADS))
def test_gmres_matches_oracle(wl, method, m, layout, device):
    A, b, x0 = WORKLOADS[wl]()
    require_layout(A, layout)
    print(f"\n[case] {wl} {method} m={m} n={A.n} layout={layout}", flush=True)
    res, x, ref = run(A, b, x0, method, m, layout=layout)
    assert_same(res, x, ref, f"{wl}/{method}/{m}")
    assert ref.status == "converged"
    assert oracle.true_residual(A, b, x) <= 1e-8


@pytest.mark.parametrize("method", list(METHODS))
def test_gmres_fixed_iterations_and_warm_start(method, device):
    A, b, _ = P.workload("convdiff2d_45")
    x0 = np.random.default_rng(3).uniform(-1, 1, A.n)
    for k in (1, 2, 7, 13, 40):
        res, x, ref = run(A, b, x0, method, 10, rtol=0.0, max_iter=k)
        assert_same(res, x, ref, f"k={k}")
        assert res.status == "not_converged" and res.k == k


def test_gmres_edge_cases(device):
    """b = 0, lambda I, an exact start, three distinct eigenvalues, n = 1."""
    for method in METHODS:
        A, b, _ = P.workload("convdiff2d_32")
        z, zx = gpu_solve(A, np.zeros(A.n), np.ones(A.n), method=method, restart=8)
        assert z.status == "converged" and z.k == 0 and not zx.any()
        I = P.scaled_identity(9, 2.0)
        res, x, ref = run(I, np.arange(1.0, 10.0), np.zeros(9), method, 5, rtol=1e-12)
        assert_same(res, x, ref, "lambda I")
        assert res.k == 1
        n = 24
        rng = np.random.default_rng(22)
        S = np.eye(n) + 0.2 * rng.standard_normal((n, n))
        M = S @ np.diag(np.repeat([1.0, 2.5, 4.0], n // 3)) @ np.linalg.inv(S)
        Am = P.dense_to_csr(M)
        bm = rng.standard_normal(n)
        res, x, ref = run(Am, bm, np.zeros(n), method, 10, rtol=1e-10)
        assert_same(res, x, ref, "3 eigenvalues")
        assert res.k == 3
        one = P.scaled_identity(1, 3.0)
        res, x, ref = run(one, np.array([2.0]), np.zeros(1), method, 4, rtol=1e-12)
        assert_same(res, x, ref, "n=1")
        xs = np.linalg.solve(M, bm)
        res, x, ref = run(Am, bm, xs, method, 10, rtol=1e-8)
        assert_same(res, x, ref, "exact start")
        assert res.k == 0


def test_gmres_api(device):
    A, b, _ = P.workload("convdiff2d_32")
    M = fk.Matrix(A)
    S = fk.Solver(M, method="gmres_pipelined", rtol=1e-8, restart=12, profile=True)
    bd, xd = dev(b), dev(np.zeros(A.n))
    assert S.solve(bd, xd) == fk.OK
    kt = S.kernel_times()
    k = S.iterations()
    # every cycle enqueues m steps; steps after the cycle ended return at once
    assert k <= kt["spmv_dot"][1] and kt["spmv_dot"][1] % 12 == 0
    assert kt["update_dot"][1] == 2 * kt["spmv_dot"][1]
    with pytest.raises(fk.FkError):
        S.scalars()
    S.close()
    for bad in (-1, 65):
        with pytest.raises(fk.FkError):
            fk.Solver(M, method="gmres_pipelined", restart=bad)


@pytest.mark.parametrize("method", list(METHODS))
def test_gmres_full_size_fixed(method, device):
    """1024^2 convection-diffusion, GMRES(30), 60 iterations (two cycles) in
    the benchmark's launch configuration, against the oracle run live."""
    A, b, x0 = P.workload("convdiff2d_1024")
    print(f"\n[case] convdiff2d_1024 {method} 60 iterations", flush=True)
    res, x, ref = run(A, b, x0, method, 30, rtol=0.0, max_iter=60)
    assert_same(res, x, ref, "1024^2")
