"""Iterative refinement in FP64 around the FP32 pipelined CG (method
"cg_mixed") through the C ABI, against the oracle's refinement
(oracle.solve_mixed) on the same seeded inputs.

The FP32 kernels round every product, row sum and vector update to FP32 as
the oracle does, and the inner products are exact products summed almost
exactly and rounded once on both sides, so sweeps, inner iteration counts,
the residual history and the iterate must agree exactly.  The error of the
result against the FP64 solver's solution is stated per case."""
import numpy as np
import pytest
import scipy.sparse

import oracle
from golden.make_golden import load, x_sha256
from gpu_util import dev, host, rel, require_layout
from paper_1410_4054_amd import fk, problems as P

pytestmark = pytest.mark.gpu


def _shifted_laplacian(n, seed):
    """A 2D Laplacian plus a random nonnegative diagonal (the uneven batch's systems)."""
    rng = np.random.default_rng(seed)
    shift = rng.uniform(0.0, 0.1, n * n)
    b = rng.uniform(-1.0, 1.0, n * n)
    return P.poisson2d(n, diag_shift=shift), b, np.zeros(n * n)


WORKLOADS = {
    "poisson2d_32": lambda: P.workload("poisson2d_32"),
    "poisson2d_37": lambda: P.workload("poisson2d_37"),
    "poisson3d_24": lambda: P.workload("poisson3d_24"),
    "heat2d_48": lambda: P.workload("heat2d_48"),
    "shifted2d_45": lambda: _shifted_laplacian(45, 7),
    "spd_dense_60": lambda: (P.dense_to_csr(P.random_spd_dense(60, 300.0, seed=2)),
                             P.rhs_uniform(60, 3), np.zeros(60)),
    "random_spd_csr": lambda: _random_spd_csr(3000, 11),
}


def _random_spd_csr(n, seed):
    """Symmetric random sparsity with empty off-diagonal rows and a long
    row, made SPD by diagonal dominance."""
    R = P.random_csr(n, 4, seed=seed, empty_rows=7, long_rows={17: 2600}).to_scipy()
    S = abs(R + R.T).tocsr()
    S.setdiag(0.0)
    S.eliminate_zeros()
    d = np.asarray(abs(S).sum(axis=1)).ravel() + 1.0
    M = (-S + scipy.sparse.diags(d)).tocsr()
    M.sort_indices()
    A = P.Csr(n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))
    return A, P.rhs_uniform(n, seed), np.zeros(n)


def mixed_solve(A, b, x0=None, rtol=1e-10, inner_rtol=1e-4, max_iter=None, max_outer=0, layout=None,
                **kw):
    M = fk.Matrix(A, layout=layout)
    bd = dev(b)
    xd = dev(np.zeros(A.n) if x0 is None else x0)
    res = fk.solve(M, bd, xd, method="cg_mixed", rtol=rtol, max_iter=max_iter,
                   inner_rtol=inner_rtol, max_outer=max_outer, **kw)
    return res, host(xd)


def assert_same(res, x, ref, label=""):
    assert res.status == ref.status, (label, res.status, ref.status)
    assert res.sweeps == ref.sweeps, (label, res.sweeps, ref.sweeps)
    assert res.k == ref.k, (label, res.k, ref.k, ref.inner_k)
    assert np.array_equal(res.history, ref.hist), (label, res.history, ref.hist)
    assert np.array_equal(x, ref.x), (label, rel(x, ref.x))


@pytest.mark.parametrize("layout", ["row_blocks", "sliced", "sliced16", "slots"])
@pytest.mark.parametrize("wl", list(WORKLOADS))
def test_mixed_matches_oracle(wl, layout, device):
    A, b, x0 = WORKLOADS[wl]()
    require_layout(A, layout)
    print(f"\n[case] mixed {wl} n={A.n} nnz={A.nnz} layout={layout}", flush=True)
    ref = oracle.solve_mixed(A, b, x0=x0, rtol=1e-10, inner_rtol=1e-4)
    res, x = mixed_solve(A, b, x0, layout=layout)
    assert_same(res, x, ref, wl)
    assert ref.status == "converged"
    # Error against the FP64 solver's solution (pipelined CG to 1e-13).
    x64 = oracle.solve(A, b, method="cg_pipelined", rtol=1e-13).x
    err = rel(x, x64)
    print(f"[result] {wl}: sweeps={res.sweeps} inner k={res.k} "
          f"||x - x_fp64||/||x_fp64|| = {err:.2e} true residual "
          f"{oracle.true_residual(A, b, x):.2e}", flush=True)
    assert oracle.true_residual(A, b, x) <= 1e-10
    assert err <= 1e-7


@pytest.mark.parametrize("inner_rtol", [1e-2, 1e-6])
@pytest.mark.parametrize("unroll,graph", [(1, False), (7, False), (16, True)])
def test_mixed_driver_modes(inner_rtol, unroll, graph, device):
    """Batch size, graph replay and the inner tolerance change only how the
    work is enqueued or how it is split into sweeps: every run equals the
    oracle's for the same options."""
    A, b, x0 = P.workload("poisson3d_24")
    ref = oracle.solve_mixed(A, b, rtol=1e-11, inner_rtol=inner_rtol)
    res, x = mixed_solve(A, b, rtol=1e-11, inner_rtol=inner_rtol, unroll=unroll, graph=graph)
    assert_same(res, x, ref, f"u{unroll} g{graph} i{inner_rtol}")


def test_mixed_warm_start(device):
    A, b, _ = P.workload("heat2d_48")
    x0 = np.random.default_rng(5).uniform(-1, 1, A.n)
    ref = oracle.solve_mixed(A, b, x0=x0, rtol=1e-10)
    res, x = mixed_solve(A, b, x0)
    assert_same(res, x, ref, "warm")


def test_mixed_edge_cases(device):
    """b = 0; an inner tolerance >= 1 (no inner step); limits on inner
    iterations and on sweeps; n = 1; the exact-in-FP32 identity."""
    A, b, _ = P.workload("poisson2d_16")
    z_ref = oracle.solve_mixed(A, np.zeros(A.n), x0=np.ones(A.n))
    z, zx = mixed_solve(A, np.zeros(A.n), np.ones(A.n))
    assert z.status == z_ref.status == "converged" and z.k == 0 and not zx.any()
    for kw in ({"inner_rtol": 2.0}, {"max_iter": 5}, {"max_iter": 40}, {"max_outer": 1},
               {"inner_rtol": 0.5, "max_outer": 3}):
        ref = oracle.solve_mixed(A, b, rtol=1e-10, **{"inner_rtol": 1e-4, **kw})
        res, x = mixed_solve(A, b, rtol=1e-10, **{"inner_rtol": 1e-4, **kw})
        assert_same(res, x, ref, str(kw))
        assert res.status == "not_converged"
    one = P.scaled_identity(1, 3.0)
    ref = oracle.solve_mixed(one, np.array([2.0]), rtol=1e-12)
    res, x = mixed_solve(one, np.array([2.0]), rtol=1e-12)
    assert_same(res, x, ref, "n=1")
    I4 = P.scaled_identity(12, 4.0)
    bi = np.arange(-6.0, 6.0) / 8.0 + 0.03125
    res, x = mixed_solve(I4, bi, rtol=1e-14)
    assert res.status == "converged" and res.sweeps == 1 and res.k == 1
    assert np.array_equal(x, bi / 4.0)


def test_mixed_breakdown(device):
    """An indefinite matrix: the FP32 inner CG meets <p, Ap> <= 0."""
    A = P.dense_to_csr(np.diag([1.0, -1.0, 2.0, -2.0]))
    b = np.ones(4)
    ref = oracle.solve_mixed(A, b)
    res, x = mixed_solve(A, b)
    assert ref.status == res.status == "breakdown"
    assert_same(res, x, ref, "breakdown")


def test_mixed_api(device):
    """History has one entry per sweep, per-iteration scalars are not kept,
    the profile has the FP64 residual kernel, and the single-workgroup path
    is not used."""
    A, b, _ = P.workload("poisson2d_32")
    M = fk.Matrix(A)
    S = fk.Solver(M, method="cg_mixed", rtol=1e-10, profile=True)
    bd, xd = dev(b), dev(np.zeros(A.n))
    assert S.solve(bd, xd) == fk.OK
    assert not S.uses_small()
    assert len(S.history()) == S.refinements() + 1
    with pytest.raises(fk.FkError) as e:
        S.scalars()
    assert e.value.status == fk.E_STATE
    kt = S.kernel_times()
    assert kt["residual"][1] == S.refinements() + 1
    assert kt["axpy"][1] == S.refinements()
    assert kt["spmv_dot"][1] > 0 and kt["update_dot"][1] > 0
    # A second solve from the result: already converged, no sweep.
    assert S.solve(bd, xd) == fk.OK
    assert S.refinements() == 0 and S.iterations() == 0
    S.close()
    with pytest.raises(fk.FkError):
        fk.Solver(M, method="cg_mixed", inner_rtol=-1.0)
    with pytest.raises(fk.FkError):
        fk.Solver(M, method="cg_mixed", max_outer=-2)


def test_mixed_full_size(device):
    """128^3 Poisson to 1e-10 in the benchmark's launch configuration
    against the stored oracle run (tests/golden/make_golden.py)."""
    g = load("poisson3d_128_cg_mixed")
    A, b, x0 = P.workload(g["workload"])
    print(f"\n[case] {g['case']} n={A.n}", flush=True)
    res, x = mixed_solve(A, b, x0, rtol=g["rtol"], inner_rtol=g["inner_rtol"])
    assert res.status == g["status"] and res.sweeps == g["sweeps"] and res.k == g["k"]
    hist = np.array([float.fromhex(h) for h in g["history_hex"]])
    assert np.array_equal(res.history, hist), (res.history, hist)
    idx = np.array(g["x_index"])
    xs = np.array([float.fromhex(h) for h in g["x_sample_hex"]])
    assert np.array_equal(x[idx], xs)
    assert x_sha256(x) == g["x_sha256"]
    assert oracle.true_residual(A, b, x) <= g["rtol"]
