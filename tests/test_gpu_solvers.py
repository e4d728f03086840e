"""Solver parity through the C ABI: the HIP path against the CPU oracle of
the same algorithm (Algorithms 1-4) on the same seeded inputs.

The HIP kernels round every operation as the oracle does (rows summed in
CSR order, vector updates written the same way, inner products rounded once
from an almost exact sum), so iteration counts and residual histories must
agree exactly and iterates to far below the 1e-10 bar."""
import numpy as np
import pytest

import oracle
from gpu_util import dev, gpu_solve, host, rel, require_layout
from gpu_util import gpu_solve as _gpu_solve
from paper_1410_4054_amd import fk, problems as P

pytestmark = pytest.mark.gpu

CG = ["cg_pipelined", "cg_classical", "cg_pipelined_1k"]
BICG = ["bicgstab_pipelined", "bicgstab_classical", "bicgstab_pipelined_2k"]
ALL = CG + BICG


def oracle_method(method):
    """The oracle's method for a GPU method: the two-kernel schedule of
    Algorithm 4 computes the four-kernel schedule's iterates, the one-kernel
    schedule of Algorithm 2 the two-kernel one's."""
    return {"bicgstab_pipelined_2k": "bicgstab_pipelined", "cg_pipelined_1k": "cg_pipelined"}.get(method, method)


def _random_nonsym(n, seed):
    rng = np.random.default_rng(seed)
    return P.dense_to_csr(np.eye(n) * 4 + rng.uniform(-0.5, 0.5, (n, n)))


WORKLOADS = {
    "poisson2d_32": lambda: P.workload("poisson2d_32"),
    "poisson3d_24": lambda: P.workload("poisson3d_24"),
    "heat2d_48": lambda: P.workload("heat2d_48"),
    "convdiff2d_64": lambda: P.workload("convdiff2d_64"),
    "spd_dense_60": lambda: (P.dense_to_csr(P.random_spd_dense(60, 300.0, seed=2)),
                             P.rhs_uniform(60, 3), np.zeros(60)),
    "nonsym_dense_70": lambda: (_random_nonsym(70, 4), P.rhs_uniform(70, 5), np.zeros(70)),
}
CASES = [(w, m) for w in ("poisson2d_32", "poisson3d_24", "heat2d_48", "spd_dense_60") for m in ALL] + \
        [(w, m) for w in ("convdiff2d_64", "nonsym_dense_70") for m in BICG]


def assert_same_run(res, x, ref, label=""):
    assert res.status == ref.status, (label, res.status, ref.status)
    assert res.k == ref.k, (label, res.k, ref.k)
    np.testing.assert_allclose(res.history, ref.hist, rtol=1e-14, atol=0, err_msg=label)
    assert rel(x, ref.x) <= 1e-10, (label, rel(x, ref.x))


@pytest.mark.parametrize("small,layout", [(True, None), (False, "row_blocks"), (False, "sliced"),
                                         (False, "sliced16"), (False, "slots")],
                         ids=["auto", "grid-row_blocks", "grid-sliced", "grid-sliced16", "grid-slots"])
@pytest.mark.parametrize("wl,method", CASES, ids=[f"{w}-{m}" for w, m in CASES])
def test_matches_oracle(wl, method, small, layout, device):
    """small=True lets the library take its single-workgroup solver where it
    applies (the small pipelined cases); small=False forces the grid kernels,
    on either layout of the products."""
    A, b, x0 = WORKLOADS[wl]()
    require_layout(A, layout)
    print(f"\n[case] {wl} {method} n={A.n} small={small} layout={layout}", flush=True)
    ref = oracle.solve(A, b, x0=x0, method=oracle_method(method), rtol=1e-8, trace=True)
    res, x = gpu_solve(A, b, x0, method=method, rtol=1e-8, small=small, layout=layout)
    assert_same_run(res, x, ref, f"{wl}/{method}")
    assert ref.status == "converged"
    assert oracle.true_residual(A, b, x) <= 1.5e-8
    # per-iteration scalars follow the oracle's trace
    np.testing.assert_allclose(res.scalars[:, 0], ref.t("alpha"), rtol=1e-13)
    if method.startswith("bicgstab"):
        om = ref.t("omega")
        ok = np.isfinite(om)
        np.testing.assert_allclose(res.scalars[ok, 2], om[ok], rtol=1e-13)


@pytest.mark.parametrize("wl", ["poisson2d_32", "poisson3d_24", "heat2d_48"])
def test_pipelined_cg_vs_classical_oracle(wl, device):
    """The literal bar on the stencil workloads: pipelined CG on the GPU
    against the oracle of classical CG (Algorithm 1): solutions within
    1e-10, iteration counts within 2."""
    A, b, x0 = WORKLOADS[wl]()
    ref = oracle.solve(A, b, method="cg_classical", rtol=1e-8)
    res, x = gpu_solve(A, b, method="cg_pipelined", rtol=1e-8)
    assert abs(res.k - ref.k) <= 2
    cl_k = oracle.solve(A, b, method="cg_classical", rtol=0.0, max_iter=res.k)
    assert rel(x, cl_k.x) <= 1e-10
    assert rel(x, ref.x) <= 1e-10


@pytest.mark.parametrize("wl,method", [("spd_dense_60", "cg"), ("convdiff2d_64", "bicgstab"),
                                       ("nonsym_dense_70", "bicgstab")])
def test_classical_gap_is_the_algorithms_own(wl, method, device):
    """Where classical and pipelined recurrences drift apart in FP64 (dense
    random SPD, BiCGStab; cf. Table 2), the GPU's distance from the classical
    oracle is exactly the pipelined oracle's distance from it."""
    A, b, x0 = WORKLOADS[wl]()
    conv, xc = gpu_solve(A, b, method=f"{method}_pipelined", rtol=1e-8)
    assert oracle.true_residual(A, b, xc) <= 1.5e-8
    # equal k on every side (rtol = 0: no early or half-step exit)
    k = conv.k
    res, x = gpu_solve(A, b, method=f"{method}_pipelined", rtol=0.0, max_iter=k)
    cl = oracle.solve(A, b, method=f"{method}_classical", rtol=0.0, max_iter=k)
    pi = oracle.solve(A, b, method=f"{method}_pipelined", rtol=0.0, max_iter=k)
    floor = rel(pi.x, cl.x)
    print(f"\n[floor] {wl} {method} k={k}: classical vs pipelined {floor:.2e}", flush=True)
    assert abs(rel(x, cl.x) - floor) <= 1e-3 * floor + 1e-15


@pytest.mark.parametrize("method", ALL)
def test_fixed_30_iterations(method, device):
    """The paper's timing protocol runs exactly 30 iterations."""
    wl = "convdiff2d_64" if method.startswith("bicg") else "poisson3d_24"
    A, b, x0 = WORKLOADS[wl]()
    ref = oracle.solve(A, b, method=oracle_method(method), rtol=0.0, max_iter=30)
    res, x = gpu_solve(A, b, method=method, rtol=0.0, max_iter=30)
    assert res.status == "not_converged" and res.k == 30
    assert_same_run(res, x, ref, method)


@pytest.mark.parametrize("small", [True, False], ids=["auto", "grid"])
@pytest.mark.parametrize("method", ALL)
def test_edge_cases(method, small, device):
    A, b, _ = P.workload("poisson2d_16")
    gpu_solve = lambda *a, **k: _gpu_solve(*a, small=small, **k)  # noqa: E731
    n = A.n
    # b = 0: x = 0, k = 0
    res, x = gpu_solve(A, np.zeros(n), np.ones(n), method=method)
    assert res.status == "converged" and res.k == 0 and not x.any()
    # warm start
    x0 = np.random.default_rng(1).standard_normal(n)
    ref = oracle.solve(A, b, x0=x0, method=oracle_method(method), rtol=1e-10)
    res, x = gpu_solve(A, b, x0, method=method, rtol=1e-10)
    assert_same_run(res, x, ref, "warm start")
    # starting guess already a solution: k = 0
    exact = np.linalg.solve(A.to_dense(), b)
    res, x = gpu_solve(A, b, exact, method=method, rtol=1e-8)
    assert res.k == 0 and res.status == "converged" and np.array_equal(x, exact)
    # max_iter = 0 and 1
    for mi in (0, 1):
        ref = oracle.solve(A, b, method=oracle_method(method), rtol=0.0, max_iter=mi)
        res, x = gpu_solve(A, b, method=method, rtol=0.0, max_iter=mi)
        assert_same_run(res, x, ref, f"max_iter={mi}")
    # eigenvector right-hand side: one iteration (BiCGStab leaves after the half step)
    v = P.laplacian_eigvec_2d(16, 2, 7)
    ref = oracle.solve(A, v, method=oracle_method(method), rtol=1e-10)
    res, x = gpu_solve(A, v, method=method, rtol=1e-10)
    assert res.k == ref.k == 1
    assert_same_run(res, x, ref, "eigenvector")
    # 1 x 1 system and A = lambda I
    for A1, b1 in ((P.scaled_identity(1, 4.0), np.array([2.0])), (P.scaled_identity(300, 2.5), P.rhs_uniform(300))):
        ref = oracle.solve(A1, b1, method=oracle_method(method), rtol=1e-12)
        res, x = gpu_solve(A1, b1, method=method, rtol=1e-12)
        assert_same_run(res, x, ref, "scaled identity")


def _half_step_exits():
    """convdiff2d_20 with tolerances at which the oracle's pipelined BiCGStab
    leaves after the half step of iteration k >= 2 (no omega in its last
    trace row), one for each parity of k - 1: the buffers the two-kernel
    schedule holds r_i, p_i and A p_i in.  Found on the CPU, by the oracle
    alone."""
    A, b, _ = P.workload("convdiff2d_20")
    found = {}
    for e in np.linspace(2.0, 12.0, 81):
        rtol = 10.0 ** -e
        ref = oracle.solve(A, b, method="bicgstab_pipelined", rtol=rtol, trace=True)
        if ref.status == "converged" and ref.k >= 2 and np.isnan(ref.t("omega")[-1]):
            found.setdefault((ref.k - 1) & 1, rtol)
        if len(found) == 2:
            break
    return A, b, found


@pytest.mark.parametrize("small", [True, False], ids=["auto", "grid"])
@pytest.mark.parametrize("method", BICG)
def test_half_step_exit_later(method, small, device):
    """A half-step exit after several iterations, with the iteration count
    of either parity: x_{i+1} = x_i + alpha_i p_i from the right buffers."""
    A, b, found = _half_step_exits()
    assert set(found) == {0, 1}
    for parity, rtol in sorted(found.items()):
        ref = oracle.solve(A, b, method=oracle_method(method), rtol=rtol, trace=True)
        print(f"\n[case] half step {method} parity {parity} rtol={rtol:.3e} k={ref.k} small={small}", flush=True)
        res, x = gpu_solve(A, b, method=method, rtol=rtol, small=small)
        assert_same_run(res, x, ref, f"half step, parity {parity}")


@pytest.mark.parametrize("small", [True, False], ids=["auto", "grid"])
@pytest.mark.parametrize("method", ALL)
def test_breakdown(method, small, device):
    gpu_solve = lambda *a, **k: _gpu_solve(*a, small=small, **k)  # noqa: E731
    if method.startswith("cg"):
        A = P.dense_to_csr(np.diag([1.0, -1.0, 2.0, -2.0]))
    else:
        S = np.zeros((4, 4))
        S[0, 1], S[1, 0], S[2, 3], S[3, 2] = 1.0, -1.0, 2.0, -2.0
        A = P.dense_to_csr(S)
    b = np.ones(4)
    ref = oracle.solve(A, b, method=oracle_method(method))
    res, x = gpu_solve(A, b, method=method)
    assert ref.status == res.status == "breakdown"
    assert res.k == ref.k
    # non-finite right-hand side
    A, b, _ = P.workload("poisson2d_16")
    b = b.copy()
    b[7] = np.nan
    ref = oracle.solve(A, b, method=oracle_method(method))
    res, x = gpu_solve(A, b, method=method)
    assert ref.status == res.status == "breakdown" and res.k == ref.k


@pytest.mark.parametrize("method", ALL)
def test_driver_modes_identical(method, device):
    """hipGraph replay, per-kernel event timing and any polling interval
    enqueue the same kernels: results are bit-identical."""
    wl = "convdiff2d_64" if method.startswith("bicg") else "poisson3d_24"
    A, b, _ = WORKLOADS[wl]()
    M = fk.Matrix(A)
    base, xb = gpu_solve(A, b, method=method, matrix=M)
    for kw in ({"graph": True}, {"graph": True, "unroll": 5}, {"profile": True},
               {"unroll": 1}, {"unroll": 3}, {"unroll": 64}):
        res, x = gpu_solve(A, b, method=method, matrix=M, **kw)
        assert res.k == base.k and np.array_equal(x, xb), kw
        assert np.array_equal(res.history, base.history), kw


def test_solver_reuse_and_api(device):
    import torch

    A, b, _ = P.workload("poisson3d_24")
    M = fk.Matrix(A)
    S = fk.Solver(M, method="cg_pipelined", rtol=1e-9)
    for seed in (0, 1, 2):
        bb = P.rhs_uniform(A.n, seed)
        ref = oracle.solve(A, bb, method="cg_pipelined", rtol=1e-9)
        xd = dev(np.zeros(A.n))
        assert S.solve(dev(bb), xd) == fk.OK
        assert S.iterations() == ref.k
        assert np.array_equal(S.history(), ref.hist)
        assert rel(host(xd), ref.x) <= 1e-10
    S.close()
    S = fk.Solver(M, method="cg_pipelined", record_history=False)
    with pytest.raises(fk.FkError):
        S.iterations()  # no solve yet
    S.solve(dev(b), dev(np.zeros(A.n)))
    with pytest.raises(fk.FkError):
        S.history()
    S.close()
    with pytest.raises(TypeError):
        fk.solve(M, torch.zeros(A.n, dtype=torch.float32, device=device), dev(np.zeros(A.n)))
    with pytest.raises(ValueError):
        fk.solve(M, dev(np.zeros(A.n + 1)), dev(np.zeros(A.n)))


def test_small_path_selection(device):
    """Which solves take the single-workgroup solver, and that it agrees
    with the grid kernels bit for bit on the latency-bound workload."""
    A, b, _ = P.workload("poisson2d_32")
    M = fk.Matrix(A)
    for method, expect in (("cg_pipelined", True), ("bicgstab_pipelined", True),
                           ("cg_classical", False), ("bicgstab_classical", False)):
        S = fk.Solver(M, method=method)
        assert S.uses_small() is expect, method
        S.close()
    S = fk.Solver(M, method="cg_pipelined", small=False)
    assert not S.uses_small()
    S.close()
    big = fk.Matrix(P.workload("poisson3d_24")[0])  # n = 13824 > 4096
    S = fk.Solver(big, method="cg_pipelined")
    assert not S.uses_small()
    S.close()
    for method in ("cg_pipelined", "bicgstab_pipelined"):
        r1, x1 = gpu_solve(A, b, method=method, matrix=M, small=True)
        r2, x2 = gpu_solve(A, b, method=method, matrix=M, small=False)
        assert r1.k == r2.k and np.array_equal(x1, x2), method
        assert np.array_equal(r1.history, r2.history), method
        S = fk.Solver(M, method=method, profile=True)
        xd = dev(np.zeros(A.n))
        S.solve(dev(b), xd)
        t = S.kernel_times()
        assert t["small"][1] == 1 and t["small"][0] > 0
        S.close()


@pytest.mark.parametrize("n,method,small", [(90, "cg_pipelined", False), (64, "cg_pipelined", True),
                                            (60, "cg_pipelined", True), (45, "cg_pipelined", True),
                                            (2, "cg_pipelined", True), (55, "cg_pipelined_1k", True),
                                            (56, "cg_pipelined_1k", False), (40, "bicgstab_pipelined", True),
                                            (31, "bicgstab_pipelined", True)])
def test_small_path_rows_per_thread(n, method, small, device):
    """1, 2 and 4 rows per thread of the single-workgroup solver, and the
    sizes where the grid kernels take over (n > 4096 for the two-kernel
    CG, n > 3072 for the one-kernel CG)."""
    A = P.poisson2d(n) if method.startswith("cg") else P.convdiff2d(n)
    b = P.rhs_uniform(A.n, 7)
    ref = oracle.solve(A, b, method=oracle_method(method), rtol=1e-9)
    res, x = gpu_solve(A, b, method=method, rtol=1e-9)
    assert fk.Solver(fk.Matrix(A), method=method).uses_small() is small
    assert_same_run(res, x, ref, f"n={n}")


@pytest.mark.parametrize("side,method", [(14, "cg_pipelined"), (20, "cg_pipelined"), (31, "cg_pipelined"),
                                         (38, "cg_pipelined"), (14, "bicgstab_pipelined"),
                                         (20, "bicgstab_pipelined"), (31, "bicgstab_pipelined"),
                                         (38, "bicgstab_pipelined")])
def test_small_workgroup_sizes(side, method, device):
    """The single-workgroup solver takes 256, 512 or 1024 threads by size
    (196 and 400 rows: 256 threads; 961: 512; 1444: 1024 with two rows per
    thread); every combination follows the oracle's trajectory."""
    A = P.poisson2d(side) if method == "cg_pipelined" else P.convdiff2d(side)
    b = P.rhs_uniform(A.n, side)
    print(f"\n[case] small {method} n={A.n}", flush=True)
    M = fk.Matrix(A)
    S = fk.Solver(M, method=method, rtol=1e-8)
    assert S.uses_small(), A.n
    S.close()
    ref = oracle.solve(A, b, method=oracle_method(method), rtol=1e-8)
    res, x = gpu_solve(A, b, method=method, rtol=1e-8, matrix=M)
    assert_same_run(res, x, ref, f"small {method} n={A.n}")
