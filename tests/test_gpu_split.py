"""The split variants of Sections 3.1 and 3.2 (the products' inner products
computed in kernels of their own: 3 launches per CG iteration, 6 per
BiCGStab iteration) against the oracle of the same pipelined recurrences.
The dots are the same exact sums rounded once, only computed in another
kernel, so iteration counts, histories, per-iteration scalars and iterates
agree with the oracle as the fused kernels' do, and with the fused kernels
bit for bit."""
import numpy as np
import pytest

import oracle
from gpu_util import gpu_solve, require_layout
from paper_1410_4054_amd import fk, problems as P

pytestmark = pytest.mark.gpu

CASES = [("poisson2d_32", "cg"), ("poisson3d_24", "cg"), ("heat2d_48", "cg"),
         ("convdiff2d_64", "bicgstab"), ("poisson3d_24", "bicgstab"), ("convdiff2d_5", "bicgstab")]


@pytest.mark.parametrize("layout", ["row_blocks", "slots"])
@pytest.mark.parametrize("wl,kind", CASES, ids=[f"{w}-{k}" for w, k in CASES])
def test_split_matches_oracle(wl, kind, layout, device):
    A, b, x0 = P.workload(wl)
    require_layout(A, layout)
    print(f"\n[case] split {wl} {kind} n={A.n} layout={layout}", flush=True)
    ref = oracle.solve(A, b, x0=x0, method=f"{kind}_pipelined", rtol=1e-8, trace=True)
    res, x = gpu_solve(A, b, x0, method=f"{kind}_pipelined_split", rtol=1e-8, layout=layout)
    assert res.status == ref.status == "converged"
    assert res.k == ref.k
    np.testing.assert_allclose(res.history, ref.hist, rtol=1e-14, atol=0)
    assert np.abs(x - ref.x).max() <= 1e-10 * np.abs(ref.x).max()
    np.testing.assert_allclose(res.scalars[:, 0], ref.t("alpha"), rtol=1e-13)


@pytest.mark.parametrize("kind", ["cg", "bicgstab"])
def test_split_equals_fused(kind, device):
    """Fixed 30 iterations: the split and fused kernels give the same bits,
    and the split variant runs one product and one dot kernel per product."""
    wl = "convdiff2d_64" if kind == "bicgstab" else "poisson3d_24"
    A, b, _ = P.workload(wl)
    fused, xf = gpu_solve(A, b, method=f"{kind}_pipelined", rtol=0.0, max_iter=30, small=False)
    split, xs = gpu_solve(A, b, method=f"{kind}_pipelined_split", rtol=0.0, max_iter=30)
    assert fused.status == split.status == "not_converged" and split.k == 30
    assert np.array_equal(fused.history, split.history)
    assert np.array_equal(xf, xs)
    M = fk.Matrix(A)
    S = fk.Solver(M, method=f"{kind}_pipelined_split", rtol=0.0, max_iter=30, profile=True)
    from gpu_util import dev
    bd, xd = dev(b), dev(np.zeros(A.n))
    S.solve(bd, xd)
    kt = S.kernel_times()
    per = 1 if kind == "cg" else 2
    assert kt["spmv"][1] >= 30 * per and kt["dot"][1] == kt["spmv"][1]
    assert kt["spmv_dot"][1] == 0
    S.close()
    M.close()


def test_split_breakdown_and_edge_cases(device):
    """b = 0, an iteration budget, and CG's breakdown on an indefinite matrix
    behave as in the fused form."""
    A, b, _ = P.workload("poisson2d_16")
    for kind in ("cg", "bicgstab"):
        z, zx = gpu_solve(A, np.zeros(A.n), np.ones(A.n), method=f"{kind}_pipelined_split")
        assert z.status == "converged" and z.k == 0 and not zx.any()
        r, x = gpu_solve(A, b, method=f"{kind}_pipelined_split", rtol=0.0, max_iter=5)
        ref = oracle.solve(A, b, method=f"{kind}_pipelined", rtol=0.0, max_iter=5)
        assert r.status == ref.status == "not_converged" and r.k == 5 and np.array_equal(x, ref.x)
    Ai = P.dense_to_csr(np.diag([1.0, -1.0, 2.0, -2.0]))
    res, _ = gpu_solve(Ai, np.ones(4), method="cg_pipelined_split")
    assert res.status == oracle.solve(Ai, np.ones(4), method="cg_pipelined").status == "breakdown"
