"""The streaming mode of the sliced products (non-temporal matrix loads and
the per-XCD sweep order) changes only how the matrix is read: row sums,
inner products and whole solves must stay bit for bit those of the oracle,
in every sliced layout, on matrices whose slices do not divide evenly among
the eight XCDs."""
import numpy as np
import pytest

import oracle
from gpu_util import dev, gpu_solve, host, rel
from paper_1410_4054_amd import fk, problems as P

pytestmark = pytest.mark.gpu

SLICED = ["sliced", "sliced16", "slots"]


def _matrix(A, layout, mode):
    M = fk.Matrix(A)
    try:
        M.set_layout(layout)
    except fk.FkError as e:
        M.close()
        if e.status == fk.E_ARG:
            pytest.skip(f"layout {layout} does not apply to this matrix")
        raise
    M.set_stream(mode)
    return M


@pytest.mark.parametrize("layout", SLICED)
@pytest.mark.parametrize("name", ["poisson3d_17", "poisson3d_40", "convdiff2d_50", "poisson2d_33"])
def test_stream_products_match_oracle(name, layout, device):
    A, _, _ = P.workload(name)
    p = np.random.default_rng(3).uniform(-1, 1, A.n)
    ref = oracle.spmv(A, p)
    M = _matrix(A, layout, 1)
    on, sweep = M.stream()
    # sweep order needs at least 8 workgroups of 4 waves with a slice each
    slices = -(-A.n // 64)
    assert on and sweep == ((slices + 3) // 4 >= 8)
    pd, qd = dev(p), dev(np.zeros(A.n))
    dots = fk.spmv(M, pd, qd, dots=True)
    q = host(qd)
    assert np.array_equal(q, ref)
    assert dots[0] == oracle.dot(p, q)
    assert dots[1] == oracle.dot(q, q)
    M.set_stream(0)
    assert M.stream() == (False, False)
    q2 = dev(np.full(A.n, np.nan))
    dots2 = fk.spmv(M, pd, q2, dots=True)
    assert np.array_equal(host(q2), q) and tuple(dots2) == tuple(dots)
    M.close()


@pytest.mark.parametrize("n", [63, 65, 4097, 70001])
def test_stream_products_ragged(n, device):
    """Slice counts that are not a multiple of 8 (the XCD eighths)."""
    A = P.random_csr(n, 6, seed=n)
    p = np.random.default_rng(n).uniform(-1, 1, n)
    M = _matrix(A, "sliced", 1)
    pd, qd = dev(p), dev(np.zeros(n))
    dots = fk.spmv(M, pd, qd, dots=True)
    q = host(qd)
    assert np.array_equal(q, oracle.spmv(A, p))
    assert dots[0] == oracle.dot(p, q) and dots[1] == oracle.dot(q, q)
    M.close()


@pytest.mark.parametrize("wl,method", [("poisson3d_24", "cg_pipelined"), ("poisson3d_24", "cg_classical"),
                                       ("poisson3d_24", "cg_pipelined_1k"),
                                       ("convdiff2d_64", "bicgstab_pipelined_2k"),
                                       ("convdiff2d_64", "bicgstab_pipelined"),
                                       ("convdiff2d_64", "bicgstab_pipelined_split"),
                                       ("poisson3d_24", "cg_mixed"), ("poisson3d_24", "cg_mixed_f32")])
def test_stream_solves_match_normal(wl, method, device):
    """A solve in streaming mode equals the same solve without it, and (for
    the FP64 methods) the oracle's."""
    A, b, _ = P.workload(wl)
    rtol = 1e-10 if "mixed" in method else 1e-8
    runs = []
    for mode in (0, 1):
        M = _matrix(A, "slots", mode)
        res, x = gpu_solve(A, b, method=method, rtol=rtol, matrix=M, small=False)
        runs.append((res, x))
        M.close()
    (r0, x0), (r1, x1) = runs
    assert r0.status == r1.status == "converged"
    if method == "cg_mixed_f32":
        # FP32-accumulated sums follow the launch shape, and the sweep order
        # has its own grid: equal only up to the FP32 summation bound
        assert abs(r0.k - r1.k) <= 0.1 * r0.k + 2
        assert oracle.true_residual(A, b, x0) <= 1.5 * rtol
        assert oracle.true_residual(A, b, x1) <= 1.5 * rtol
        return
    assert r0.k == r1.k
    assert np.array_equal(x0, x1)
    assert np.array_equal(r0.history, r1.history)
    if "mixed" not in method:
        base = method.replace("_split", "").replace("_2k", "").replace("_1k", "")
        ref = oracle.solve(A, b, method=base, rtol=rtol, trace=True)
        assert r1.k == ref.k
        assert rel(x1, ref.x) <= 1e-10


def test_stream_by_size(device):
    """By size: off for the 128^3 Poisson matrix (126 MB of slots + four
    vectors fit the 256 MiB cache), on for 160^3 (247 MB + 131 MB)."""
    small, _, _ = P.workload("poisson3d_64")
    M = fk.Matrix(small)
    assert M.stream() == (False, False)
    M.close()
    big, _, _ = P.workload("poisson3d_160")
    M = fk.Matrix(big)
    assert M.layout()[0] == "slots"
    assert M.matrix_bytes() + 32 * big.n > 256 << 20
    assert M.stream() == (True, True)
    M.set_stream(0)
    assert M.stream() == (False, False)
    M.set_stream(-1)
    assert M.stream() == (True, True)
    M.close()


def test_stream_refused_while_solver_exists(device):
    A, _, _ = P.workload("poisson2d_33")
    M = fk.Matrix(A)
    S = fk.Solver(M, method="cg_pipelined")
    with pytest.raises(fk.FkError) as e:
        M.set_stream(1)
    assert e.value.status == fk.E_STATE
    S.close()
    with pytest.raises(fk.FkError) as e:
        M.set_stream(2)
    assert e.value.status == fk.E_ARG
    M.close()
