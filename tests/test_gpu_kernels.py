"""Kernel-level parity through the C ABI: the fused CSR product and its
first-stage reductions, the device dot, the copy kernel.  The oracle sums
each row left to right, as the HIP kernels do for rows of at most
FK_LONG_ROW nonzeros, so those rows must agree bit for bit; inner products
are rounded once from an (almost) exact sum on both sides."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import dev, host
from paper_1410_4054_amd import fk, problems as P

pytestmark = pytest.mark.gpu


LAYOUTS = ["row_blocks", "sliced", "sliced16", "slots"]


def check_spmv(A, seed=0, layout=None):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-1, 1, A.n)
    if layout == "slots" and _slot_plan(A) is None:
        # not applicable: refused, and the matrix keeps a working layout
        M = fk.Matrix(A)
        with pytest.raises(fk.FkError) as e:
            M.set_layout("slots")
        assert e.value.status == fk.E_ARG
        M.close()
        return None
    M = fk.Matrix(A, layout=layout)
    if layout is not None:
        assert M.layout()[0] == layout
    pd, qd = dev(p), dev(np.zeros(A.n))
    dots = fk.spmv(M, pd, qd, dots=True)
    q = host(qd)
    ref = oracle.spmv(A, p)
    # The sliced layout sums every row left to right; row blocks use a
    # fixed tree for rows longer than FK_LONG_ROW.
    short = np.diff(A.row_ptr) <= (fk.LONG_ROW if M.layout()[0] == "row_blocks" else np.inf)
    assert np.array_equal(q[short], ref[short]), "row sums differ from CSR-order sums"
    if (~short).any():
        np.testing.assert_allclose(q[~short], ref[~short], rtol=1e-12, atol=1e-12)
    assert dots[0] == oracle.dot(p, q)
    assert dots[1] == oracle.dot(q, q)
    # plain product (no reductions) gives the same vector
    q2 = dev(np.full(A.n, np.nan))
    fk.spmv(M, pd, q2)
    assert np.array_equal(host(q2), q)
    M.close()
    return M


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("nnz_row", [4, 28])
def test_spmv_random_columns(nnz_row, layout, device):
    """The fused SpMV+dot benchmark matrices: 4 and 28 uniformly random
    nonzeros per row, with empty rows and rows longer than FK_LONG_ROW."""
    A = P.random_csr(20000, nnz_row, seed=nnz_row, empty_rows=31,
                     long_rows={3: 3000, 9000: 20000, 19999: 2049})
    check_spmv(A, seed=nnz_row, layout=layout)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("name", ["poisson2d_33", "poisson3d_17", "convdiff2d_50", "heat2d_40",
                                  "poisson2d_32", "poisson3d_64"])
def test_spmv_stencils(name, layout, device):
    A, _, _ = P.workload(name)
    check_spmv(A, seed=1, layout=layout)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 255, 256, 257, 511, 513, 4097])
def test_spmv_ragged_sizes(n, layout, device):
    """Sizes around the 64-row slice, the 256-row block and the
    8-workgroup XCD split."""
    check_spmv(P.random_csr(n, 5, seed=n), seed=n, layout=layout)


def _slice_entries(A):
    """Entries of the sliced layout, padding included: 64 times the longest
    row of each run of 64 rows; the longest row; whether every column lies
    within 32767 of its row."""
    lens = np.diff(A.row_ptr)
    pad = np.zeros(-(-A.n // 64) * 64, dtype=np.int64)
    pad[:A.n] = lens
    rows = np.repeat(np.arange(A.n), lens)
    narrow = bool(np.all(np.abs(A.col_idx.astype(np.int64) - rows) <= 32767))
    return int(pad.reshape(-1, 64).max(axis=1).sum() * 64), int(lens.max(initial=0)), narrow


def _slot_plan(A):
    """The slot layout counted from the CSR: None when a row's columns do
    not strictly ascend, a 64-row slice has more than 32 distinct column
    offsets or the slots pad the entries by more than a quarter; else
    (entries, bytes of matrix data one FP64 product reads)."""
    if A.nnz == 0:
        return None
    lens = np.diff(A.row_ptr)
    rows = np.repeat(np.arange(A.n, dtype=np.int64), lens)
    cols = A.col_idx.astype(np.int64)
    same = rows[1:] == rows[:-1]
    if np.any(cols[1:][same] <= cols[:-1][same]):
        return None
    pairs = np.unique(np.stack([rows // 64, cols - rows]), axis=1)
    nsl = -(-A.n // 64)
    per_slice = np.bincount(pairs[0], minlength=nsl)
    if per_slice.max() > 32:
        return None
    slots = int(per_slice.sum())
    entries = 64 * slots
    if 4 * entries > 5 * A.nnz:
        return None
    return entries, 8 * entries + 4 * slots + 4 * 64 * nsl + 4 * (nsl + 1)


def _far_stencil(n=200000, d=40000, seed=5):
    """Three diagonals at offsets -d, 0, +d (d beyond 16 bits): no 16-bit
    offsets, but three slots per slice and no padding."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for off in (-d, 0, d):
        r = np.arange(max(0, -off), min(n, n - off))
        rows.append(r)
        cols.append(r + off)
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, rows + 1, 1)
    return P.Csr(n, np.cumsum(rp).astype(np.int32), cols.astype(np.int32), rng.uniform(-1, 1, rows.size))


def test_spmv_slots_far_offsets(device):
    """Column offsets of +-40000: SLICED16 refused, SLOTS bit-exact."""
    A = _far_stencil()
    assert _slot_plan(A) == (A.nnz, 8 * A.nnz + 4 * (A.nnz // 64) + 4 * 64 * 3125 + 4 * 3126)
    M = fk.Matrix(A)
    assert M.layout() == ("slots", A.nnz)
    assert fk.lib().fk_csr_set_layout(M.handle, fk.LAYOUTS["sliced16"], None) == fk.E_ARG
    M.close()
    check_spmv(A, seed=3, layout="slots")
    check_spmv(A, seed=3, layout="sliced")


def _banded(n, half, seed=7, descending_row=None):
    """Rows i with columns i-half .. i+half inside [0, n): 2*half + 1
    distinct column offsets per slice away from the ends.  descending_row:
    that row's columns stored in descending order (still valid CSR)."""
    rng = np.random.default_rng(seed)
    rp, ci = [0], []
    for i in range(n):
        cols = list(range(max(0, i - half), min(n, i + half + 1)))
        if i == descending_row:
            cols = cols[::-1]
        ci.extend(cols)
        rp.append(len(ci))
    return P.Csr(n, np.array(rp, np.int32), np.array(ci, np.int32), rng.uniform(-1, 1, len(ci)))


@pytest.mark.parametrize("half,slots", [(15, True), (16, False)], ids=["31-offsets", "33-offsets"])
def test_slots_offset_limit(half, slots, device):
    """At most 32 distinct column offsets per slice (one mask bit each): a
    31-diagonal band takes the slot layout, a 33-diagonal band is refused
    and the creation rule falls back to 16-bit offsets; both products equal
    the CSR-order sums."""
    A = _banded(3000, half)
    assert (_slot_plan(A) is not None) == slots
    M = fk.Matrix(A)
    assert M.layout()[0] == ("slots" if slots else "sliced16")
    M.close()
    check_spmv(A, seed=half, layout="slots")
    check_spmv(A, seed=half, layout=None)


def test_slots_full_mask(device):
    """Exactly 32 distinct offsets in a slice: the 32nd slot uses the
    mask's top bit."""
    n = 640
    rng = np.random.default_rng(11)
    offs = np.array(list(range(-16, 0)) + list(range(1, 17)), dtype=np.int64)
    rp, ci = [0], []
    for i in range(n):
        cols = sorted(int(i + o) for o in offs if 0 <= i + o < n)
        ci.extend(cols)
        rp.append(len(ci))
    A = P.Csr(n, np.array(rp, np.int32), np.array(ci, np.int32), rng.uniform(-1, 1, len(ci)))
    assert _slot_plan(A) is not None
    check_spmv(A, seed=2, layout="slots")


def test_slots_need_ascending_columns(device):
    """A row stored with descending columns: slot order would not be CSR
    order, so the slot layout is refused and the products keep summing
    that row in its stored order."""
    A = _banded(1000, 2, descending_row=500)
    assert _slot_plan(A) is None
    M = fk.Matrix(A)
    assert M.layout()[0] == "sliced16"
    M.close()
    check_spmv(A, seed=4, layout="slots")  # refused with FK_E_ARG
    check_spmv(A, seed=4, layout=None)


def _matrix_bytes(A, layout):
    """Bytes of matrix data one FP64 product reads, counted from the CSR."""
    lens = np.diff(A.row_ptr)
    pad = np.zeros(-(-A.n // 64) * 64, dtype=np.int64)
    pad[:A.n] = lens
    widths = pad.reshape(-1, 64).max(axis=1)
    slices = widths.size
    if layout == "row_blocks":
        return 12 * A.nnz + 4 * (A.n + 1)
    if layout == "sliced":
        return 12 * int(widths.sum()) * 64 + 4 * (slices + 1)
    return 8 * int(widths.sum()) * 64 + 8 * int(((widths + 3) // 4).sum()) * 64 + 8 * (slices + 1)


@pytest.mark.parametrize("case", ["poisson3d_17", "convdiff2d_50", "random5", "long_row", "padding",
                                  "empty"])
def test_layout_rule(case, device):
    """fk_csr_create takes the slot layout when it applies, else the sliced
    layout when no row exceeds 64 nonzeros and padding adds at most a
    quarter; the entries and bytes it reports are counted here
    independently."""
    if case in ("poisson3d_17", "convdiff2d_50"):
        A = P.workload(case)[0]
    elif case == "random5":
        A = P.random_csr(1000, 5, seed=1)
    elif case == "long_row":
        A = P.random_csr(1000, 5, seed=1, long_rows={7: 65})
    elif case == "padding":
        A = P.random_csr(6400, 1, seed=2, long_rows={64 * k: 3 for k in range(100)})
    else:
        A = P.Csr(5, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0))
    entries, longest, narrow = _slice_entries(A)
    sliced = A.nnz > 0 and longest <= 64 and 4 * entries <= 5 * A.nnz
    assert sliced == (case in ("poisson3d_17", "convdiff2d_50", "random5"))
    plan = _slot_plan(A)
    assert (plan is not None) == (case in ("poisson3d_17", "convdiff2d_50"))
    auto = "slots" if plan else ("sliced16" if narrow else "sliced") if sliced else "row_blocks"
    M = fk.Matrix(A)
    if plan:
        assert M.layout() == ("slots", plan[0]) and M.matrix_bytes() == plan[1]
    else:
        assert M.layout() == ((auto, entries) if sliced else ("row_blocks", A.nnz))
    M.set_layout("sliced")
    assert M.layout() == ("sliced", entries)
    M.set_layout("row_blocks")
    assert M.layout() == ("row_blocks", A.nnz)
    assert M.matrix_bytes() == _matrix_bytes(A, "row_blocks")
    M.set_layout("sliced16")
    assert M.layout() == ("sliced16", entries)
    assert M.matrix_bytes() == _matrix_bytes(A, "sliced16")
    M.set_layout("sliced")
    assert M.matrix_bytes() == _matrix_bytes(A, "sliced")
    if plan:
        M.set_layout("slots")
        assert M.layout() == ("slots", plan[0]) and M.matrix_bytes() == plan[1]
    else:
        with pytest.raises(fk.FkError) as e:
            M.set_layout("slots")
        assert e.value.status == fk.E_ARG
    M.set_layout("auto")
    assert M.layout()[0] == auto


def test_layout_errors(device):
    A = P.workload("poisson2d_33")[0]
    M = fk.Matrix(A)
    assert fk.lib().fk_csr_set_layout(M.handle, 5, None) == fk.E_ARG
    assert fk.lib().fk_csr_set_layout(None, 1, None) == fk.E_ARG
    # a column 40000 away from its row: no 16-bit offsets, 32-bit ones work
    far = P.Csr(40001, np.array([0, 1] + [2] * 40000, np.int32), np.array([40000, 0], np.int32),
                np.array([1.0, 2.0]))
    F = fk.Matrix(far, layout="sliced")
    assert fk.lib().fk_csr_set_layout(F.handle, fk.LAYOUTS["sliced16"], None) == fk.E_ARG
    assert F.layout()[0] == "sliced"
    check_spmv(far, layout="sliced")
    S = fk.Solver(M)
    with pytest.raises(fk.FkError) as e:
        M.set_layout("row_blocks")
    assert e.value.status == fk.E_STATE
    S.close()
    M.set_layout("row_blocks")
    assert M.layout()[0] == "row_blocks"


def test_spmv_degenerate(device):
    # all rows empty
    A = P.Csr(5, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0))
    M = fk.Matrix(A)
    qd = dev(np.full(5, 7.0))
    d = fk.spmv(M, dev(np.ones(5)), qd, dots=True)
    assert np.array_equal(host(qd), np.zeros(5)) and d == (0.0, 0.0)
    # single row holding every nonzero, and rows at the long-row threshold
    check_spmv(P.random_csr(1, 5000, seed=2))
    check_spmv(P.random_csr(3, 1, seed=3, long_rows={0: fk.LONG_ROW, 1: fk.LONG_ROW + 1, 2: 1}))
    blocks = fk.Matrix(P.random_csr(3, 1, seed=3, long_rows={0: fk.LONG_ROW, 1: fk.LONG_ROW + 1})).blocks()
    assert blocks[1] == 1


@pytest.mark.parametrize("layout", [None, "sliced", "row_blocks"], ids=["auto", "sliced", "row_blocks"])
def test_spmv_full_size_128(layout, device):
    """The 128^3 workload at full size in the launch configuration the
    benchmark uses (the library's own layout choice, sliced), and in row
    blocks: every row equal to the CSR-order sum."""
    A, _, _ = P.workload("poisson3d_128")
    check_spmv(A, seed=5, layout=layout)


@pytest.mark.parametrize("n", [1, 7, 255, 256, 257, 1000, 123457, 2097152])
def test_dot(n, device):
    rng = np.random.default_rng(n)
    a, b = rng.standard_normal(n), rng.uniform(-1, 1, n) * 1e3
    assert fk.dot(dev(a), dev(b)) == oracle.dot(a, b)
    assert fk.dot(dev(a), dev(a)) == oracle.dot(a, a)


def test_dot_cancellation(device):
    rng = np.random.default_rng(3)
    a = rng.standard_normal(100000) * 1e6
    b = rng.standard_normal(100000)
    a2 = np.concatenate([a, -a, [1e-3]])
    b2 = np.concatenate([b, b, [1.0]])
    got = fk.dot(dev(a2), dev(b2))
    assert got == oracle.dot(a2, b2)
    assert abs(got - 1e-3) < 1e-12


def test_reproducible(device):
    A, _, _ = P.workload("poisson3d_32")
    p = np.random.default_rng(0).uniform(-1, 1, A.n)
    M = fk.Matrix(A)
    outs = []
    for _ in range(3):
        qd = dev(np.zeros(A.n))
        d = fk.spmv(M, dev(p), qd, dots=True)
        outs.append((host(qd), d))
    for q, d in outs[1:]:
        assert np.array_equal(q, outs[0][0]) and d == outs[0][1]


@pytest.mark.parametrize("nbytes", [1, 15, 16, 17, 4096, 1000003, 64 << 20])
def test_copy(nbytes, device):
    import torch

    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device=device)
    dst = torch.zeros_like(src)
    fk.copy(dst, src, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


@pytest.mark.parametrize("mode", ["product", "fused", "split"])
def test_spmv_time(mode, device):
    """fk_spmv_time runs the product it times: q equals the oracle's A p and
    the fused reduction still completes; bad arguments are refused."""
    A = P.random_csr(5000, 4, seed=4)
    p = np.random.default_rng(7).uniform(-1, 1, A.n)
    M = fk.Matrix(A)
    pd, qd = dev(p), dev(np.zeros(A.n))
    us = fk.spmv_time(M, pd, qd, mode=mode, reps=5)
    assert us > 0.0
    assert np.array_equal(host(qd), oracle.spmv(A, p))
    dots = fk.spmv(M, pd, qd, dots=True)
    assert dots[1] == oracle.dot(host(qd), host(qd))
    L = fk.lib()
    out = ctypes.c_double()
    for reps, md in ((0, 1), (1, 3), (1, -1)):
        st = L.fk_spmv_time(M.handle, ctypes.c_void_p(pd.data_ptr()), ctypes.c_void_p(qd.data_ptr()), md, reps,
                            ctypes.byref(out), None)
        assert st == fk.E_ARG
    M.close()
