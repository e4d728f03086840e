"""Seeded synthetic inputs: sparse matrices in CSR form and right-hand sides.

This module only *builds inputs*.  It holds none of the solver arithmetic
(no products with vectors, no inner products, no iteration), so both the HIP
path and the CPU oracle may take their inputs from it.

The paper measures on 2D/3D finite-element meshes and on a set of public
sparse matrices (Section 4, Table 1); none of those are available here.  The
generators below stand in for them with finite-difference stencils of the
same sparsity regime (about 5 to 7 nonzeros per row) and the same size range,
plus the random-column matrices of the fused SpMV+dot microbenchmark
(Section 2.2, four and 28 uniformly random nonzeros per row).

Conventions for every stencil matrix:
  * homogeneous Dirichlet boundary, interior unknowns only;
  * lexicographic order with x fastest: row = ix + n*iy (+ n*n*iz);
  * column indices strictly ascending inside each row;
  * int32 row_ptr / col_idx, float64 values.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Csr:
    """A square CSR matrix held in host memory (numpy arrays)."""

    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col_idx: np.ndarray  # int32[nnz]
    vals: np.ndarray  # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.vals, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        np.add.at(d, (rows, self.col_idx), self.vals)
        return d


def _from_coo(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> Csr:
    """Sort (row, col) pairs and pack them as CSR; duplicates are kept as-is
    (in their input order: a stable sort on the key row * n + col)."""
    order = np.argsort(rows.astype(np.int64) * n + cols.astype(np.int64), kind="stable")
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz does not fit int32")
    return Csr(
        n=n,
        row_ptr=row_ptr.astype(np.int32),
        col_idx=cols.astype(np.int32),
        vals=np.ascontiguousarray(vals, dtype=np.float64),
    )


def _stencil(shape: tuple[int, ...], diag: float, offdiag: dict[tuple[int, ...], float]) -> Csr:
    """Constant-coefficient stencil on an interior grid of `shape` (x first).

    `offdiag` maps a neighbour offset (dx, dy[, dz]) to its coefficient;
    neighbours that fall outside the grid are dropped (Dirichlet).
    """
    dims = len(shape)
    n = int(np.prod(shape))
    coords = np.indices(shape[::-1], dtype=np.int32).reshape(dims, -1)[::-1]  # coords[0] = x
    strides = [1]
    for s in shape[:-1]:
        strides.append(strides[-1] * s)
    idx = np.arange(n, dtype=np.int64)
    # (column shift, coefficient, valid rows) per stencil entry; entries are
    # placed in ascending shift order, so columns come out sorted per row.
    entries = [(0, diag, None)]
    for off, coef in offdiag.items():
        ok = np.ones(n, dtype=bool)
        shift = 0
        for d in range(dims):
            c = coords[d] + off[d]
            ok &= (c >= 0) & (c < shape[d])
            shift += off[d] * strides[d]
        entries.append((shift, coef, ok))
    entries.sort(key=lambda e: e[0])
    counts = np.zeros(n, dtype=np.int64)
    for _, _, ok in entries:
        counts += 1 if ok is None else ok
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    if nnz > np.iinfo(np.int32).max:
        raise ValueError("nnz does not fit int32")
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    pos = row_ptr[:-1].copy()
    for shift, coef, ok in entries:
        rows = idx if ok is None else idx[ok]
        at = pos if ok is None else pos[ok]
        col[at] = rows + shift
        val[at] = coef
        if ok is None:
            pos += 1
        else:
            pos[ok] += 1
    return Csr(n=n, row_ptr=row_ptr.astype(np.int32), col_idx=col, vals=val)


def poisson2d(n: int, diag_shift: np.ndarray | float | None = None) -> Csr:
    """5-point Laplacian on an n x n interior grid: 4 on the diagonal, -1 off.

    `diag_shift` (scalar or length n*n) is added to the diagonal.
    """
    a = _stencil((n, n), 4.0, {(-1, 0): -1.0, (1, 0): -1.0, (0, -1): -1.0, (0, 1): -1.0})
    if diag_shift is not None:
        a = _add_diag(a, diag_shift)
    return a


def poisson3d(n: int) -> Csr:
    """7-point Laplacian on an n^3 interior grid: 6 on the diagonal, -1 off."""
    off = {}
    for d in range(3):
        for s in (-1, 1):
            o = [0, 0, 0]
            o[d] = s
            off[tuple(o)] = -1.0
    return _stencil((n, n, n), 6.0, off)


def convdiff2d(n: int, peclet: float = 50.0, direction=(1.0, 0.5)) -> Csr:
    """-Laplace(u) + v.grad(u) on the unit square, first-order upwind, scaled by h^2.

    v = peclet * direction (both components >= 0, so upwind = backward
    differences); h = 1/(n+1).  Row coefficients: diagonal 4 + h(vx+vy),
    west -(1 + h vx), south -(1 + h vy), east -1, north -1.  Nonsymmetric.
    """
    vx, vy = peclet * direction[0], peclet * direction[1]
    if vx < 0 or vy < 0:
        raise ValueError("upwind stencil here assumes nonnegative velocity")
    h = 1.0 / (n + 1)
    return _stencil(
        (n, n),
        4.0 + h * (vx + vy),
        {(-1, 0): -(1.0 + h * vx), (1, 0): -1.0, (0, -1): -(1.0 + h * vy), (0, 1): -1.0},
    )


def heat2d(n: int, c: float = 4.0, ny: int | None = None) -> Csr:
    """Backward-Euler heat operator I + c*L5 on an n x n (or n x ny) interior
    grid, x fastest (c = dt*kappa/h^2)."""
    return _stencil((n, n if ny is None else ny), 1.0 + 4.0 * c,
                    {(-1, 0): -c, (1, 0): -c, (0, -1): -c, (0, 1): -c})


def scaled_identity(n: int, lam: float) -> Csr:
    idx = np.arange(n)
    return _from_coo(n, idx, idx, np.full(n, float(lam)))


def _add_diag(a: Csr, shift) -> Csr:
    shift = np.broadcast_to(np.asarray(shift, dtype=np.float64), (a.n,))
    rows = np.repeat(np.arange(a.n), np.diff(a.row_ptr))
    vals = a.vals.copy()
    on_diag = rows == a.col_idx
    vals[on_diag] += shift[rows[on_diag]]
    return Csr(a.n, a.row_ptr, a.col_idx, vals)


def random_csr(n: int, nnz_per_row: int, seed: int = 0, empty_rows: int = 0,
               long_rows: dict[int, int] | None = None) -> Csr:
    """Rows with `nnz_per_row` column indices drawn uniformly from [0, n).

    Values are uniform in [-1, 1).  Duplicated column indices inside a row are
    kept (CSR allows them; a product sums them).  `empty_rows` rows (chosen by
    the same generator) get no entries; `long_rows` maps row -> its own count.
    """
    rng = np.random.default_rng(seed)
    counts = np.full(n, nnz_per_row, dtype=np.int64)
    if empty_rows:
        counts[rng.choice(n, size=empty_rows, replace=False)] = 0
    for r, c in (long_rows or {}).items():
        counts[r] = c
    rows = np.repeat(np.arange(n), counts)
    cols = rng.integers(0, n, size=rows.size)
    vals = rng.uniform(-1.0, 1.0, size=rows.size)
    return _from_coo(n, rows, cols, vals)


def random_spd_dense(n: int, cond: float, seed: int = 0) -> np.ndarray:
    """Dense SPD matrix Q diag(geomspace(1, cond)) Q^T with a seeded orthogonal Q."""
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, cond, n)
    return (q * lam) @ q.T


def dense_to_csr(a: np.ndarray, drop_zeros: bool = True) -> Csr:
    n = a.shape[0]
    if drop_zeros:
        rows, cols = np.nonzero(a)
    else:
        rows, cols = np.indices(a.shape).reshape(2, -1)
    return _from_coo(n, rows, cols, a[rows, cols])


def rhs_uniform(n: int, seed: int = 0) -> np.ndarray:
    """b uniform in [-1, 1) from numpy's default_rng(seed)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


# --- Closed-form spectral data of the stencil Laplacians (inputs for pins) ---

def laplacian_eigvec_2d(n: int, j: int, k: int) -> np.ndarray:
    """Eigenvector sin(j pi a/(n+1)) sin(k pi b/(n+1)) of the 5-point Laplacian, unit 2-norm."""
    a = np.arange(1, n + 1)
    v = np.outer(np.sin(k * np.pi * a / (n + 1)), np.sin(j * np.pi * a / (n + 1))).ravel()
    return v / np.linalg.norm(v)


def laplacian_eigval_2d(n: int, j: int, k: int) -> float:
    t = np.pi / (n + 1)
    return 4.0 - 2.0 * np.cos(j * t) - 2.0 * np.cos(k * t)


def laplacian_eigvec_3d(n: int, j: int, k: int, l: int) -> np.ndarray:
    a = np.arange(1, n + 1)
    sx = np.sin(j * np.pi * a / (n + 1))
    sy = np.sin(k * np.pi * a / (n + 1))
    sz = np.sin(l * np.pi * a / (n + 1))
    v = (sz[:, None, None] * sy[None, :, None] * sx[None, None, :]).ravel()
    return v / np.linalg.norm(v)


def laplacian_eigval_3d(n: int, j: int, k: int, l: int) -> float:
    t = np.pi / (n + 1)
    return 6.0 - 2.0 * (np.cos(j * t) + np.cos(k * t) + np.cos(l * t))


# --- The workloads -----------------------------------------------------------

def workload(name: str):
    """Return (A, b, x0) for a named workload.

    poisson2d_32     : 2D 5-point Poisson, 32x32 interior grid, N = 1,024
    poisson3d_128    : 3D 7-point Poisson, 128^3 interior grid, N = 2,097,152
    convdiff2d_1024  : 2D upwind convection-diffusion, 1024^2, Peclet 50, v=(1,0.5)
    poisson3d_<n>    : size variants used for sweeps and parity at reduced size
    poisson2d_<n>, convdiff2d_<n>, heat2d_<n> likewise.
    b = uniform[-1,1) from default_rng(0); x0 = 0.
    """
    kind, _, size = name.rpartition("_")
    n = int(size)
    if kind == "poisson2d":
        a = poisson2d(n)
    elif kind == "poisson3d":
        a = poisson3d(n)
    elif kind == "convdiff2d":
        a = convdiff2d(n)
    elif kind == "heat2d":
        a = heat2d(n)
    else:
        raise KeyError(name)
    b = rhs_uniform(a.n, 0)
    return a, b, np.zeros(a.n)


def heat_transient(n: int = 512, seed: int = 0, steps: int = 400, c: float = 4.0):
    """Transient 2D heat equation, backward Euler: A u^{m} = u^{m-1} + dt f^{m}.

    A = I + c L5 on the n x n interior grid of the unit square (points
    (i+1)/(n+1)).  u^0 is a sum of 16 Gaussians from default_rng(seed):
    centres uniform in [0.1, 0.9]^2, widths uniform in [0.03, 0.1], amplitudes
    uniform in [-1, 1].  dt f^m is a unit-amplitude Gaussian of width 0.05
    whose centre moves on a circle about (0.5, 0.5): for seed 0 radius 0.25,
    phase 0, counter-clockwise, one turn in `steps` steps; other seeds draw
    radius in [0.15, 0.35], a phase and a direction after the initial field.
    Returns (A, u0, source) with source(m) = dt f^m (m = 1 .. steps).
    """
    A = heat2d(n, c)
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.1, 0.9, (16, 2))
    widths = rng.uniform(0.03, 0.1, 16)
    amps = rng.uniform(-1.0, 1.0, 16)
    if seed == 0:
        radius, phase, direction = 0.25, 0.0, 1.0
    else:
        radius = rng.uniform(0.15, 0.35)
        phase = rng.uniform(0.0, 2.0 * np.pi)
        direction = float(rng.choice([-1.0, 1.0]))
    h = 1.0 / (n + 1)
    t = (np.arange(n) + 1.0) * h
    X = np.tile(t, n)      # x fastest: row = ix + n * iy
    Y = np.repeat(t, n)
    u0 = np.zeros(n * n)
    for (cx, cy), w, a in zip(centres, widths, amps):
        u0 += a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * w * w))

    def source(m: int) -> np.ndarray:
        th = phase + direction * 2.0 * np.pi * m / steps
        cx, cy = 0.5 + radius * np.cos(th), 0.5 + radius * np.sin(th)
        return np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * 0.05 * 0.05))

    return A, u0, source


def net_init(layers: int, seed: int = 0, channels: int = 16) -> np.ndarray:
    """Initial weights of the warm-start network, canonical order (layer after
    layer, W[co][ci][ky][kx]; 1 input and 1 output channel): uniform in
    +-sqrt(6 / (9 cin)) from default_rng(seed), the last layer scaled by 0.1
    so that the first guesses stay close to the extrapolation.  float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(layers):
        cin = 1 if l == 0 else channels
        cout = 1 if l == layers - 1 else channels
        bound = np.sqrt(6.0 / (9 * cin)) * (0.1 if l == layers - 1 else 1.0)
        parts.append(rng.uniform(-bound, bound, cout * cin * 9))
    return np.concatenate(parts).astype(np.float32)


def batch_systems(count: int = 512, seed: int = 0, nmin: int = 16, nmax: int = 512):
    """Uneven batch: 2D Poisson on n_s x n_s grids plus a random diagonal shift.

    n_s = rng.integers(nmin, nmax+1, count); then, for each system in order,
    shift = rng.uniform(0, 0.1, n_s^2) and b = rng.uniform(-1, 1, n_s^2).
    Yields (n_s, shift, b) without assembling the matrices.
    """
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, count)
    for ns in sizes:
        shift = rng.uniform(0.0, 0.1, int(ns) * int(ns))
        b = rng.uniform(-1.0, 1.0, int(ns) * int(ns))
        yield int(ns), shift, b


def block_diagonal(systems) -> tuple[Csr, np.ndarray]:
    """Stack square CSR matrices into one block-diagonal CSR matrix; returns
    it and sys_ptr (row offsets, int64, count + 1 entries)."""
    systems = list(systems)
    sizes = np.array([a.n for a in systems], dtype=np.int64)
    sys_ptr = np.concatenate([[0], np.cumsum(sizes)])
    nnzs = np.array([a.nnz for a in systems], dtype=np.int64)
    nnz_ptr = np.concatenate([[0], np.cumsum(nnzs)])
    n, nnz = int(sys_ptr[-1]), int(nnz_ptr[-1])
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col_idx = np.empty(nnz, dtype=np.int32)
    vals = np.empty(nnz, dtype=np.float64)
    for s, a in enumerate(systems):
        r0, j0 = int(sys_ptr[s]), int(nnz_ptr[s])
        row_ptr[r0: r0 + a.n] = a.row_ptr[:-1] + j0
        col_idx[j0: j0 + a.nnz] = a.col_idx + r0
        vals[j0: j0 + a.nnz] = a.vals
    row_ptr[n] = nnz
    return Csr(n, row_ptr, col_idx, vals), sys_ptr


def batch_problem(count: int = 512, seed: int = 0, nmin: int = 16, nmax: int = 512):
    """The uneven batch as (block-diagonal A, sys_ptr, b): system s is the 2D
    5-point Laplacian on an n_s x n_s grid plus its diagonal shift, with its
    right-hand side, in the draw order of batch_systems.  Each system is
    written straight into the batch arrays."""
    draws = list(batch_systems(count, seed, nmin, nmax))
    sizes = np.array([ns * ns for ns, _, _ in draws], dtype=np.int64)
    nnzs = np.array([5 * ns * ns - 4 * ns for ns, _, _ in draws], dtype=np.int64)
    sys_ptr = np.concatenate([[0], np.cumsum(sizes)])
    nnz_ptr = np.concatenate([[0], np.cumsum(nnzs)])
    n, nnz = int(sys_ptr[-1]), int(nnz_ptr[-1])
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col_idx = np.empty(nnz, dtype=np.int32)
    vals = np.empty(nnz, dtype=np.float64)
    b = np.empty(n, dtype=np.float64)
    for s, (ns, shift, bs) in enumerate(draws):
        a = poisson2d(ns)
        r0, j0 = int(sys_ptr[s]), int(nnz_ptr[s])
        assert a.nnz == nnzs[s]
        row_ptr[r0: r0 + a.n] = a.row_ptr[:-1] + j0
        col_idx[j0: j0 + a.nnz] = a.col_idx + r0
        v = vals[j0: j0 + a.nnz]
        v[:] = a.vals
        # the diagonal follows the south and west neighbours in each row
        ix = np.tile(np.arange(ns), ns)
        iy = np.repeat(np.arange(ns), ns)
        v[a.row_ptr[:-1] + (iy > 0) + (ix > 0)] += shift
        b[r0: r0 + a.n] = bs
    row_ptr[n] = nnz
    return Csr(n, row_ptr, col_idx, vals), sys_ptr, b


def system_of(A: Csr, sys_ptr, s: int) -> Csr:
    """System s of a block-diagonal batch as its own CSR matrix."""
    r0, r1 = int(sys_ptr[s]), int(sys_ptr[s + 1])
    j0, j1 = int(A.row_ptr[r0]), int(A.row_ptr[r1])
    return Csr(r1 - r0, (A.row_ptr[r0: r1 + 1] - j0).astype(np.int32), (A.col_idx[j0:j1] - r0).astype(np.int32),
               A.vals[j0:j1].copy())
