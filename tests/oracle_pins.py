"""Pins of the CPU oracle against facts fixed outside it.

Every function takes an oracle instance (oracle.Oracle) and raises
AssertionError when the oracle disagrees with something the paper or the
mathematics fixes: closed-form Laplacian eigenpairs, exact sine-transform
solves, dense LAPACK solves, exact rational arithmetic, finite termination,
and the identities the pipelined recurrences rest on (Eq. (3) and the
BiCGStab derivations of Section 3.2).  test_oracle_pins.py runs them on the
oracle; test_oracle_mutations.py runs them on copies of oracle.c with a
planted mistake and requires each copy to fail at least one pin.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import scipy.fft
import scipy.sparse

from paper_1410_4054_amd import problems as P

CG = ("cg_classical", "cg_pipelined")
BICG = ("bicgstab_classical", "bicgstab_pipelined")
ALL = CG + BICG


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


# --------------------------------------------------------------- products

def pin_spmv_bruteforce(O):
    """CSR product of Section 2.2: each row summed left to right, checked bit
    for bit against Python float arithmetic (IEEE double, one rounding per
    operation) on a small matrix with duplicates, empty and long rows."""
    A = P.random_csr(60, 5, seed=3, empty_rows=4, long_rows={7: 40})
    p = np.random.default_rng(4).uniform(-1, 1, A.n)
    q = O.spmv(A, p)
    for i in range(A.n):
        acc = 0.0
        for j in range(A.row_ptr[i], A.row_ptr[i + 1]):
            acc = acc + float(A.vals[j]) * float(p[A.col_idx[j]])
        assert q[i] == acc, (i, q[i], acc)
    assert _rel(q, A.to_dense() @ p) < 1e-14


def pin_spmv_scipy(O):
    """CSR product against scipy.sparse on 4 and 28 random nonzeros per row
    (the matrices of the fused SpMV+dot benchmark, Section 2.2)."""
    for nz, seed in ((4, 1), (28, 2)):
        A = P.random_csr(3000, nz, seed=seed, empty_rows=5)
        p = np.random.default_rng(seed).standard_normal(A.n)
        np.testing.assert_allclose(O.spmv(A, p), A.to_scipy() @ p, rtol=1e-12, atol=1e-13)


def _exact_dot(a, b) -> float:
    s = Fraction(0)
    for x, y in zip(a, b):
        s += Fraction(float(x)) * Fraction(float(y))
    return float(s)  # Fraction -> float rounds to nearest


def pin_dot_rounding(O):
    """<a, b> against the exactly rounded sum of exact products (rational
    arithmetic).  The oracle's dot is accurate as if computed in twice the
    working precision: |res - s| <= eps |s| + gamma_n^2 sum |a_i b_i|
    (Ogita, Rump, Oishi 2005).  Checked on wide-range and on cancelling data;
    on moderately conditioned data it must also equal the correctly rounded
    value in the vast majority of cases."""
    rng = np.random.default_rng(11)
    eps = 2.0 ** -53
    exact_hits = total = 0
    for t in range(160):
        n = int(rng.integers(1, 120))
        a = rng.standard_normal(n) * 10.0 ** rng.integers(-8, 8, n)
        b = rng.standard_normal(n)
        cancel = t % 4 == 1
        if cancel:  # exact cancellation down to a tiny remainder
            a = np.concatenate([a, -a[::-1], [1e-20]])
            b = np.concatenate([b, b[::-1], [3.0]])
        got = O.dot(a, b)
        ref = _exact_dot(a, b)
        m = a.size
        gamma = m * eps / (1 - m * eps)
        bound = eps * abs(ref) + gamma ** 2 * float(np.sum(np.abs(a * b))) * 1.01
        assert abs(got - ref) <= max(bound, math.ulp(ref) / 2), (t, got, ref)
        if not cancel and ref != 0.0:
            exact_hits += got == ref
            total += 1
    assert exact_hits >= 0.95 * total, (exact_hits, total)
    assert O.dot(np.zeros(0), np.zeros(0)) == 0.0


# ------------------------------------------------------- closed-form spectra

def pin_eigenvector_one_step(O):
    """b = an eigenvector of the 2D/3D Laplacian (closed form): every method
    converges in exactly one iteration with alpha_0 = 1/lambda and x = b/lambda."""
    cases = [
        (P.poisson2d(16), P.laplacian_eigvec_2d(16, 3, 5), P.laplacian_eigval_2d(16, 3, 5)),
        (P.poisson3d(8), P.laplacian_eigvec_3d(8, 2, 3, 4), P.laplacian_eigval_3d(8, 2, 3, 4)),
    ]
    for A, v, lam in cases:
        assert np.allclose(A.to_scipy() @ v, lam * v, atol=1e-13)
        for m in ALL:
            res = O.solve(A, v, method=m, rtol=1e-10, trace=True)
            assert res.status == "converged" and res.k == 1, (m, res.k, res.status)
            assert _rel(res.x, v / lam) < 1e-13, m
            assert abs(res.t("alpha")[0] * lam - 1.0) < 1e-13, m


def pin_distinct_eigenvalues_terminate(O):
    """b spanning m eigenvectors with m distinct eigenvalues: CG reaches
    machine-level residual after exactly m iterations and not before."""
    n = 20
    A = P.poisson2d(n)
    picks = [(1, 1), (2, 5), (4, 4), (7, 3), (9, 9)]
    lams = [P.laplacian_eigval_2d(n, j, k) for j, k in picks]
    assert len(set(np.round(lams, 12))) == len(picks)
    b = sum((i + 1.0) * P.laplacian_eigvec_2d(n, j, k) for i, (j, k) in enumerate(picks))
    m = len(picks)
    for meth in CG:
        res = O.solve(A, b, method=meth, rtol=0.0, max_iter=m)
        assert res.hist[m] < 1e-10, (meth, res.hist)
        assert res.hist[m - 1] > 1e-6, (meth, res.hist)


def _dst_solve_2d(n, b):
    t = np.pi * np.arange(1, n + 1) / (n + 1)
    lam = 4.0 - 2.0 * np.cos(t)[:, None] - 2.0 * np.cos(t)[None, :]
    bh = scipy.fft.dstn(b.reshape(n, n), type=1, norm="ortho")
    return scipy.fft.idstn(bh / lam, type=1, norm="ortho").ravel(), lam.max() / lam.min()


def _dst_solve_3d(n, b):
    t = np.pi * np.arange(1, n + 1) / (n + 1)
    c = np.cos(t)
    lam = 6.0 - 2.0 * (c[:, None, None] + c[None, :, None] + c[None, None, :])
    bh = scipy.fft.dstn(b.reshape(n, n, n), type=1, norm="ortho")
    return scipy.fft.idstn(bh / lam, type=1, norm="ortho").ravel(), lam.max() / lam.min()


def pin_exact_poisson_solution(O):
    """Poisson problems solved exactly by the separable sine transform; the
    CG iterate at rtol must lie within kappa*rtol of it, and the solver's
    residual must equal the true residual up to roundoff."""
    rtol = 1e-12
    for A, (xs, kappa) in (
        (P.poisson2d(31), _dst_solve_2d(31, P.rhs_uniform(31 * 31, 0))),
        (P.poisson3d(15), _dst_solve_3d(15, P.rhs_uniform(15 ** 3, 0))),
    ):
        b = P.rhs_uniform(A.n, 0)
        assert _rel(A.to_scipy() @ xs, b) < 1e-13
        for m in ALL:
            res = O.solve(A, b, method=m, rtol=rtol)
            assert res.status == "converged", m
            assert _rel(res.x, xs) <= kappa * rtol * 1.01, (m, _rel(res.x, xs))
            tr = O.true_residual(A, b, res.x)
            assert tr <= rtol * 1.5, (m, tr)


def pin_dense_lapack(O):
    """Tiny SPD and nonsymmetric systems against LAPACK (numpy.linalg.solve)."""
    rtol = 1e-13
    Ad = P.random_spd_dense(40, 100.0, seed=5)
    A = P.dense_to_csr(Ad)
    b = np.random.default_rng(6).standard_normal(40)
    xs = np.linalg.solve(Ad, b)
    for m in ALL:
        res = O.solve(A, b, method=m, rtol=rtol)
        assert res.status == "converged", m
        assert _rel(res.x, xs) <= 100.0 * rtol * 2, (m, _rel(res.x, xs))
    rng = np.random.default_rng(7)
    for A in (P.convdiff2d(6), P.dense_to_csr(np.eye(50) * 4 + rng.uniform(-0.5, 0.5, (50, 50)))):
        Ad = A.to_dense()
        b = rng.standard_normal(A.n)
        xs = np.linalg.solve(Ad, b)
        kappa = np.linalg.cond(Ad)
        for m in BICG:
            res = O.solve(A, b, method=m, rtol=rtol)
            assert res.status == "converged", m
            assert _rel(res.x, xs) <= kappa * rtol * 2, (m, _rel(res.x, xs))


def pin_cg_finite_termination(O):
    """CG on a random SPD system of size N <= 12 reaches a residual below
    1e-10 within N iterations.  (Exact-arithmetic termination; in FP64 loss
    of orthogonality delays it once the condition number grows, so the
    systems here have condition numbers 5 to 30.)"""
    for n, cond, seed in ((5, 10.0, 1), (8, 10.0, 2), (12, 10.0, 3), (12, 5.0, 4), (10, 30.0, 5)):
        A = P.dense_to_csr(P.random_spd_dense(n, cond, seed=seed))
        b = np.random.default_rng(seed).standard_normal(n)
        for m in CG:
            res = O.solve(A, b, method=m, rtol=0.0, max_iter=n)
            assert res.hist[-1] <= 1e-10, (m, n, res.hist[-1])


# ------------------------------------------------------------ invariants

def pin_cg_invariants(O):
    """Classical CG: consecutive residuals orthogonal, consecutive search
    directions A-conjugate, recursive residual = true residual up to
    roundoff; pipelined CG: Eq. (3) gives the same beta as the ratio
    <r_{i+1},r_{i+1}>/<r_i,r_i>."""
    A = P.poisson2d(24)
    b = P.rhs_uniform(A.n, 1)
    S = A.to_scipy()
    runs = [O.solve(A, b, method="cg_classical", rtol=0.0, max_iter=k) for k in (20, 21, 22)]
    r20, r21 = runs[0].r, runs[1].r
    assert abs(r20 @ r21) <= 1e-10 * np.linalg.norm(r20) * np.linalg.norm(r21)
    d1 = runs[1].x - runs[0].x  # proportional to p_20
    d2 = runs[2].x - runs[1].x  # proportional to p_21
    assert abs(d2 @ (S @ d1)) <= 1e-9 * np.linalg.norm(d2) * np.linalg.norm(S @ d1)
    for res in runs:
        gap = np.linalg.norm(res.r - (b - S @ res.x)) / np.linalg.norm(b)
        assert gap < 1e-13, gap
    pr = O.solve(A, b, method="cg_pipelined", rtol=0.0, max_iter=40, trace=True)
    rr = pr.t("rr")  # <r_i, r_i> at the start of step i
    beta = pr.t("beta")
    ratio = rr[1:] / rr[:-1]
    np.testing.assert_allclose(beta[:-1], ratio, rtol=1e-9)


def pin_bicgstab_invariants(O):
    """Pipelined BiCGStab: beta from <As,r0*>/<Ap,r0*> equals the classical
    (rho_{i+1}/rho_i)(alpha_i/omega_i), i.e. <s_i, r0*> = 0; the expanded
    <r_{i+1},r_{i+1}> equals the directly computed one; the recursive
    residual stays the true residual."""
    A = P.convdiff2d(20)
    b = P.rhs_uniform(A.n, 2)
    res = O.solve(A, b, method="bicgstab_pipelined", rtol=0.0, max_iter=12, trace=True)
    alpha, omega, beta, rho = res.t("alpha"), res.t("omega"), res.t("beta"), res.t("rho")
    classical_beta = (rho[1:] / rho[:-1]) * (alpha[:-1] / omega[:-1])
    np.testing.assert_allclose(beta[:-1], classical_beta, rtol=1e-7)
    np.testing.assert_allclose(res.t("rr_expanded"), res.t("rr_direct"), rtol=1e-9)
    gap = np.linalg.norm(res.r - (b - A.to_scipy() @ res.x)) / np.linalg.norm(b)
    assert gap < 1e-12, gap
    cl = O.solve(A, b, method="bicgstab_classical", rtol=0.0, max_iter=12, trace=True)
    np.testing.assert_allclose(cl.t("alpha"), alpha, rtol=1e-7)
    np.testing.assert_allclose(cl.t("omega"), omega, rtol=1e-7)


def pin_classical_vs_pipelined(O):
    """Classical and pipelined CG agree after 30 iterations to well below
    1e-10 (the comparison of Table 2)."""
    for A in (P.poisson2d(32), P.poisson3d(16)):
        b = P.rhs_uniform(A.n, 0)
        c = O.solve(A, b, method="cg_classical", rtol=0.0, max_iter=30)
        p = O.solve(A, b, method="cg_pipelined", rtol=0.0, max_iter=30)
        assert _rel(p.x, c.x) < 1e-12
        assert abs(p.hist[-1] / c.hist[-1] - 1.0) < 1e-10


# ------------------------------------------------------- special cases

def pin_special_cases(O):
    """A = lambda I converges in one step; b = 0 gives x = 0 and k = 0; a
    starting guess that already solves the system gives k = 0; a nonzero
    starting guess converges to the LAPACK solution; max_iter bounds k."""
    A = P.scaled_identity(10, 2.5)
    b = np.arange(1.0, 11.0)
    for m in ALL:
        res = O.solve(A, b, method=m, rtol=1e-12)
        assert res.k == 1 and res.status == "converged", m
        assert np.allclose(res.x, b / 2.5, rtol=1e-15), m
        z = O.solve(A, np.zeros(10), x0=np.ones(10), method=m)
        assert z.k == 0 and z.status == "converged" and not z.x.any(), m
    Ad = P.random_spd_dense(30, 50.0, seed=8)
    A = P.dense_to_csr(Ad)
    b = np.random.default_rng(9).standard_normal(30)
    xs = np.linalg.solve(Ad, b)
    for m in ALL:
        res = O.solve(A, b, x0=xs, method=m, rtol=1e-8)
        assert res.k == 0 and res.status == "converged", m
        x0 = np.random.default_rng(10).standard_normal(30) * 3.0
        res = O.solve(A, b, x0=x0, method=m, rtol=1e-13)
        assert res.status == "converged" and _rel(res.x, xs) < 1e-10, m
        r0 = O.solve(A, b, x0=x0, method=m, rtol=0.0, max_iter=0)
        assert r0.k == 0 and r0.status == "not_converged", m
        np.testing.assert_allclose(r0.r, b - Ad @ x0, rtol=1e-13, atol=1e-13)
        r7 = O.solve(A, b, method=m, rtol=0.0, max_iter=7)
        assert r7.k == 7 and r7.status == "not_converged", m


def pin_breakdown(O):
    """CG on an indefinite matrix meets <p, Ap> <= 0; BiCGStab on a
    skew-symmetric matrix meets <A r0, r0*> = 0; both report breakdown."""
    d = np.array([1.0, -1.0, 2.0, -2.0])
    A = P.dense_to_csr(np.diag(d))
    b = np.ones(4)
    for m in CG:
        assert O.solve(A, b, method=m).status == "breakdown", m
    S = np.zeros((4, 4))
    S[0, 1], S[1, 0], S[2, 3], S[3, 2] = 1.0, -1.0, 2.0, -2.0
    A = P.dense_to_csr(S)
    for m in BICG:
        assert O.solve(A, b, method=m).status == "breakdown", m


# ------------------------------------------------- GMRES(m), Algorithms 5-6

def _krylov_lstsq(M, b, x0, k):
    """Minimiser of ||b - M x|| over x0 + K_k(M, r0), by dense least squares."""
    r0 = b - M @ x0
    K = np.zeros((len(b), k))
    v = r0.copy()
    for j in range(k):
        K[:, j] = v / np.linalg.norm(v)
        v = M @ K[:, j]
    Q, _ = np.linalg.qr(K)
    c, *_ = np.linalg.lstsq(M @ Q, r0, rcond=None)
    return x0 + Q @ c


def pin_gmres_least_squares(O):
    """Without a restart, GMRES's iterate after k steps is the minimiser of
    the residual over x0 + K_k (dense least squares), and its history entry
    is that minimum residual; both Gram-Schmidt forms agree."""
    n = 30
    rng = np.random.default_rng(21)
    M = 3.0 * np.eye(n) + rng.uniform(-0.5, 0.5, (n, n))
    A = P.dense_to_csr(M)
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n) * 0.1
    for k in (1, 2, 5, 9):
        xr = _krylov_lstsq(M, b, x0, k)
        res_ref = np.linalg.norm(b - M @ xr) / np.linalg.norm(b)
        for pip in (True, False):
            r = O.solve_gmres(A, b, x0=x0, m=40, pipelined=pip, rtol=0.0, max_iter=k)
            assert r.k == k and r.status == "not_converged", (k, pip, r.k, r.status)
            assert _rel(r.x, xr) < 1e-11, (k, pip, _rel(r.x, xr))
            assert abs(r.hist[k - 1 + 1] - res_ref) <= 1e-10 * res_ref + 1e-15, (k, pip)


def pin_gmres_termination_and_restarts(O):
    """A diagonalizable matrix with 3 distinct eigenvalues: GMRES stops after
    3 steps; lambda I after 1; restarted GMRES(m) on convection-diffusion
    meets the tolerance on the true residual; b = 0 gives x = 0."""
    n = 24
    rng = np.random.default_rng(22)
    S = np.eye(n) + 0.2 * rng.standard_normal((n, n))
    lam = np.repeat([1.0, 2.5, 4.0], n // 3)
    M = S @ np.diag(lam) @ np.linalg.inv(S)
    A = P.dense_to_csr(M)
    b = rng.standard_normal(n)
    for pip in (True, False):
        r = O.solve_gmres(A, b, m=10, pipelined=pip, rtol=1e-10)
        assert r.status == "converged" and r.k == 3, (pip, r.k, r.status)
        assert np.linalg.norm(b - M @ r.x) <= 1e-9 * np.linalg.norm(b)
        z = O.solve_gmres(P.scaled_identity(9, 2.0), np.arange(1.0, 10.0), m=5, pipelined=pip, rtol=1e-12)
        assert z.k == 1 and np.allclose(z.x, np.arange(1.0, 10.0) / 2.0, rtol=1e-15)
        e = O.solve_gmres(A, np.zeros(n), x0=np.ones(n), pipelined=pip)
        assert e.k == 0 and e.status == "converged" and not e.x.any()
    Ac, bc, _ = P.workload("convdiff2d_32")
    for m in (5, 20):
        rs = [O.solve_gmres(Ac, bc, m=m, pipelined=pip, rtol=1e-9) for pip in (True, False)]
        for r in rs:
            assert r.status == "converged"
            assert np.linalg.norm(bc - Ac.to_scipy() @ r.x) <= 1.0001e-9 * np.linalg.norm(bc)
        assert abs(rs[0].k - rs[1].k) <= 1 and _rel(rs[0].x, rs[1].x) < 1e-8


# ------------------------------------ iterative refinement, FP32 inner CG

def pin_f32_products(O):
    """FP32 CSR product and FP32 dot of the refinement's inner solver: the
    product bit for bit against numpy float32 scalar arithmetic (IEEE single,
    one rounding per operation, rows left to right); the dot within one
    rounding of the exact rational value of the float operands."""
    A = P.random_csr(50, 5, seed=11, empty_rows=3, long_rows={5: 30})
    p = np.random.default_rng(12).uniform(-1, 1, A.n).astype(np.float32)
    q = O.spmv_f32(A, p)
    v32 = A.vals.astype(np.float32)
    for i in range(A.n):
        acc = np.float32(0.0)
        for j in range(A.row_ptr[i], A.row_ptr[i + 1]):
            acc = np.float32(acc + np.float32(v32[j] * p[A.col_idx[j]]))
        assert q[i] == acc, (i, q[i], acc)
    rng = np.random.default_rng(13)
    for n in (1, 7, 300):
        a = rng.standard_normal(n).astype(np.float32)
        b = rng.standard_normal(n).astype(np.float32)
        exact = sum(Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b))
        got = O.dot_f32(a, b)
        assert abs(Fraction(got) - exact) <= abs(exact) * Fraction(2) ** -52, (n, got, float(exact))


def pin_f32acc_dot(O):
    """The FP32-accumulating dot of the second inner solver: within the
    recursive-summation bound gamma_n sum |a_i b_i| (u = 2^-24) of the exact
    rational value; exact when every product and partial sum is a small
    integer; each product rounded to FP32 before it is added ((1 + 2^-12)^2
    gives 1 + 2^-11, not the exact 1 + 2^-11 + 2^-24); and the sum kept in
    FP32 left to right (2^24 + 1 + 1 + 1 + 1 stays 2^24 by round-to-even,
    where a wider or reordered sum would not)."""
    u = Fraction(1, 2 ** 24)
    rng = np.random.default_rng(21)
    for n in (1, 7, 300, 4000):
        a = rng.standard_normal(n).astype(np.float32)
        b = rng.standard_normal(n).astype(np.float32)
        prods = [Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b)]
        exact = sum(prods)
        gamma = n * u / (1 - n * u)
        got = O.dot_f32acc(a, b)
        assert isinstance(got, np.float32)
        assert abs(Fraction(float(got)) - exact) <= gamma * sum(abs(t) for t in prods), (n, got)
    ia = rng.integers(-50, 51, 500).astype(np.float32)
    ib = rng.integers(-50, 51, 500).astype(np.float32)
    assert float(O.dot_f32acc(ia, ib)) == float(np.dot(ia.astype(np.int64), ib.astype(np.int64)))
    one = np.float32(1.0 + 2.0 ** -12)
    assert float(O.dot_f32acc(np.array([one]), np.array([one]))) == 1.0 + 2.0 ** -11
    # 2^-25 first, then (1 + 2^-12)^2: rounding the product first gives
    # 1 + 2^-11 and the sum stays there; one rounding of the exact sum would
    # give 1 + 2^-11 + 2^-23.
    sa = np.array([2.0 ** -12, one], dtype=np.float32)
    sb = np.array([2.0 ** -13, one], dtype=np.float32)
    assert float(O.dot_f32acc(sa, sb)) == 1.0 + 2.0 ** -11
    big = np.array([2.0 ** 24, 1, 1, 1, 1], dtype=np.float32)
    assert float(O.dot_f32acc(big, np.ones(5, np.float32))) == 2.0 ** 24
    assert float(O.dot_f32acc(big[::-1].copy(), np.ones(5, np.float32))) == 2.0 ** 24 + 4
    assert float(O.dot_f32acc(np.zeros(0, np.float32), np.zeros(0, np.float32))) == 0.0


ACCS = ("exact", "f32")


def pin_mixed_identity(O):
    """A = 4 I with b exactly representable in FP32: the inner CG takes one
    step (alpha = 1/4, beta = 0), the FP64 update gives x = b/4 exactly and
    the next residual is 0, so one sweep and one inner iteration."""
    A = P.scaled_identity(12, 4.0)
    b = np.arange(-6.0, 6.0) / 8.0 + 0.03125
    for acc in ACCS:
        res = O.solve_mixed(A, b, rtol=1e-14, acc=acc)
        assert res.status == "converged" and res.sweeps == 1 and res.k == 1, (acc, res)
        assert np.array_equal(res.x, b / 4.0)
        assert res.hist[1] == 0.0 and res.hist[0] == 1.0


def pin_mixed_eigen_termination(O):
    """b spanning 3 Laplacian eigenvectors with distinct eigenvalues (closed
    form): the FP32 inner CG of the first sweep terminates after exactly 3
    iterations at inner_rtol = 1e-3 (finite termination of Algorithm 2)."""
    n = 20
    A = P.poisson2d(n)
    picks = [(1, 2), (3, 3), (6, 1)]
    b = sum((i + 1.0) * P.laplacian_eigvec_2d(n, j, k) for i, (j, k) in enumerate(picks))
    for acc in ACCS:
        res = O.solve_mixed(A, b, rtol=1e-10, inner_rtol=1e-3, acc=acc)
        assert res.status == "converged", (acc, res)
        assert res.inner_k[0] == len(picks), (acc, res.inner_k)


def pin_mixed_exact_poisson(O):
    """Refinement on Poisson problems solved exactly by the sine transform:
    x within kappa*rtol of the exact solution, the last recorded residual
    equal to the true residual computed by scipy, and every sweep cutting
    the residual by at least 1e-3 (inner_rtol = 1e-4, kappa * eps_32 << 1)."""
    rtol = 1e-11
    for A, (xs, kappa) in (
        (P.poisson2d(31), _dst_solve_2d(31, P.rhs_uniform(31 * 31, 0))),
        (P.poisson3d(15), _dst_solve_3d(15, P.rhs_uniform(15 ** 3, 0))),
    ):
        b = P.rhs_uniform(A.n, 0)
        for acc in ACCS:
            res = O.solve_mixed(A, b, rtol=rtol, inner_rtol=1e-4, acc=acc)
            assert res.status == "converged", (acc, res)
            assert _rel(res.x, xs) <= kappa * rtol * 1.01, (acc, _rel(res.x, xs))
            tr = float(np.linalg.norm(b - A.to_scipy() @ res.x) / np.linalg.norm(b))
            assert tr <= rtol and abs(res.hist[-1] - tr) <= 1e-3 * tr, (acc, tr, res.hist)
            assert res.hist[0] == 1.0
            assert np.all(res.hist[1:] <= 1e-3 * res.hist[:-1]), (acc, res.hist)
            assert res.k == int(res.inner_k.sum())


def pin_mixed_fp32_floor(O):
    """One sweep with a very tight inner tolerance stops at the FP32 level:
    the true residual of x_1 (scipy, FP64) lies between 1e-9 and 1e-4, far
    above what the same number of FP64 iterations reaches, and equals the
    recorded history entry."""
    A = P.poisson2d(31)
    b = P.rhs_uniform(A.n, 1)
    for acc in ACCS:
        res = O.solve_mixed(A, b, rtol=1e-14, inner_rtol=1e-13, max_iter=400, max_outer=1, acc=acc)
        assert res.sweeps == 1 and res.status == "not_converged", (acc, res)
        tr = float(np.linalg.norm(b - A.to_scipy() @ res.x) / np.linalg.norm(b))
        assert 1e-9 < tr < 1e-4, (acc, tr)
        assert abs(res.hist[1] - tr) <= 1e-6 * tr, (acc, res.hist, tr)
        r64 = O.solve(A, b, method="cg_pipelined", rtol=0.0, max_iter=res.k)
        assert O.true_residual(A, b, r64.x) < 1e-3 * tr


def pin_mixed_special_cases(O):
    """b = 0 gives x = 0; limits on inner iterations and sweeps; an inner
    tolerance >= 1 makes no step and ends the solve unconverged; a dense SPD
    system reaches the LAPACK solution; a starting guess that already solves
    the system gives no sweep."""
    A = P.poisson2d(10)
    b = P.rhs_uniform(A.n, 3)
    Ad = P.random_spd_dense(30, 50.0, seed=8)
    Ac = P.dense_to_csr(Ad)
    bd = np.random.default_rng(9).standard_normal(30)
    xs = np.linalg.solve(Ad, bd)
    for acc in ACCS:
        z = O.solve_mixed(A, np.zeros(A.n), x0=np.ones(A.n), acc=acc)
        assert z.status == "converged" and z.k == 0 and z.sweeps == 0 and not z.x.any()
        r5 = O.solve_mixed(A, b, max_iter=5, acc=acc)
        assert r5.status == "not_converged" and r5.k == 5 and r5.sweeps == 1, (acc, r5)
        r2 = O.solve_mixed(A, b, inner_rtol=0.5, max_outer=2, acc=acc)
        assert r2.status == "not_converged" and r2.sweeps == 2 and len(r2.hist) == 3, (acc, r2)
        assert r2.hist[2] < r2.hist[1] < r2.hist[0]
        s = O.solve_mixed(A, b, inner_rtol=2.0, acc=acc)
        assert s.status == "not_converged" and s.k == 0 and s.sweeps == 0, (acc, s)
        res = O.solve_mixed(Ac, bd, rtol=1e-12, acc=acc)
        assert res.status == "converged" and _rel(res.x, xs) < 1e-10, (acc, res)
        w = O.solve_mixed(Ac, bd, x0=xs, rtol=1e-10, acc=acc)
        assert w.status == "converged" and w.k == 0 and w.sweeps == 0, (acc, w)


PINS = [
    pin_spmv_bruteforce,
    pin_spmv_scipy,
    pin_dot_rounding,
    pin_eigenvector_one_step,
    pin_distinct_eigenvalues_terminate,
    pin_exact_poisson_solution,
    pin_dense_lapack,
    pin_cg_finite_termination,
    pin_cg_invariants,
    pin_bicgstab_invariants,
    pin_classical_vs_pipelined,
    pin_special_cases,
    pin_breakdown,
    pin_gmres_least_squares,
    pin_gmres_termination_and_restarts,
    pin_f32_products,
    pin_f32acc_dot,
    pin_mixed_identity,
    pin_mixed_eigen_termination,
    pin_mixed_exact_poisson,
    pin_mixed_fp32_floor,
    pin_mixed_special_cases,
]
