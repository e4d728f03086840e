/*
 * Plain FP64 CPU oracle for the Krylov solvers of Rupp, Weinbub, Juengel and
 * Grasser, "Pipelined Iterative Solvers with Kernel Fusion for Graphics
 * Processing Units" (arXiv:1410.4054).
 *
 * TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the benchmark's CPU
 * baseline call it to obtain expected values.  The GPU library never links,
 * loads or calls this file and shares no code, header or constant with it.
 *
 * Everything is sequential, in the order the paper states it:
 *   - oracle_spmv   : q = A p, one row at a time, each row summed left to
 *                     right in CSR order (Section 2.2, the CSR product);
 *   - oracle_dot    : <a, b> computed as if in twice the working precision
 *                     (the compensated "Dot2" of Ogita, Rump and Oishi,
 *                     SIAM J. Sci. Comput. 26(6), 2005), then rounded once;
 *   - cg_classical       : Algorithm 1;
 *   - cg_pipelined       : Algorithm 2 with the beta recurrence of Eq. (3);
 *   - bicgstab_classical : Algorithm 3;
 *   - bicgstab_pipelined : Algorithm 4, beta from the orthogonality
 *                          <s_i, r0*> = 0 and the residual norm from the
 *                          expansion of <r_{i+1}, r_{i+1}> (Section 3.2);
 *   - gmres (methods 4, 5): restarted simpler GMRES(m) with classical
 *                          Gram-Schmidt, Algorithm 5 (residual updated in
 *                          the loop) and Algorithm 6 (pipelined: xi_i from
 *                          the initial residual, no update) of Section 3.3;
 *   - oracle_solve_mixed : classical iterative refinement (residual and
 *                          update in FP64) whose correction equation is
 *                          solved by Algorithm 2 + Eq. (3) in FP32 storage
 *                          and arithmetic, an extension of the paper's
 *                          pipelined CG (Section 3.1 cites mixed-precision
 *                          pipelined CG as prior work); its inner products
 *                          are either exact sums of the FP32 operands or
 *                          accumulated in FP32 (oracle_dot_f32acc).
 *
 * Build with -ffp-contract=off: every product and every sum is rounded on its
 * own; the only fused multiply-add is the explicit fma() that extracts the
 * exact rounding error of a product inside the compensated dot.
 *
 * Readings where the paper is silent or its listing is garbled:
 *   - alpha in Algorithm 2 is <r_i,r_i>/<p_i,Ap_i> (as in Algorithm 1);
 *   - the search-direction update of Algorithms 3 and 4 is
 *     p_{i+1} = r_{i+1} + beta_i (p_i - omega_i A p_i);
 *   - beta in Algorithm 4 is -<As_i,r0*>/<Ap_i,r0*>;
 *   - r0* = r0 = b - A x0;
 *   - convergence: ||r_k|| <= rtol ||b|| on the recursively updated residual;
 *     pipelined BiCGStab decides on the expanded norm, clamped at 0;
 *   - BiCGStab stops after the half step when ||s_i|| <= rtol ||b||
 *     (x_{i+1} = x_i + alpha_i p_i), which also avoids omega = 0/0;
 *   - k counts solution updates; b = 0 returns x = 0, k = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_CONVERGED = 0, OR_NOT_CONVERGED = 1, OR_BREAKDOWN = 2, OR_BAD_ARG = 3 };
enum { OR_CG_CLASSICAL = 0, OR_CG_PIPELINED = 1, OR_BICGSTAB_CLASSICAL = 2, OR_BICGSTAB_PIPELINED = 3,
       OR_GMRES_CLASSICAL = 4, OR_GMRES_PIPELINED = 5 };

/* Per-iteration trace record: TRACE_STRIDE doubles per iteration. */
#define TRACE_STRIDE 12

/* Summation mode of oracle_dot; 0 (compensated) is the oracle.  Modes 1 and 2
 * exist only to measure how sensitive a trajectory is to summation order. */
static int g_dot_mode = 0;

void oracle_set_dot_mode(int mode) { g_dot_mode = mode; }
int oracle_get_dot_mode(void) { return g_dot_mode; }

/* ---------------------------------------------------------------- products */

/* q_i = sum_j vals[j] * p[col[j]] for j = row_ptr[i] .. row_ptr[i+1]-1, summed
 * left to right starting from 0 (Section 2.2, CSR sparse matrix-vector
 * product). */
void oracle_spmv(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                 const double *vals, const double *p, double *q)
{
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j)
            acc = acc + vals[j] * p[col_idx[j]];
        q[i] = acc;
    }
}

/* Error-free transformations (Knuth's TwoSum; TwoProduct through fma). */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

static double dot_compensated(int64_t n, const double *a, const double *b)
{
    if (n == 0)
        return 0.0;
    double p, s;
    two_prod(a[0], b[0], &p, &s);
    for (int64_t i = 1; i < n; ++i) {
        double h, r, q;
        two_prod(a[i], b[i], &h, &r);
        two_sum(p, h, &p, &q);
        s = s + (q + r);
    }
    return p + s;
}

static double dot_sequential(int64_t n, const double *a, const double *b)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i)
        acc = acc + a[i] * b[i];
    return acc;
}

static double dot_pairwise(int64_t n, const double *a, const double *b)
{
    if (n <= 8)
        return dot_sequential(n, a, b);
    int64_t h = n / 2;
    return dot_pairwise(h, a, b) + dot_pairwise(n - h, a + h, b + h);
}

double oracle_dot(int64_t n, const double *a, const double *b)
{
    switch (g_dot_mode) {
    case 1: return dot_sequential(n, a, b);
    case 2: return dot_pairwise(n, a, b);
    default: return dot_compensated(n, a, b);
    }
}

/* ------------------------------------------------------------ small helpers */

typedef struct {
    int64_t n;
    const int32_t *rp;
    const int32_t *ci;
    const double *v;
} csr_t;

static void matvec(const csr_t *A, const double *p, double *q)
{
    oracle_spmv(A->n, A->rp, A->ci, A->v, p, q);
}

static int finite(double a) { return isfinite(a) ? 1 : 0; }

static double *vec(int64_t n)
{
    return (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
}

static void put_trace(double *trace, int32_t cap, int32_t it, int slot, double value)
{
    if (trace && it < cap)
        trace[(int64_t)it * TRACE_STRIDE + slot] = value;
}

static void put_hist(double *hist, int32_t cap, int32_t it, double value)
{
    if (hist && it < cap)
        hist[it] = value;
}

/* r = b - A x; returns 0 on allocation failure. */
static int initial_residual(const csr_t *A, const double *b, const double *x, double *r)
{
    double *ax = vec(A->n);
    if (!ax)
        return 0;
    matvec(A, x, ax);
    for (int64_t i = 0; i < A->n; ++i)
        r[i] = b[i] - ax[i];
    free(ax);
    return 1;
}

/* ---------------------------------------------------- Algorithm 1: CG */

static int cg_classical(const csr_t *A, const double *b, double *x, double *r,
                        double rtol, int32_t max_iter, double *hist, double *trace,
                        int32_t cap, int32_t *k_out)
{
    int64_t n = A->n;
    double *p = vec(n), *q = vec(n);
    int status = OR_NOT_CONVERGED;
    int32_t k = 0;
    if (!p || !q) { status = OR_BAD_ARG; goto done; }

    double bnorm = sqrt(oracle_dot(n, b, b));
    double tol = rtol * bnorm;
    if (!initial_residual(A, b, x, r)) { status = OR_BAD_ARG; goto done; }
    memcpy(p, r, (size_t)n * sizeof(double));            /* p_0 = r_0 */
    double rr = oracle_dot(n, r, r);
    put_hist(hist, cap, 0, sqrt(rr) / bnorm);
    if (!finite(rr)) { status = OR_BREAKDOWN; goto done; }
    if (sqrt(rr) <= tol) { status = OR_CONVERGED; goto done; }

    for (int32_t i = 0; i < max_iter; ++i) {
        matvec(A, p, q);                                   /* A p_i */
        double pq = oracle_dot(n, p, q);                   /* <p_i, A p_i> */
        if (!(pq > 0.0) || !finite(pq)) { status = OR_BREAKDOWN; break; }
        double alpha = rr / pq;
        for (int64_t j = 0; j < n; ++j) x[j] = x[j] + alpha * p[j];
        for (int64_t j = 0; j < n; ++j) r[j] = r[j] - alpha * q[j];
        double rr_new = oracle_dot(n, r, r);               /* <r_{i+1}, r_{i+1}> */
        k = i + 1;
        put_hist(hist, cap, k, sqrt(rr_new) / bnorm);
        put_trace(trace, cap, i, 0, alpha);
        put_trace(trace, cap, i, 2, rr);
        put_trace(trace, cap, i, 3, pq);
        put_trace(trace, cap, i, 5, rr_new);
        if (!finite(rr_new)) { status = OR_BREAKDOWN; break; }
        if (sqrt(rr_new) <= tol) { status = OR_CONVERGED; break; }
        double beta = rr_new / rr;
        put_trace(trace, cap, i, 1, beta);
        for (int64_t j = 0; j < n; ++j) p[j] = r[j] + beta * p[j];
        rr = rr_new;
    }
done:
    free(p); free(q);
    *k_out = k;
    return status;
}

/* ------------------------------------------ Algorithm 2: pipelined CG */

static int cg_pipelined(const csr_t *A, const double *b, double *x, double *r,
                        double rtol, int32_t max_iter, double *hist, double *trace,
                        int32_t cap, int32_t *k_out)
{
    int64_t n = A->n;
    double *p = vec(n), *ap = vec(n);
    int status = OR_NOT_CONVERGED;
    int32_t k = 0;
    if (!p || !ap) { status = OR_BAD_ARG; goto done; }

    double bnorm = sqrt(oracle_dot(n, b, b));
    double tol = rtol * bnorm;
    if (!initial_residual(A, b, x, r)) { status = OR_BAD_ARG; goto done; }
    memcpy(p, r, (size_t)n * sizeof(double));            /* p_0 = r_0 */
    double rr = oracle_dot(n, r, r);                       /* <r_0, r_0> */
    put_hist(hist, cap, 0, sqrt(rr) / bnorm);
    if (!finite(rr)) { status = OR_BREAKDOWN; goto done; }
    if (sqrt(rr) <= tol) { status = OR_CONVERGED; goto done; }

    matvec(A, p, ap);                                      /* A p_0 */
    double pap = oracle_dot(n, p, ap);
    double apap = oracle_dot(n, ap, ap);
    if (!(pap > 0.0) || !finite(pap) || !finite(apap)) { status = OR_BREAKDOWN; goto done; }
    double alpha = rr / pap;
    double beta = alpha * alpha * apap / rr - 1.0;         /* Eq. (3) */

    for (int32_t i = 1; i <= max_iter; ++i) {
        put_trace(trace, cap, i - 1, 0, alpha);
        put_trace(trace, cap, i - 1, 1, beta);
        put_trace(trace, cap, i - 1, 2, rr);
        put_trace(trace, cap, i - 1, 3, pap);
        put_trace(trace, cap, i - 1, 4, apap);
        for (int64_t j = 0; j < n; ++j) x[j] = x[j] + alpha * p[j];   /* x_i */
        for (int64_t j = 0; j < n; ++j) r[j] = r[j] - alpha * ap[j];  /* r_i */
        for (int64_t j = 0; j < n; ++j) p[j] = r[j] + beta * p[j];    /* p_i */
        rr = oracle_dot(n, r, r);                                      /* <r_i, r_i> */
        k = i;
        put_hist(hist, cap, k, sqrt(rr) / bnorm);
        put_trace(trace, cap, i - 1, 5, rr);
        if (!finite(rr)) { status = OR_BREAKDOWN; break; }
        if (sqrt(rr) <= tol) { status = OR_CONVERGED; break; }
        if (i == max_iter) break;
        matvec(A, p, ap);                                              /* A p_i */
        pap = oracle_dot(n, p, ap);                                    /* <p_i, A p_i> */
        apap = oracle_dot(n, ap, ap);                                  /* <A p_i, A p_i> */
        if (!(pap > 0.0) || !finite(pap) || !finite(apap)) { status = OR_BREAKDOWN; break; }
        alpha = rr / pap;
        beta = alpha * alpha * apap / rr - 1.0;                        /* Eq. (3) */
    }
done:
    free(p); free(ap);
    *k_out = k;
    return status;
}

/* -------------------------------------------- Algorithm 3: BiCGStab */

static int bicgstab_classical(const csr_t *A, const double *b, double *x, double *r,
                              double rtol, int32_t max_iter, double *hist, double *trace,
                              int32_t cap, int32_t *k_out)
{
    int64_t n = A->n;
    double *rs = vec(n), *p = vec(n), *v = vec(n), *s = vec(n), *t = vec(n);
    int status = OR_NOT_CONVERGED;
    int32_t k = 0;
    if (!rs || !p || !v || !s || !t) { status = OR_BAD_ARG; goto done; }

    double bnorm = sqrt(oracle_dot(n, b, b));
    double tol = rtol * bnorm;
    if (!initial_residual(A, b, x, r)) { status = OR_BAD_ARG; goto done; }
    memcpy(rs, r, (size_t)n * sizeof(double));           /* r0* = r0 */
    memcpy(p, r, (size_t)n * sizeof(double));            /* p0 = r0 */
    double rr0 = oracle_dot(n, r, r);
    put_hist(hist, cap, 0, sqrt(rr0) / bnorm);
    if (!finite(rr0)) { status = OR_BREAKDOWN; goto done; }
    if (sqrt(rr0) <= tol) { status = OR_CONVERGED; goto done; }
    double rho = oracle_dot(n, r, rs);                     /* <r_0, r0*> */

    for (int32_t i = 0; i < max_iter; ++i) {
        matvec(A, p, v);                                   /* A p_i */
        double vr = oracle_dot(n, v, rs);                  /* <A p_i, r0*> */
        if (vr == 0.0 || !finite(vr) || rho == 0.0 || !finite(rho)) { status = OR_BREAKDOWN; break; }
        double alpha = rho / vr;
        for (int64_t j = 0; j < n; ++j) s[j] = r[j] - alpha * v[j];   /* s_i */
        double ss = oracle_dot(n, s, s);
        put_trace(trace, cap, i, 0, alpha);
        put_trace(trace, cap, i, 3, rho);
        put_trace(trace, cap, i, 4, vr);
        put_trace(trace, cap, i, 5, ss);
        if (sqrt(ss) <= tol) {                             /* half-step exit */
            for (int64_t j = 0; j < n; ++j) x[j] = x[j] + alpha * p[j];
            memcpy(r, s, (size_t)n * sizeof(double));
            k = i + 1;
            put_hist(hist, cap, k, sqrt(ss) / bnorm);
            status = OR_CONVERGED;
            break;
        }
        matvec(A, s, t);                                   /* A s_i */
        double ts = oracle_dot(n, t, s);                   /* <A s_i, s_i> */
        double tt = oracle_dot(n, t, t);                   /* <A s_i, A s_i> */
        if (tt == 0.0 || !finite(tt) || !finite(ts)) { status = OR_BREAKDOWN; break; }
        double omega = ts / tt;
        for (int64_t j = 0; j < n; ++j) x[j] = x[j] + alpha * p[j] + omega * s[j];
        for (int64_t j = 0; j < n; ++j) r[j] = s[j] - omega * t[j];
        double rr = oracle_dot(n, r, r);
        k = i + 1;
        put_hist(hist, cap, k, sqrt(rr) / bnorm);
        put_trace(trace, cap, i, 2, omega);
        put_trace(trace, cap, i, 6, ts);
        put_trace(trace, cap, i, 7, tt);
        put_trace(trace, cap, i, 10, rr);
        if (!finite(rr)) { status = OR_BREAKDOWN; break; }
        if (sqrt(rr) <= tol) { status = OR_CONVERGED; break; }
        double rho_new = oracle_dot(n, r, rs);             /* <r_{i+1}, r0*> */
        if (omega == 0.0 || rho_new == 0.0 || !finite(rho_new)) { status = OR_BREAKDOWN; break; }
        double beta = (rho_new / rho) * (alpha / omega);
        put_trace(trace, cap, i, 1, beta);
        for (int64_t j = 0; j < n; ++j) p[j] = r[j] + beta * (p[j] - omega * v[j]);
        rho = rho_new;
    }
done:
    free(rs); free(p); free(v); free(s); free(t);
    *k_out = k;
    return status;
}

/* ----------------------------------- Algorithm 4: pipelined BiCGStab */

static int bicgstab_pipelined(const csr_t *A, const double *b, double *x, double *r,
                              double rtol, int32_t max_iter, double *hist, double *trace,
                              int32_t cap, int32_t *k_out)
{
    int64_t n = A->n;
    double *rs = vec(n), *p = vec(n), *ap = vec(n), *s = vec(n), *as = vec(n);
    int status = OR_NOT_CONVERGED;
    int32_t k = 0;
    if (!rs || !p || !ap || !s || !as) { status = OR_BAD_ARG; goto done; }

    double bnorm = sqrt(oracle_dot(n, b, b));
    double tol = rtol * bnorm;
    if (!initial_residual(A, b, x, r)) { status = OR_BAD_ARG; goto done; }
    memcpy(rs, r, (size_t)n * sizeof(double));           /* r0* = r0 */
    memcpy(p, r, (size_t)n * sizeof(double));            /* p0 = r0 */
    double rr0 = oracle_dot(n, r, r);
    put_hist(hist, cap, 0, sqrt(rr0) / bnorm);
    if (!finite(rr0)) { status = OR_BREAKDOWN; goto done; }
    if (sqrt(rr0) <= tol) { status = OR_CONVERGED; goto done; }
    double rho = oracle_dot(n, r, rs);                     /* <r_0, r0*> */

    for (int32_t i = 0; i < max_iter; ++i) {
        matvec(A, p, ap);                                  /* A p_i */
        double apr = oracle_dot(n, ap, rs);                /* <A p_i, r0*> */
        if (apr == 0.0 || !finite(apr) || rho == 0.0 || !finite(rho)) { status = OR_BREAKDOWN; break; }
        double alpha = rho / apr;
        for (int64_t j = 0; j < n; ++j) s[j] = r[j] - alpha * ap[j];  /* s_i */
        double ss = oracle_dot(n, s, s);                   /* <s_i, s_i> */
        put_trace(trace, cap, i, 0, alpha);
        put_trace(trace, cap, i, 3, rho);
        put_trace(trace, cap, i, 4, apr);
        put_trace(trace, cap, i, 5, ss);
        if (sqrt(ss) <= tol) {                             /* half-step exit */
            for (int64_t j = 0; j < n; ++j) x[j] = x[j] + alpha * p[j];
            memcpy(r, s, (size_t)n * sizeof(double));
            k = i + 1;
            put_hist(hist, cap, k, sqrt(ss) / bnorm);
            status = OR_CONVERGED;
            break;
        }
        matvec(A, s, as);                                  /* A s_i */
        double ass = oracle_dot(n, as, s);                 /* <A s_i, s_i> */
        double asas = oracle_dot(n, as, as);               /* <A s_i, A s_i> */
        double asr = oracle_dot(n, as, rs);                /* <A s_i, r0*> */
        if (asas == 0.0 || !finite(asas) || !finite(ass) || !finite(asr)) { status = OR_BREAKDOWN; break; }
        double beta = -asr / apr;                          /* beta via <s_i, r0*> = 0 */
        double omega = ass / asas;
        /* <r_{i+1}, r_{i+1}> expanded in <s,s>, <s,As>, <As,As> */
        double rr_next = ss - 2.0 * omega * ass + omega * omega * asas;
        for (int64_t j = 0; j < n; ++j) x[j] = x[j] + alpha * p[j] + omega * s[j];
        for (int64_t j = 0; j < n; ++j) r[j] = s[j] - omega * as[j];
        for (int64_t j = 0; j < n; ++j) p[j] = r[j] + beta * (p[j] - omega * ap[j]);
        rho = oracle_dot(n, r, rs);                        /* <r_{i+1}, r0*> */
        double rnorm = sqrt(rr_next > 0.0 ? rr_next : 0.0);
        k = i + 1;
        put_hist(hist, cap, k, rnorm / bnorm);
        put_trace(trace, cap, i, 1, beta);
        put_trace(trace, cap, i, 2, omega);
        put_trace(trace, cap, i, 6, ass);
        put_trace(trace, cap, i, 7, asas);
        put_trace(trace, cap, i, 8, asr);
        put_trace(trace, cap, i, 9, rr_next);
        if (trace && i < cap)
            put_trace(trace, cap, i, 10, oracle_dot(n, r, r));   /* diagnostic only */
        if (!finite(rr_next)) { status = OR_BREAKDOWN; break; }
        if (rnorm <= tol) { status = OR_CONVERGED; break; }
        if (omega == 0.0) { status = OR_BREAKDOWN; break; }
    }
done:
    free(rs); free(p); free(ap); free(s); free(as);
    *k_out = k;
    return status;
}


/* ------------------------------------------- Algorithms 5 and 6: GMRES(m) */

/*
 * Restarted simpler GMRES(m) (Walker and Zhou) with classical Gram-Schmidt.
 * A cycle starts from r0 = b - A x (its true norm rho0 is the history entry
 * at the restart and decides convergence), v_0 = r0/rho0, and for
 * i = 1..m: w = A v_{i-1}; R[j][i] = <v_j, w> for j = 1..i-1, all from the
 * same w; w = w - sum_j R[j][i] v_j (j in order); R[i][i] = ||w||;
 * v_i = w / R[i][i]; xi_i = <r, v_i> with r = v_0 (pipelined) or the
 * residual updated as r = r - xi_i v_i (classical).  The estimate
 * rho0 * zeta_i, zeta_i^2 = max(zeta_{i-1}^2 - xi_i^2, 0), zeta_0 = 1, is the
 * history entry of iteration i and ends the cycle early when it meets the
 * tolerance.  Then R eta = xi is solved by back substitution and
 * x = x + rho0 (eta_1 v_0 + sum_{j=2}^{i} eta_j v_{j-1}).  R[i][i] = 0 or
 * not finite ends the cycle before step i (breakdown if that leaves no
 * step).  k counts products A v over all cycles.
 */
static int gmres(const csr_t *A, const double *b, double *x, double *r, int pipelined, int32_t m,
                 double rtol, int32_t max_iter, double *hist, int32_t cap, int32_t *k_out)
{
    int64_t n = A->n;
    int status = OR_NOT_CONVERGED;
    int32_t k = 0;
    double *V = (double *)calloc((size_t)(m + 1) * (size_t)n, sizeof(double));
    double *w = vec(n), *rr = vec(n);
    double *R = (double *)calloc((size_t)(m + 1) * (size_t)(m + 1), sizeof(double));
    double *xi = (double *)calloc((size_t)(m + 1), sizeof(double));
    double *eta = (double *)calloc((size_t)(m + 1), sizeof(double));
    if (!V || !w || !rr || !R || !xi || !eta) { status = OR_BAD_ARG; goto done; }
    double bnorm = sqrt(oracle_dot(n, b, b));
    double tol = rtol * bnorm;
    for (;;) {
        if (!initial_residual(A, b, x, r)) { status = OR_BAD_ARG; break; }
        double rho0 = sqrt(oracle_dot(n, r, r));
        put_hist(hist, cap, k, rho0 / bnorm);
        if (!finite(rho0)) { status = OR_BREAKDOWN; break; }
        if (rho0 <= tol) { status = OR_CONVERGED; break; }
        if (k >= max_iter) { status = OR_NOT_CONVERGED; break; }
        double *v0 = V;
        for (int64_t t = 0; t < n; ++t) { v0[t] = r[t] / rho0; rr[t] = v0[t]; }
        double zeta2 = 1.0;
        int32_t used = 0;
        for (int32_t i = 1; i <= m && k < max_iter; ++i) {
            double *vi = V + (size_t)i * n;
            matvec(A, V + (size_t)(i - 1) * n, w);                          /* w = A v_{i-1} */
            for (int32_t j = 1; j < i; ++j)
                R[j * (m + 1) + i] = oracle_dot(n, V + (size_t)j * n, w);    /* R_{j,i} */
            for (int32_t j = 1; j < i; ++j) {
                const double rj = R[j * (m + 1) + i];
                const double *vj = V + (size_t)j * n;
                for (int64_t t = 0; t < n; ++t) w[t] = w[t] - rj * vj[t];
            }
            const double rii = sqrt(oracle_dot(n, w, w));
            if (!(rii > 0.0) || !finite(rii)) break;                        /* no step i */
            R[i * (m + 1) + i] = rii;
            for (int64_t t = 0; t < n; ++t) vi[t] = w[t] / rii;
            xi[i] = oracle_dot(n, rr, vi);
            if (!pipelined)
                for (int64_t t = 0; t < n; ++t) rr[t] = rr[t] - xi[i] * vi[t];
            zeta2 = zeta2 - xi[i] * xi[i];
            if (zeta2 < 0.0) zeta2 = 0.0;
            ++k;
            used = i;
            put_hist(hist, cap, k, rho0 * sqrt(zeta2) / bnorm);
            if (rho0 * sqrt(zeta2) <= tol) break;
        }
        if (used == 0) { status = OR_BREAKDOWN; break; }
        for (int32_t i = used; i >= 1; --i) {                               /* R eta = xi */
            double s = xi[i];
            for (int32_t j = i + 1; j <= used; ++j) s = s - R[i * (m + 1) + j] * eta[j];
            eta[i] = s / R[i * (m + 1) + i];
        }
        for (int64_t t = 0; t < n; ++t) {
            double s = eta[1] * V[t];
            for (int32_t j = 2; j <= used; ++j) s = s + eta[j] * V[(size_t)(j - 1) * n + t];
            x[t] = x[t] + rho0 * s;
        }
    }
done:
    free(V); free(w); free(rr); free(R); free(xi); free(eta);
    *k_out = k;
    return status;
}

int oracle_solve_gmres(int pipelined, int32_t m, int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                       const double *vals, const double *b, double *x, double *r, double rtol,
                       int32_t max_iter, double *hist, int32_t cap, int32_t *k_out)
{
    *k_out = 0;
    if (n <= 0 || m < 1 || !row_ptr || !col_idx || !vals || !b || !x || max_iter < 0 || !(rtol >= 0.0))
        return OR_BAD_ARG;
    csr_t A = {n, row_ptr, col_idx, vals};
    double *rbuf = r ? r : vec(n);
    if (!rbuf)
        return OR_BAD_ARG;
    int status;
    if (oracle_dot(n, b, b) == 0.0) {                                        /* b = 0: x = 0 */
        for (int64_t j = 0; j < n; ++j) { x[j] = 0.0; rbuf[j] = 0.0; }
        put_hist(hist, cap, 0, 0.0);
        status = OR_CONVERGED;
    } else {
        status = gmres(&A, b, x, rbuf, pipelined, m, rtol, max_iter, hist, cap, k_out);
    }
    if (!r)
        free(rbuf);
    return status;
}

/* --------------------------------------------------------------- entry */

/*
 * Solve A x = b.  x holds x0 on entry and the last iterate on return; r (may
 * be NULL) receives the recursively updated residual.  hist (may be NULL)
 * receives ||r_i||/||b|| for i = 0..k; trace (may be NULL) receives
 * TRACE_STRIDE scalars per iteration; cap bounds both.  Returns OR_*.
 */
int oracle_solve(int method, int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                 const double *vals, const double *b, double *x, double *r,
                 double rtol, int32_t max_iter, double *hist, double *trace,
                 int32_t cap, int32_t *k_out)
{
    *k_out = 0;
    if (n <= 0 || !row_ptr || !col_idx || !vals || !b || !x || max_iter < 0 || !(rtol >= 0.0))
        return OR_BAD_ARG;
    csr_t A = {n, row_ptr, col_idx, vals};
    double *rbuf = r ? r : vec(n);
    if (!rbuf)
        return OR_BAD_ARG;

    double bb = oracle_dot(n, b, b);
    int status;
    if (bb == 0.0) {                                       /* b = 0: x = 0 */
        for (int64_t j = 0; j < n; ++j) { x[j] = 0.0; rbuf[j] = 0.0; }
        put_hist(hist, cap, 0, 0.0);
        status = OR_CONVERGED;
    } else {
        switch (method) {
        case OR_CG_CLASSICAL:
            status = cg_classical(&A, b, x, rbuf, rtol, max_iter, hist, trace, cap, k_out); break;
        case OR_CG_PIPELINED:
            status = cg_pipelined(&A, b, x, rbuf, rtol, max_iter, hist, trace, cap, k_out); break;
        case OR_BICGSTAB_CLASSICAL:
            status = bicgstab_classical(&A, b, x, rbuf, rtol, max_iter, hist, trace, cap, k_out); break;
        case OR_BICGSTAB_PIPELINED:
            status = bicgstab_pipelined(&A, b, x, rbuf, rtol, max_iter, hist, trace, cap, k_out); break;
        default:
            status = OR_BAD_ARG;
        }
    }
    if (!r)
        free(rbuf);
    return status;
}

int oracle_trace_stride(void) { return TRACE_STRIDE; }

/* ------------------------------- iterative refinement, FP32 inner solver */

/* The product of two floats is exact in double, so the compensated dot of
 * the widened operands is the FP32 dot "as if in twice the precision" of
 * the FP64 oracle_dot. */
double oracle_dot_f32(int64_t n, const float *a, const float *b)
{
    if (n == 0)
        return 0.0;
    double p = (double)a[0] * (double)b[0], s = 0.0;
    for (int64_t i = 1; i < n; ++i) {
        double h = (double)a[i] * (double)b[i], q;
        two_sum(p, h, &p, &q);
        s = s + q;
    }
    return p + s;
}

/* <a, b> accumulated in FP32: each product a_i b_i rounded to FP32, then
 * added to an FP32 running sum, left to right (recursive summation in single
 * precision; its error is at most gamma_n sum |a_i b_i|, gamma_n =
 * n u / (1 - n u), u = 2^-24). */
float oracle_dot_f32acc(int64_t n, const float *a, const float *b)
{
    float acc = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        const float prod = a[i] * b[i];
        acc = acc + prod;
    }
    return acc;
}

/* q = A p in FP32: every product and every partial row sum rounded to FP32,
 * rows summed left to right in CSR order. */
void oracle_spmv_f32(int64_t n, const int32_t *rp, const int32_t *ci, const float *v,
                     const float *p, float *q)
{
    for (int64_t i = 0; i < n; ++i) {
        float acc = 0.0f;
        for (int64_t j = rp[i]; j < rp[i + 1]; ++j)
            acc = acc + v[j] * p[ci[j]];
        q[i] = acc;
    }
}

/* Algorithm 2 with Eq. (3) for A d = r with d_0 = 0, in FP32: alpha, beta
 * are formed in FP64 from the dots and rounded to FP32 for the updates.
 * Stops when ||r_i|| <= rtol ||r_0|| (recursive residual) or after cap
 * iterations.  r is overwritten by the inner residual.  Returns OR_*. */
static int cg_pipelined_f32(int64_t n, const int32_t *rp, const int32_t *ci, const float *v,
                            float *r, float *d, float *p, float *ap, double rtol, int64_t cap,
                            int64_t *k_out)
{
    int64_t k = 0;
    for (int64_t j = 0; j < n; ++j) { d[j] = 0.0f; p[j] = r[j]; }
    double rr = oracle_dot_f32(n, r, r);
    *k_out = 0;
    if (rr == 0.0) return OR_CONVERGED;                     /* r = 0: d = 0, no step */
    double tol = rtol * sqrt(rr);
    if (!finite(rr)) return OR_BREAKDOWN;
    if (sqrt(rr) <= tol) return OR_CONVERGED;
    oracle_spmv_f32(n, rp, ci, v, p, ap);
    double pap = oracle_dot_f32(n, p, ap), apap = oracle_dot_f32(n, ap, ap);
    if (!(pap > 0.0) || !finite(pap) || !finite(apap)) return OR_BREAKDOWN;
    double alpha = rr / pap;
    double beta = alpha * alpha * apap / rr - 1.0;         /* Eq. (3) */
    int status = OR_NOT_CONVERGED;
    for (int64_t i = 1; i <= cap; ++i) {
        const float af = (float)alpha, bf = (float)beta;
        for (int64_t j = 0; j < n; ++j) d[j] = d[j] + af * p[j];
        for (int64_t j = 0; j < n; ++j) r[j] = r[j] - af * ap[j];
        for (int64_t j = 0; j < n; ++j) p[j] = r[j] + bf * p[j];
        rr = oracle_dot_f32(n, r, r);
        k = i;
        if (!finite(rr)) { status = OR_BREAKDOWN; break; }
        if (sqrt(rr) <= tol) { status = OR_CONVERGED; break; }
        if (i == cap) break;
        oracle_spmv_f32(n, rp, ci, v, p, ap);
        pap = oracle_dot_f32(n, p, ap);
        apap = oracle_dot_f32(n, ap, ap);
        if (!(pap > 0.0) || !finite(pap) || !finite(apap)) { status = OR_BREAKDOWN; break; }
        alpha = rr / pap;
        beta = alpha * alpha * apap / rr - 1.0;
    }
    *k_out = k;
    return status;
}

/* The same iteration (Algorithm 2 with Eq. (3), d_0 = 0) entirely in FP32:
 * FP32 vectors, FP32 products, inner products accumulated in FP32
 * (oracle_dot_f32acc) and the scalars alpha, beta, the tolerance and the
 * test formed in FP32.  Stops when ||r_i|| <= rtol ||r_0|| or after cap
 * iterations; r is overwritten by the inner residual.  Returns OR_*. */
static int cg_pipelined_f32acc(int64_t n, const int32_t *rp, const int32_t *ci, const float *v,
                               float *r, float *d, float *p, float *ap, double rtol, int64_t cap,
                               int64_t *k_out)
{
    int64_t k = 0;
    for (int64_t j = 0; j < n; ++j) { d[j] = 0.0f; p[j] = r[j]; }
    float rr = oracle_dot_f32acc(n, r, r);
    *k_out = 0;
    if (rr == 0.0f) return OR_CONVERGED;                    /* r = 0: d = 0, no step */
    if (!isfinite(rr)) return OR_BREAKDOWN;
    const float tol = (float)rtol * sqrtf(rr);
    if (sqrtf(rr) <= tol) return OR_CONVERGED;
    oracle_spmv_f32(n, rp, ci, v, p, ap);
    float pap = oracle_dot_f32acc(n, p, ap), apap = oracle_dot_f32acc(n, ap, ap);
    if (!(pap > 0.0f) || !isfinite(pap) || !isfinite(apap)) return OR_BREAKDOWN;
    float alpha = rr / pap;
    float beta = alpha * alpha * apap / rr - 1.0f;          /* Eq. (3) */
    int status = OR_NOT_CONVERGED;
    for (int64_t i = 1; i <= cap; ++i) {
        for (int64_t j = 0; j < n; ++j) d[j] = d[j] + alpha * p[j];
        for (int64_t j = 0; j < n; ++j) r[j] = r[j] - alpha * ap[j];
        for (int64_t j = 0; j < n; ++j) p[j] = r[j] + beta * p[j];
        rr = oracle_dot_f32acc(n, r, r);
        k = i;
        if (!isfinite(rr)) { status = OR_BREAKDOWN; break; }
        if (sqrtf(rr) <= tol) { status = OR_CONVERGED; break; }
        if (i == cap) break;
        oracle_spmv_f32(n, rp, ci, v, p, ap);
        pap = oracle_dot_f32acc(n, p, ap);
        apap = oracle_dot_f32acc(n, ap, ap);
        if (!(pap > 0.0f) || !isfinite(pap) || !isfinite(apap)) { status = OR_BREAKDOWN; break; }
        alpha = rr / pap;
        beta = alpha * alpha * apap / rr - 1.0f;
    }
    *k_out = k;
    return status;
}

/*
 * Iterative refinement: for j = 0, 1, ...: r_j = b - A x_j in FP64; stop when
 * ||r_j|| <= rtol ||b||; solve A d = (float) r_j with the FP32 pipelined CG
 * above (matrix values rounded to FP32) to inner_rtol; x_{j+1} = x_j + d.
 * Limits: max_iter inner iterations in total, max_outer sweeps; a sweep
 * whose inner solve makes no iteration ends the solve (not converged).
 * hist[j] = ||r_j||/||b|| (j = 0..sweeps, up to cap); inner_k[j] (may be
 * NULL) = inner iterations of sweep j.  *k_out = inner iterations in total.
 * acc selects the inner solver: 0 = cg_pipelined_f32 (inner products exact
 * sums of the FP32 operands, scalars in FP64), 1 = cg_pipelined_f32acc
 * (inner products accumulated in FP32, scalars in FP32).
 * Returns OR_*; b = 0 gives x = 0.
 */
int oracle_solve_mixed(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                       const double *vals, const double *b, double *x, double rtol,
                       double inner_rtol, int32_t max_iter, int32_t max_outer, double *hist,
                       int32_t *inner_k, int32_t cap, int32_t *k_out, int32_t *sweeps_out,
                       int32_t acc)
{
    *k_out = 0;
    *sweeps_out = 0;
    if (n <= 0 || !row_ptr || !col_idx || !vals || !b || !x || max_iter < 0 || max_outer < 0 ||
        !(rtol >= 0.0) || !(inner_rtol >= 0.0) || acc < 0 || acc > 1)
        return OR_BAD_ARG;
    const int64_t nnz = row_ptr[n];
    csr_t A = {n, row_ptr, col_idx, vals};
    double *r = vec(n);
    float *v32 = (float *)calloc((size_t)(nnz > 0 ? nnz : 1), sizeof(float));
    float *r32 = (float *)calloc((size_t)n, sizeof(float));
    float *d = (float *)calloc((size_t)n, sizeof(float));
    float *p = (float *)calloc((size_t)n, sizeof(float));
    float *ap = (float *)calloc((size_t)n, sizeof(float));
    int status = OR_BAD_ARG;
    if (!r || !v32 || !r32 || !d || !p || !ap) goto done;
    for (int64_t j = 0; j < nnz; ++j) v32[j] = (float)vals[j];

    double bb = oracle_dot(n, b, b);
    if (bb == 0.0) {
        for (int64_t j = 0; j < n; ++j) x[j] = 0.0;
        put_hist(hist, cap, 0, 0.0);
        status = OR_CONVERGED;
        goto done;
    }
    double bnorm = sqrt(bb), tol = rtol * bnorm;
    int64_t used = 0;
    int32_t sweeps = 0;
    for (;;) {
        if (!initial_residual(&A, b, x, r)) { status = OR_BAD_ARG; break; }   /* r_j */
        double rr = oracle_dot(n, r, r);
        put_hist(hist, cap, sweeps, sqrt(rr) / bnorm);
        if (!finite(rr)) { status = OR_BREAKDOWN; break; }
        if (sqrt(rr) <= tol) { status = OR_CONVERGED; break; }
        if (sweeps >= max_outer || used >= max_iter) { status = OR_NOT_CONVERGED; break; }
        for (int64_t j = 0; j < n; ++j) r32[j] = (float)r[j];
        int64_t kj = 0;
        int st = acc == 0 ? cg_pipelined_f32(n, row_ptr, col_idx, v32, r32, d, p, ap, inner_rtol,
                                             (int64_t)max_iter - used, &kj)
                          : cg_pipelined_f32acc(n, row_ptr, col_idx, v32, r32, d, p, ap, inner_rtol,
                                                (int64_t)max_iter - used, &kj);
        used += kj;
        if (inner_k && sweeps < cap) inner_k[sweeps] = (int32_t)kj;
        if (st == OR_BREAKDOWN) { status = OR_BREAKDOWN; break; }
        if (kj == 0) { status = OR_NOT_CONVERGED; break; }
        for (int64_t j = 0; j < n; ++j) x[j] = x[j] + (double)d[j];       /* x_{j+1} */
        sweeps++;
    }
    *k_out = (int32_t)used;
    *sweeps_out = sweeps;
done:
    free(r); free(v32); free(r32); free(d); free(p); free(ap);
    return status;
}

/* ------------------------------------------------ timing build (OpenMP) */

#ifdef _OPENMP
#include <omp.h>

/*
 * Compiled only into the timing build (gcc -fopenmp); the parity build has
 * no OpenMP and none of this.  Algorithm 1 exactly as cg_classical, with the
 * rows of the product and of every vector update split over `threads`
 * threads in static contiguous chunks, and each inner product computed per
 * chunk by the compensated dot of oracle_dot, the chunk results added in
 * chunk order (TwoSum).  The result depends on the thread count, never on
 * scheduling.  For timing the oracle on the host's cores; no history.
 */
static void omp_chunk(int64_t n, int t, int T, int64_t *lo, int64_t *hi)
{
    *lo = n * t / T;
    *hi = n * (t + 1) / T;
}

static double omp_dot(int64_t n, const double *a, const double *b, double *part, int T)
{
#pragma omp parallel num_threads(T)
    {
        int64_t lo, hi;
        omp_chunk(n, omp_get_thread_num(), T, &lo, &hi);
        part[omp_get_thread_num()] = dot_compensated(hi - lo, a + lo, b + lo);
    }
    double s = part[0], c = 0.0;
    for (int t = 1; t < T; ++t) {
        double e;
        two_sum(s, part[t], &s, &e);
        c = c + e;
    }
    return s + c;
}

static void omp_matvec(const csr_t *A, const double *p, double *q, int T)
{
#pragma omp parallel num_threads(T)
    {
        int64_t lo, hi;
        omp_chunk(A->n, omp_get_thread_num(), T, &lo, &hi);
        for (int64_t i = lo; i < hi; ++i) {
            double acc = 0.0;
            for (int64_t j = A->rp[i]; j < A->rp[i + 1]; ++j)
                acc = acc + A->v[j] * p[A->ci[j]];
            q[i] = acc;
        }
    }
}

int oracle_cg_classical_omp(int32_t threads, int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                            const double *vals, const double *b, double *x, double rtol, int32_t max_iter,
                            int32_t *k_out)
{
    *k_out = 0;
    if (threads < 1 || n <= 0 || !row_ptr || !col_idx || !vals || !b || !x || max_iter < 0)
        return OR_BAD_ARG;
    const int T = threads;
    csr_t A = {n, row_ptr, col_idx, vals};
    double *r = vec(n), *p = vec(n), *q = vec(n), *part = vec(T);
    int status = OR_NOT_CONVERGED;
    int32_t k = 0;
    if (!r || !p || !q || !part) { status = OR_BAD_ARG; goto done; }

    double bnorm = sqrt(omp_dot(n, b, b, part, T));
    double tol = rtol * bnorm;
    omp_matvec(&A, x, q, T);
#pragma omp parallel for schedule(static) num_threads(T)
    for (int64_t j = 0; j < n; ++j) { r[j] = b[j] - q[j]; p[j] = r[j]; }
    double rr = omp_dot(n, r, r, part, T);
    if (!finite(rr)) { status = OR_BREAKDOWN; goto done; }
    if (sqrt(rr) <= tol) { status = OR_CONVERGED; goto done; }
    for (int32_t i = 0; i < max_iter; ++i) {
        omp_matvec(&A, p, q, T);                                /* A p_i */
        double pq = omp_dot(n, p, q, part, T);                  /* <p_i, A p_i> */
        if (!(pq > 0.0) || !finite(pq)) { status = OR_BREAKDOWN; break; }
        double alpha = rr / pq;
#pragma omp parallel for schedule(static) num_threads(T)
        for (int64_t j = 0; j < n; ++j) x[j] = x[j] + alpha * p[j];
#pragma omp parallel for schedule(static) num_threads(T)
        for (int64_t j = 0; j < n; ++j) r[j] = r[j] - alpha * q[j];
        double rr_new = omp_dot(n, r, r, part, T);              /* <r_{i+1}, r_{i+1}> */
        k = i + 1;
        if (!finite(rr_new)) { status = OR_BREAKDOWN; break; }
        if (sqrt(rr_new) <= tol) { status = OR_CONVERGED; break; }
        double beta = rr_new / rr;
#pragma omp parallel for schedule(static) num_threads(T)
        for (int64_t j = 0; j < n; ++j) p[j] = r[j] + beta * p[j];
        rr = rr_new;
    }
done:
    free(r); free(p); free(q); free(part);
    *k_out = k;
    return status;
}
#endif /* _OPENMP */
