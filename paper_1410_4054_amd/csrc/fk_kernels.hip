// HIP kernels for gfx950 (CDNA4, wave64) of the pipelined CG and BiCGStab
// iterations (Sections 2.2, 3.1 and 3.2 of arXiv:1410.4054).
//
// Structure shared by every kernel that ends in a reduction point:
//   1. the kernel returns at once unless the solver state is in its run mask
//      (the state is written only by the last workgroup of the previous
//      reduction point, so the test is uniform across the grid);
//   2. each thread accumulates its share of up to KMAX inner products as
//      error-free double-double sums (TwoProduct through fma, TwoSum);
//   3. the workgroup combines them with a wave64 DPP tree and LDS,
//      and wave 0 stores one double-double partial per inner product while
//      the other waves exit (the first reduction stage of Section 2.2);
//   4. the second stage runs in polling group leaders: a two-level tree
//      (see reduce_point) sums all partials in a fixed order, rounds once,
//      and the last workgroup evaluates the scalar recurrences (alpha,
//      beta, omega, convergence)
//      on the device.
// Partials are published with agent-scope (device-coherent) atomic stores
// and read back with agent-scope atomic loads, and the store counter is
// drained before arriving at a counter.  A release/acquire fence would do the
// same but, with one L2 per XCD, it writes back and invalidates the whole
// L2 of the issuing XCD; taken by thousands of workgroups per launch that
// cost more than the kernel's own memory traffic.  Counters are split into
// groups because same-address device atomics serialize: thousands of them
// arriving together at one counter would add tens of microseconds.
// No floating-point atomics are used: results do not depend on which
// workgroup finishes last and are bitwise reproducible.
//
// Files are built with -ffp-contract=off: products and sums are rounded one
// by one, exactly as written; fma appears only where the error of a product
// is extracted.
#include "fk_dd.hpp"
#include "fk_internal.hpp"

#include <hip/hip_ext.h>

// Minimum waves per SIMD the product kernels are compiled for (caps VGPRs).
#ifndef FK_SPMV_MIN_WAVES
#define FK_SPMV_MIN_WAVES 8
#endif
// Unroll factor of the grid-stride loops of the per-iteration vector-update
// kernels (measured: 4 beats 1 and 2 on MI355X).
#ifndef FK_VEC_UNROLL
#define FK_VEC_UNROLL 4
#endif
// Entries of a row requested together by the sliced-layout products.
#ifndef FK_SELL_UNROLL
#define FK_SELL_UNROLL 8
#endif

namespace fk {
namespace {

// Sum K double-double values over the workgroup; the result is valid in
// thread 0.  Ends with every thread past a barrier that follows the last
// LDS read, so `lds` may be reused right away.
template <int K, int NW = WAVES>
__device__ __forceinline__ void block_reduce(dd (&v)[K], dd (*lds)[KMAX])
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k)
        v[k] = wave_reduce(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            lds[wave][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            dd a = lds[0][k];
            for (int w = 1; w < NW; ++w)
                a = dd_add(a, lds[w][k]);
            v[k] = a;
        }
    }
    __syncthreads();
}

// Fixed-order workgroup sum of one plain double (long CSR rows).
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = v + __shfl_xor(v, off, 64);
    if (lane == 0)
        lds[wave] = v;
    __syncthreads();
    double s = lds[0];
    for (int w = 1; w < WAVES; ++w)
        s = s + lds[w];
    __syncthreads();
    return s;
}

// Device-coherent (agent-scope) store and load of one double.
__device__ __forceinline__ void store_coherent(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double load_coherent(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A load of the matrix stream.  NT: non-temporal (the products of a matrix
// whose data and vectors exceed the Infinity Cache read each entry once per
// launch from HBM; marking those loads non-temporal keeps them from evicting
// the vector lines that neighbouring slices gather again).  Below that size
// the cache holds the matrix from one product to the next, and ordinary
// loads keep it there.
template <bool NT = false, typename T>
__device__ __forceinline__ T load_stream(const T *p)
{
    if constexpr (NT) {
        if constexpr (sizeof(T) == 8 && !std::is_arithmetic_v<T>) {
            // packed 16-bit offsets: one 8-byte non-temporal load
            const uint64_t u = __builtin_nontemporal_load(reinterpret_cast<const uint64_t *>(p));
            return __builtin_bit_cast(T, u);
        } else {
            return __builtin_nontemporal_load(p);
        }
    } else {
        return *p;
    }
}

__device__ __forceinline__ bool runs(const RedArgs &red)
{
    return ((1u << red.st->status) & red.run_mask) != 0u;
}

// Workgroups are dispatched to the eight XCDs round robin.  Renumber them so
// that each XCD owns a contiguous range of logical workgroups, hence a
// contiguous slab of rows: the gathers of neighbouring rows then hit that
// XCD's own L2.
__device__ __forceinline__ int logical_wg()
{
    const int G = gridDim.x;
    const int b = blockIdx.x;
    if (G < 8 || (G & 7) != 0)
        return b;
    return (b & 7) * (G >> 3) + (b >> 3);
}

// ------------------------------------------------------------- finalize

__device__ __forceinline__ void put_hist(const DevState *st, double *hist, int it, double v)
{
    if (hist && it < st->hist_cap)
        hist[it] = v;
}

__device__ __forceinline__ void put_scal(const DevState *st, double *scal, int it, int slot, double v)
{
    if (scal && it < st->hist_cap)
        scal[4 * it + slot] = v;
}

// Scalar work of a reduction point (one thread).  The expressions and their
// order follow Algorithms 1-4 exactly; see the comments per case.
// Algorithm 2, alpha_i = <r_i,r_i> / <p_i,Ap_i> and beta_i by Eq. (3).
__device__ void cg_alpha(DevState *st, double pap, double apap, double *scal)
{
    if (!(pap > 0.0) || !isfinite(pap) || !isfinite(apap)) {
        st->status = ST_BREAKDOWN;
        return;
    }
    const double alpha = st->rr / pap;
    const double beta = alpha * alpha * apap / st->rr - 1.0;  // Eq. (3)
    st->alpha = alpha;
    st->beta = beta;
    put_scal(st, scal, st->it, 0, alpha);
    put_scal(st, scal, st->it, 1, beta);
    if (st->it >= st->max_iter)
        st->status = ST_NOT_CONVERGED;
}

// Algorithm 2, <r_i, r_i>: iteration i done, residual history, convergence.
__device__ void cg_rr(DevState *st, double rr, double *hist, double *scal)
{
    const int it = st->it + 1;
    st->it = it;
    st->rr = rr;
    const double rel = sqrt(rr) / st->bnorm;
    st->last_rel = rel;
    put_hist(st, hist, it, rel);
    put_scal(st, scal, it - 1, 3, rr);
    if (!isfinite(rr))
        st->status = ST_BREAKDOWN;
    else if (sqrt(rr) <= st->tol)
        st->status = ST_CONVERGED;
    else if (it >= st->max_iter)
        st->status = ST_NOT_CONVERGED;
}

// Algorithm 2 in FP32 (the FP32-accumulating inner solver): the same steps
// with alpha_i, beta_i (Eq. (3)), the norm and the test formed in FP32.
// The state's doubles hold the FP32 values exactly.
__device__ void cg_alpha32(DevState *st, float pap, float apap)
{
    if (!(pap > 0.0f) || !isfinite(pap) || !isfinite(apap)) {
        st->status = ST_BREAKDOWN;
        return;
    }
    const float rr = (float)st->rr;
    const float alpha = rr / pap;
    const float beta = alpha * alpha * apap / rr - 1.0f;  // Eq. (3)
    st->alpha = alpha;
    st->beta = beta;
    if (st->it >= st->max_iter)
        st->status = ST_NOT_CONVERGED;
}

__device__ void cg_rr32(DevState *st, float rr)
{
    const int it = st->it + 1;
    st->it = it;
    st->rr = rr;
    st->last_rel = (double)sqrtf(rr) / st->bnorm;
    if (!isfinite(rr))
        st->status = ST_BREAKDOWN;
    else if (sqrtf(rr) <= (float)st->tol)
        st->status = ST_CONVERGED;
    else if (it >= st->max_iter)
        st->status = ST_NOT_CONVERGED;
}

// Algorithm 4: omega_i = <As,s>/<As,As>, beta_i = -<As,r0*>/<Ap,r0*> (the
// form of Section 3.2), and <r_{i+1}, r_{i+1}> expanded in <s,s>, <s,As>,
// <As,As>.
// Algorithms 3/4: alpha_i = rho_i / <Ap_i, r0*>.
__device__ void b_alpha(DevState *st, double apr, double *scal)
{
    const double rho = st->rho;
    if (apr == 0.0 || !isfinite(apr) || rho == 0.0 || !isfinite(rho)) {
        st->status = ST_BREAKDOWN;
        return;
    }
    st->apr = apr;
    st->alpha = rho / apr;
    put_scal(st, scal, st->it, 0, st->alpha);
}

__device__ void b_omega(DevState *st, double ass, double asas, double asr, double *scal)
{
    if (asas == 0.0 || !isfinite(asas) || !isfinite(ass) || !isfinite(asr)) {
        st->status = ST_BREAKDOWN;
        return;
    }
    const double beta = -asr / st->apr;  // via <s_i, r0*> = 0
    const double omega = ass / asas;
    st->beta = beta;
    st->omega = omega;
    st->rr_next = st->ss - 2.0 * omega * ass + omega * omega * asas;
    put_scal(st, scal, st->it, 1, beta);
    put_scal(st, scal, st->it, 2, omega);
}

__device__ void finalize(DevState *st, int fin, const double *d, int K, double *hist, double *scal)
{
    for (int k = 0; k < K; ++k)
        st->dots[k] = d[k];
    switch (fin) {
    case FIN_NONE:
        break;
    case FIN_SETUP: {  // d = {<r0,r0>, <b,b>}
        const double rr = d[0], bb = d[1];
        st->it = 0;
        st->rho_pub = 0;
        st->rr = rr;
        st->rho = rr;  // r0* = r0, so <r0, r0*> = <r0, r0>
        if (bb == 0.0) {
            st->bnorm = 0.0;
            st->tol = 0.0;
            st->last_rel = 0.0;
            put_hist(st, hist, 0, 0.0);
            st->status = ST_ZERO_RHS;
            break;
        }
        const double bnorm = sqrt(bb);
        st->bnorm = bnorm;
        st->tol = st->rtol * bnorm;
        const double rel = sqrt(rr) / bnorm;
        st->last_rel = rel;
        put_hist(st, hist, 0, rel);
        if (!isfinite(rr))
            st->status = ST_BREAKDOWN;
        else if (sqrt(rr) <= st->tol)
            st->status = ST_CONVERGED;
        break;
    }
    case FIN_CG_ALPHA:  // Algorithm 2: d = {<p_i,Ap_i>, <Ap_i,Ap_i>}
        cg_alpha(st, d[0], d[1], scal);
        break;
    case FIN_SETUP32: {  // FP32 inner start: d = {<r0,r0>, <r0,r0>} (FP32 values)
        const float rr = (float)d[0];
        st->it = 0;
        st->rho_pub = 0;
        st->rr = rr;
        if (rr == 0.0f) {
            st->bnorm = 0.0;
            st->tol = 0.0;
            st->last_rel = 0.0;
            st->status = ST_ZERO_RHS;
            break;
        }
        if (!isfinite(rr)) {
            st->status = ST_BREAKDOWN;
            break;
        }
        const float tol = (float)st->rtol * sqrtf(rr);
        st->bnorm = (double)sqrtf(rr);
        st->tol = tol;
        st->last_rel = 1.0;
        if (sqrtf(rr) <= tol)
            st->status = ST_CONVERGED;
        break;
    }
    case FIN_CG_ALPHA32:  // d = {<p_i,Ap_i>, <Ap_i,Ap_i>} (FP32 values)
        cg_alpha32(st, (float)d[0], (float)d[1]);
        break;
    case FIN_CG_RR_ALPHA32:  // d = {<p_i,Ap_i>, <Ap_i,Ap_i>, <r_i,r_i>} (FP32 values)
        cg_rr32(st, (float)d[2]);
        if (st->status == ST_RUNNING)
            cg_alpha32(st, (float)d[0], (float)d[1]);
        break;
    case FIN_CG_RR:  // Algorithm 2: d = {<r_i,r_i>}
        cg_rr(st, d[0], hist, scal);
        break;
    case FIN_CG_RR_ALPHA:  // d = {<p_i,Ap_i>, <Ap_i,Ap_i>, <r_i,r_i>}
        // The convergence test on r_i comes first, as when <r_i,r_i> is
        // reduced on its own; alpha_i, beta_i only while still running.
        cg_rr(st, d[2], hist, scal);
        if (st->status == ST_RUNNING)
            cg_alpha(st, d[0], d[1], scal);
        break;
    case FIN_B_ALPHA:  // Algorithms 3/4: d = {<Ap_i, r0*>}
        b_alpha(st, d[0], scal);
        break;
    case FIN_B_RHO_ALPHA:  // d = {<Ap_i, r0*>, <r_i, r0*>, <r_i, r_i>}
        // rho_i and the direct <r_i,r_i> come from the update's published
        // partials, except in the first iteration (rho_0 from the setup).
        if (st->rho_pub) {
            st->rho = d[1];
            st->rr = d[2];
            st->rho_pub = 0;
        }
        b_alpha(st, d[0], scal);
        break;
    case FIN_B_XRP_ALPHA:  // d = {<Ap_{i+1}, r0*>, <r_{i+1}, r0*>, <r_{i+1}, r_{i+1}>}
        // (two-kernel schedule: the update and the product in one launch)
        st->rho = d[1];
        st->rr = d[2];
        b_alpha(st, d[0], scal);
        break;
    case FIN_B_SS: {  // d = {<s_i, s_i>}: half-step test
        st->ss = d[0];
        if (sqrt(d[0]) <= st->tol)
            st->status = ST_HALF;
        break;
    }
    case FIN_B_OMEGA:  // Algorithm 4: d = {<As,s>, <As,As>, <As,r0*>}
        b_omega(st, d[0], d[1], d[2], scal);
        break;
    case FIN_B_SS_OMEGA: {  // d = {<As,s>, <As,As>, <As,r0*>, <s,s>}
        // The half-step test on s_i first, as when <s_i,s_i> is reduced on
        // its own; omega, beta only while still running.  The decision on
        // iteration i+1 needs only the expanded <r_{i+1}, r_{i+1}> and omega,
        // so it is taken here; the x, r, p update still runs after it.
        st->ss = d[3];
        if (sqrt(d[3]) <= st->tol) {
            st->status = ST_HALF;
            break;
        }
        b_omega(st, d[0], d[1], d[2], scal);
        if (st->status != ST_RUNNING)
            break;
        const int it = st->it + 1;
        st->it = it;
        const double rr_next = st->rr_next;
        const double rnorm = sqrt(rr_next > 0.0 ? rr_next : 0.0);
        const double rel = rnorm / st->bnorm;
        st->last_rel = rel;
        put_hist(st, hist, it, rel);
        put_scal(st, scal, it - 1, 3, rr_next);
        if (!isfinite(rr_next))
            st->status = ST_FINAL_BREAKDOWN;
        else if (rnorm <= st->tol)
            st->status = ST_FINAL_CONVERGED;
        else if (st->omega == 0.0)
            st->status = ST_FINAL_BREAKDOWN;
        else if (it >= st->max_iter)
            st->status = ST_FINAL_NOT_CONVERGED;
        break;
    }
    case FIN_B_XRP_PUB:  // the update after a decision: d = {<r,r0*>, <r,r>}
        if (st->status == ST_HALF) {
            const int it = st->it + 1;
            st->it = it;
            const double rel = sqrt(st->ss) / st->bnorm;
            st->last_rel = rel;
            put_hist(st, hist, it, rel);
            put_scal(st, scal, it - 1, 3, st->ss);
            st->status = ST_CONVERGED;
            break;
        }
        st->rho = d[0];
        st->rr = d[1];
        st->status = st->status == ST_FINAL_CONVERGED       ? ST_CONVERGED
                     : st->status == ST_FINAL_NOT_CONVERGED ? ST_NOT_CONVERGED
                                                            : ST_BREAKDOWN;
        break;
    case FIN_B_XRP: {  // Algorithm 4: d = {<r_{i+1}, r0*>, <r_{i+1}, r_{i+1}>}
        const int it = st->it + 1;
        st->it = it;
        if (st->status == ST_HALF) {
            const double rel = sqrt(st->ss) / st->bnorm;
            st->last_rel = rel;
            put_hist(st, hist, it, rel);
            put_scal(st, scal, it - 1, 3, st->ss);
            st->status = ST_CONVERGED;
            break;
        }
        st->rho = d[0];
        st->rr = d[1];
        const double rr_next = st->rr_next;
        const double rnorm = sqrt(rr_next > 0.0 ? rr_next : 0.0);
        const double rel = rnorm / st->bnorm;
        st->last_rel = rel;
        put_hist(st, hist, it, rel);
        put_scal(st, scal, it - 1, 3, rr_next);
        if (!isfinite(rr_next))
            st->status = ST_BREAKDOWN;
        else if (rnorm <= st->tol)
            st->status = ST_CONVERGED;
        else if (st->omega == 0.0)
            st->status = ST_BREAKDOWN;
        else if (it >= st->max_iter)
            st->status = ST_NOT_CONVERGED;
        break;
    }
    case FIN_C_CG_ALPHA: {  // Algorithm 1: d = {<p_i, A p_i>}
        const double pq = d[0];
        if (!(pq > 0.0) || !isfinite(pq)) {
            st->status = ST_BREAKDOWN;
            break;
        }
        st->alpha = st->rr / pq;
        put_scal(st, scal, st->it, 0, st->alpha);
        break;
    }
    case FIN_C_CG_BETA: {  // Algorithm 1: d = {<r_{i+1}, r_{i+1}>}
        const double rr_new = d[0];
        const int it = st->it + 1;
        st->it = it;
        const double rel = sqrt(rr_new) / st->bnorm;
        st->last_rel = rel;
        put_hist(st, hist, it, rel);
        put_scal(st, scal, it - 1, 3, rr_new);
        if (!isfinite(rr_new)) {
            st->status = ST_BREAKDOWN;
        } else if (sqrt(rr_new) <= st->tol) {
            st->status = ST_CONVERGED;
        } else if (it >= st->max_iter) {
            st->status = ST_NOT_CONVERGED;
        } else {
            st->beta = rr_new / st->rr;
            put_scal(st, scal, it - 1, 1, st->beta);
            st->rr = rr_new;
        }
        break;
    }
    case FIN_C_B_OMEGA: {  // Algorithm 3: d = {<t,s>, <t,t>}, t = A s_i
        const double ts = d[0], tt = d[1];
        if (tt == 0.0 || !isfinite(tt) || !isfinite(ts)) {
            st->status = ST_BREAKDOWN;
            break;
        }
        st->omega = ts / tt;
        put_scal(st, scal, st->it, 2, st->omega);
        break;
    }
    case FIN_C_B_RR: {  // Algorithm 3: d = {<r_{i+1}, r_{i+1}>}
        const double rr = d[0];
        const int it = st->it + 1;
        st->it = it;
        st->rr = rr;
        const double rel = sqrt(rr) / st->bnorm;
        st->last_rel = rel;
        put_hist(st, hist, it, rel);
        put_scal(st, scal, it - 1, 3, rr);
        if (!isfinite(rr))
            st->status = ST_BREAKDOWN;
        else if (sqrt(rr) <= st->tol)
            st->status = ST_CONVERGED;
        break;
    }
    case FIN_C_B_RHO: {  // Algorithm 3: d = {<r_{i+1}, r0*>}
        const double rho_new = d[0];
        if (st->omega == 0.0 || rho_new == 0.0 || !isfinite(rho_new)) {
            st->status = ST_BREAKDOWN;
            break;
        }
        st->beta = (rho_new / st->rho) * (st->alpha / st->omega);
        put_scal(st, scal, st->it - 1, 1, st->beta);
        st->rho = rho_new;
        if (st->it >= st->max_iter)
            st->status = ST_NOT_CONVERGED;
        break;
    }
    case FIN_MIX_OUTER: {  // mixed precision: d = {<r,r>, <b,b>} of r = b - A x in FP64
        const double rr = d[0], bb = d[1];
        const int it = st->it;  // residuals evaluated so far
        if (it == 0) {
            if (bb == 0.0) {
                st->bnorm = 0.0;
                st->tol = 0.0;
                st->last_rel = 0.0;
                put_hist(st, hist, 0, 0.0);
                st->it = 1;
                st->status = ST_ZERO_RHS;
                break;
            }
            st->bnorm = sqrt(bb);
            st->tol = st->rtol * st->bnorm;
        }
        st->rr = rr;
        const double rel = sqrt(rr) / st->bnorm;
        st->last_rel = rel;
        put_hist(st, hist, it, rel);
        st->it = it + 1;
        if (!isfinite(rr))
            st->status = ST_BREAKDOWN;
        else if (sqrt(rr) <= st->tol)
            st->status = ST_CONVERGED;
        break;
    }
    case FIN_GM_SETUP: {  // GMRES cycle start: d = {<r0,r0>, <b,b>}
        const double rr = d[0], bb = d[1];
        if (st->bnorm == 0.0) {  // first cycle of the solve
            if (bb == 0.0) {
                st->last_rel = 0.0;
                put_hist(st, hist, 0, 0.0);
                st->status = ST_ZERO_RHS;
                break;
            }
            st->bnorm = sqrt(bb);
            st->tol = st->rtol * st->bnorm;
        }
        const double rho0 = sqrt(rr);
        st->rho0 = rho0;
        st->last_rel = rho0 / st->bnorm;
        put_hist(st, hist, st->it, rho0 / st->bnorm);
        if (!isfinite(rho0))
            st->status = ST_BREAKDOWN;
        else if (rho0 <= st->tol)
            st->status = ST_CONVERGED;
        else if (st->it >= st->max_iter)
            st->status = ST_NOT_CONVERGED;
        else {
            st->zeta2 = 1.0;
            st->gi = 1;
        }
        break;
    }
    case FIN_GM_R1:  // R[i-1][i] = <v_{i-1}, w> (scal points to R)
        scal[(st->gi - 1) * (st->gm + 1) + st->gi] = d[0];
        break;
    case FIN_GM_NORM: {  // R[i][i] = ||w||; a zero or non-finite norm ends the cycle before step i
        const double rii = sqrt(d[0]);
        if (!(rii > 0.0) || !isfinite(rii))
            st->status = ST_CYCLE_DONE;
        else
            scal[st->gi * (st->gm + 1) + st->gi] = rii;
        break;
    }
    case FIN_GM_XI: {  // xi_i = <r, v_i>; norm estimate rho0 sqrt(zeta2)
        const double xi = d[0];
        const int i = st->gi;
        scal[i] = xi;  // row 0 of R
        double z = st->zeta2 - xi * xi;
        if (z < 0.0)
            z = 0.0;
        st->zeta2 = z;
        const int it = st->it + 1;
        st->it = it;
        const double est = st->rho0 * sqrt(z);
        st->last_rel = est / st->bnorm;
        put_hist(st, hist, it, est / st->bnorm);
        st->gi = i + 1;
        if (est <= st->tol || i + 1 > st->gm || it >= st->max_iter)
            st->status = ST_CYCLE_DONE;
        break;
    }
    case FIN_HALF_DONE: {  // BiCGStab exit after the half step
        const int it = st->it + 1;
        st->it = it;
        const double rel = sqrt(st->ss) / st->bnorm;
        st->last_rel = rel;
        put_hist(st, hist, it, rel);
        put_scal(st, scal, it - 1, 3, st->ss);
        st->status = ST_CONVERGED;
        break;
    }
    default:
        break;
    }
}

// The reduction point at the end of a kernel; every thread of every
// workgroup of the grid must call it exactly once, and return right after.
//
// First stage.  Each wave sums its lanes' partials (wave_sum); waves 1 ..
// WAVES-1 leave theirs in LDS, meet wave 0 at one barrier and exit.  Wave 0
// adds them in wave order.
//
// Second stage, without arrival counters.  Workgroup g of a group of RGROUP
// consecutive (logical) workgroups stores its partials into its own slots
// and ends at once: no wait for the stores, no atomic.  The group's last
// workgroup, its leader, reads the other members' slots, one member per
// lane, polling until none holds the empty marker any more, adds them with
// its own in a wave tree (a fixed order), puts the empty marker back
// and stores the group sum the same way; the leader of the last group,
// workgroup G-1, collects the group sums likewise, rounds once and runs the
// scalar recurrences (finalize).  A slot is read only after the value
// written into it has arrived (each double is stored and read whole, and
// the marker is a signalling NaN, which no arithmetic returns), so no store
// needs to be waited for, and the critical path after the last workgroup's
// rows is two store-to-poll hand-overs instead of arrival round trips.
// Forward progress: at most GMAX / RGROUP leaders poll at once, each holding
// one workgroup slot, and the members they wait for need none of them, so
// the other slots run every member to the end whatever the dispatch order.
// Every poll loop is bounded (RED_SPIN_LIMIT); running out sets red_fault
// and ends the solve with a breakdown, which the host reports as an error
// (and rewrites the markers before the next use).
//
// Published partials.  With fin == FIN_PUBLISH a kernel only stores its
// workgroup partials (first stage) and ends.  A reduction point in a later
// kernel with kpub > 0 folds them in: the leader of group j also sums the
// j-th of ngroups equal slices of the npub published partials (complete
// since the earlier kernel ended), so they ride the same two levels as the
// kernel's own dots.  Algorithm 2 needs <r_i, r_i> only with the product's
// two dots (alpha_i and beta_i need all three), which is what lets the
// update kernel publish it instead of reducing it.
static_assert(RGROUP == 64 && GMAX / RGROUP <= 64, "group and top level are one wave64 each");

// Polls a leader makes before it gives a reduction up (each waits for a
// load from the device's coherence point; 2^22 of them take seconds).
#ifndef FK_RED_SPIN_LIMIT
#define FK_RED_SPIN_LIMIT (1 << 22)
#endif

__device__ __forceinline__ bool red_empty(double x)
{
    return (uint64_t)__double_as_longlong(x) == RED_EMPTY;
}

__device__ __forceinline__ double red_empty_value() { return __longlong_as_double((long long)RED_EMPTY); }

// How a reduction point accumulates.  AccDD: double-double sums of exact
// FP64 products, rounded once (the FP64 path and the exact FP32 mode).
// AccF32: plain FP32 sums (the FP32-accumulating inner solver); a partial is
// stored as the double holding the float, exactly.  Either way every sum
// has a fixed order that depends only on the launch shape.  A slot is two
// doubles; `take` reads one and reports whether it has been written.
struct AccDD {
    using T = dd;
    __device__ static T zero() { return dd{0.0, 0.0}; }
    __device__ static T add(T a, T b) { return dd_add(a, b); }
    __device__ static T wave(T v) { return wave_reduce(v); }
    __device__ static void store(double *slot, T v)
    {
        store_coherent(slot, v.hi);
        store_coherent(slot + 1, v.lo);
    }
    __device__ static T load(const double *slot) { return dd{load_coherent(slot), load_coherent(slot + 1)}; }
    __device__ static bool take(const double *slot, T &out)
    {
        out = load(slot);
        return !red_empty(out.hi) && !red_empty(out.lo);
    }
    __device__ static void clear(double *slot)
    {
        store_coherent(slot, red_empty_value());
        store_coherent(slot + 1, red_empty_value());
    }
    __device__ static double round(T v) { return v.hi + v.lo; }
};

struct AccF32 {
    using T = float;
    __device__ static T zero() { return 0.0f; }
    __device__ static T add(T a, T b) { return a + b; }
    __device__ static T wave(T v) { return wave_sum(v); }
    __device__ static void store(double *slot, T v) { store_coherent(slot, (double)v); }
    __device__ static T load(const double *slot) { return (float)load_coherent(slot); }
    __device__ static bool take(const double *slot, T &out)
    {
        const double d = load_coherent(slot);
        out = (float)d;
        return !red_empty(d);
    }
    __device__ static void clear(double *slot) { store_coherent(slot, red_empty_value()); }
    __device__ static double round(T v) { return (double)v; }
};

// Lane l < count (other than `own`) reads the K slots of member l (slot of
// dot k at base + 2 (k * stride + l)) until all have been written; lane
// `own` takes `mine`, lanes from count on take zero.  Returns false when the
// poll limit ran out.
template <int K, typename ACC>
__device__ __forceinline__ bool collect(const double *base, int stride, int count, int own,
                                        const typename ACC::T (&mine)[K], typename ACC::T (&out)[K])
{
    const int lane = threadIdx.x & 63;
    bool ok = lane >= count || lane == own;
#pragma unroll
    for (int k = 0; k < K; ++k)
        out[k] = lane == own ? mine[k] : ACC::zero();
    for (int spin = 0;; ++spin) {
        if (!ok) {
            bool all = true;
#pragma unroll
            for (int k = 0; k < K; ++k)
                all = ACC::take(base + 2 * ((size_t)k * stride + lane), out[k]) && all;
            ok = all;
        }
        if (__builtin_amdgcn_ballot_w64(!ok) == 0)
            return true;
        if (spin >= FK_RED_SPIN_LIMIT)
            return false;
        __builtin_amdgcn_s_sleep(1);
    }
}

template <int K, typename ACC = AccDD>
__device__ __forceinline__ void reduce_point(typename ACC::T (&v)[K], const RedArgs &red, int g, int G)
{
    using T = typename ACC::T;
    __shared__ T lds[WAVES][KMAX];
    double *const part1 = red.partials;
    double *const part2 = red.partials + RED_L2_OFFSET;
    double *const pub = red.partials + RED_PUB_OFFSET;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int ngroups = (G + RGROUP - 1) / RGROUP;
    const int grp = g / RGROUP;
    const int gbase = grp * RGROUP;
    const int gsize = min(RGROUP, G - gbase);

    // The workgroup that runs finalize asks for the state's lines now, so
    // that they are in its XCD's L2 when finalize reads them (the matrix
    // stream has long evicted them since the kernel read the status).
    double state_line = 0.0;
    const bool finalizer = g == G - 1 && wave == 0 && red.fin != FIN_PUBLISH;
    if (finalizer && lane < (int)(sizeof(DevState) / 128))
        state_line = ((const double *)red.st)[16 * lane];

#pragma unroll
    for (int k = 0; k < K; ++k)
        v[k] = ACC::wave(v[k]);
    if (wave > 0 && lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            lds[wave][k] = v[k];
    }
    __syncthreads();
    if (wave > 0)
        return;
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int w = 1; w < WAVES; ++w)
            v[k] = ACC::add(v[k], lds[w][k]);

    if (red.fin == FIN_PUBLISH) {
        // First stage only; a later reduction point of the same solver, in
        // a later kernel, folds these partials into its own second stage.
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                ACC::store(pub + 2 * ((size_t)k * GMAX + g), v[k]);
        }
        return;
    }
    const int own = gsize - 1;  // the leader's lane: the group's last member
    if (g != gbase + own) {
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                ACC::store(part1 + 2 * ((size_t)k * GMAX + g), v[k]);
        }
        return;
    }

    // Group leader.
    constexpr int KP = (K + KPUB <= KMAX) ? KPUB : KMAX - K;
    constexpr int KT = K + KP;
    const int kpub = KP > 0 ? red.kpub : 0;
    const int kt = K + kpub;
    T mem[K];
    bool done = collect<K, ACC>(part1 + 2 * (size_t)gbase, GMAX, gsize, own, v, mem);
    T acc[KT];
#pragma unroll
    for (int k = 0; k < K; ++k)
        acc[k] = mem[k];
#pragma unroll
    for (int k = K; k < KT; ++k)
        acc[k] = ACC::zero();
    if (kpub > 0) {
        // this group's share of the published partials, in index order
        const int p0 = (int)(((int64_t)red.npub * grp) / ngroups);
        const int p1 = (int)(((int64_t)red.npub * (grp + 1)) / ngroups);
        for (int j = p0 + lane; j < p1; j += 64) {
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                if (k < kpub)
                    acc[K + k] = ACC::add(acc[K + k], ACC::load(pub + 2 * ((size_t)k * GMAX + j)));
            }
        }
    }
    // (slots past kt hold zero in every lane: no sum to form)
#pragma unroll
    for (int k = 0; k < KT; ++k)
        if (k < kt)
            acc[k] = ACC::wave(acc[k]);
    if (ngroups > 1) {
        const int top = ngroups - 1;
        if (grp != top) {
            if (lane == 0) {
                // all KT slots (those past kt hold zero), which the top
                // leader collects whatever kpub is
#pragma unroll
                for (int k = 0; k < KT; ++k)
                    ACC::store(part2 + 2 * ((size_t)k * RNGROUPS_MAX + grp), acc[k]);
                // a leader that gave up voids the reduction and stops the
                // solve; the top leader still receives a sum and ends
                if (!done) {
                    red.st->red_fault = 1;
                    red.st->status = ST_BREAKDOWN;
                }
            }
            // the members' slots are free again for the next launch
            if (lane < gsize && lane != own) {
#pragma unroll
                for (int k = 0; k < K; ++k)
                    ACC::clear(part1 + 2 * ((size_t)k * GMAX + gbase + lane));
            }
            return;
        }
        // Leader of the last group: collect the group sums.
        T sums[KT];
        done = collect<KT, ACC>(part2, RNGROUPS_MAX, ngroups, top, acc, sums) && done;
#pragma unroll
        for (int k = 0; k < KT; ++k)
            if (k < kt)
                acc[k] = ACC::wave(sums[k]);
        if (lane < top) {
#pragma unroll
            for (int k = 0; k < KT; ++k)
                ACC::clear(part2 + 2 * ((size_t)k * RNGROUPS_MAX + lane));
        }
    }
    // the members' slots (of the last group) are free again
    if (lane < gsize && lane != own) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            ACC::clear(part1 + 2 * ((size_t)k * GMAX + gbase + lane));
    }
    asm volatile("" ::"v"(state_line));
    if (lane == 0) {
        if (!done) {
            red.st->red_fault = 1;
            red.st->status = ST_BREAKDOWN;
            return;
        }
        double d[KT > 0 ? KT : 1];
#pragma unroll
        for (int k = 0; k < KT; ++k)
            d[k] = ACC::round(acc[k]);
        finalize(red.st, red.fin, d, kt, red.hist, red.scal);
    }
}

// ---------------------------------------------------- fused CSR products

constexpr int popc3(int b) { return (b & 1) + ((b >> 1) & 1) + ((b >> 2) & 1); }

enum RowMode : int {
    ROW_SPMV = 0,    // y = A v, dots selected by DOTS
    ROW_RESID = 1,   // r = b - A x, p = r (and rs = r); dots <r,r>, <b,b>
    ROW_RESID32 = 2, // r = b - A x rounded to FP32 (r32); dots <r,r>, <b,b> of the FP64 r
};

struct RowIo {
    const double *v;  // vector multiplied (p, s or x)
    double *y;        // result (ROW_SPMV) / r (ROW_RESID)
    const double *w;  // third vector of <y,w> (ROW_SPMV) / b (ROW_RESID*)
    double *p;        // ROW_RESID: p = r
    double *rs;       // ROW_RESID: r0* = r (may be null)
    float *r32;       // ROW_RESID32: FP32 copy of r
};

template <int MODE, int DOTS, int K>
__device__ __forceinline__ void row_epilogue(const RowIo &io, int row, double q, double vrow,
                                             double wrow, dd (&acc)[K])
{
    if constexpr (MODE == ROW_SPMV) {
        io.y[row] = q;
        int k = 0;
        if constexpr ((DOTS & D_YV) != 0) dd_fma(acc[k++], q, vrow);
        if constexpr ((DOTS & D_YY) != 0) dd_fma(acc[k++], q, q);
        if constexpr ((DOTS & D_YW) != 0) dd_fma(acc[k++], q, wrow);
        (void)k;
        (void)vrow;
        (void)wrow;
    } else if constexpr (MODE == ROW_RESID) {
        const double ri = wrow - q;  // wrow = b_i
        io.y[row] = ri;
        io.p[row] = ri;
        if (io.rs)
            io.rs[row] = ri;
        dd_fma(acc[0], ri, ri);
        dd_fma(acc[1], wrow, wrow);
    } else {
        const double ri = wrow - q;  // wrow = b_i
        io.r32[row] = (float)ri;
        dd_fma(acc[0], ri, ri);
        dd_fma(acc[1], wrow, wrow);
    }
}

// One launch processes the row blocks of the plan; workgroup g takes a
// contiguous chunk of blocks.  A block holds at most WG rows and at most
// NNZ_MAX nonzeros (or is a single long row).  Products of a block are
// computed with coalesced loads of vals/col_idx and gathers of v, staged in
// LDS, and each row is then summed left to right by one thread.  Every
// load a block needs (its nonzeros, row pointers and the row entries of the
// vectors in its inner products) is issued before the first wait.
template <int MODE, int DOTS>
__global__ __launch_bounds__(WG, FK_SPMV_MIN_WAVES) void k_csr_rows(DevCsr A, RowIo io, RedArgs red)
{
    if (!runs(red))
        return;
    constexpr int K = (MODE != ROW_SPMV) ? 2 : popc3(DOTS);
    constexpr int KA = K > 0 ? K : 1;
    constexpr bool NEED_V = MODE == ROW_SPMV && (DOTS & D_YV) != 0;
    constexpr bool NEED_W = MODE != ROW_SPMV || (DOTS & D_YW) != 0;
    __shared__ double prod[NNZ_MAX];
    __shared__ int32_t rptr[WG + 1];
    __shared__ double red_lds[WAVES];

    const int G = gridDim.x;
    const int g = logical_wg();
    const int b_begin = (int)(((int64_t)A.nblocks * g) / G);
    const int b_end = (int)(((int64_t)A.nblocks * (g + 1)) / G);
    const int tid = threadIdx.x;
    const double *__restrict__ v = io.v;
    const double *__restrict__ w = io.w;
    const int32_t *__restrict__ col = A.col_idx;
    const double *__restrict__ vals = A.vals;
    const int32_t *__restrict__ row_ptr = A.row_ptr;

    dd acc[KA];
#pragma unroll
    for (int k = 0; k < KA; ++k)
        acc[k] = dd{0.0, 0.0};

    for (int blk = b_begin; blk < b_end; ++blk) {
        const int r0 = A.blocks[blk];
        const int r1 = A.blocks[blk + 1];
        const int j0 = A.block_j0[blk];
        const int nrows = r1 - r0;
        const int nz = A.block_j0[blk + 1] - j0;
        if (nz <= NNZ_MAX) {
            double vrow = 0.0, wrow = 0.0;
            if (tid < nrows) {
                if constexpr (NEED_V)
                    vrow = v[r0 + tid];
                if constexpr (NEED_W)
                    wrow = w[r0 + tid];
                rptr[tid] = row_ptr[r0 + tid] - j0;
            }
            if (tid == 0)
                rptr[nrows] = nz;
            int ci[ITEMS];
            double va[ITEMS];
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int e = tid + i * WG;
                if (e < nz) {
                    ci[i] = load_stream(col + j0 + e);
                    va[i] = load_stream(vals + j0 + e);
                }
            }
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int e = tid + i * WG;
                if (e < nz)
                    prod[e] = va[i] * v[ci[i]];
            }
            __syncthreads();
            if (tid < nrows) {
                const int e0 = rptr[tid], e1 = rptr[tid + 1];
                double q = 0.0;
                for (int e = e0; e < e1; ++e)
                    q = q + prod[e];
                if constexpr (K > 0)
                    row_epilogue<MODE, DOTS, KA>(io, r0 + tid, q, vrow, wrow, acc);
                else
                    io.y[r0 + tid] = q;
            }
            __syncthreads();
        } else {
            // A single row longer than NNZ_MAX: strided partial sums, then a
            // fixed-order tree over the workgroup.
            double part = 0.0;
            for (int e = tid; e < nz; e += WG)
                part = part + vals[j0 + e] * v[col[j0 + e]];
            const double q = block_sum(part, red_lds);
            if (tid == 0) {
                if constexpr (K > 0)
                    row_epilogue<MODE, DOTS, KA>(io, r0, q, NEED_V ? v[r0] : 0.0,
                                                 NEED_W ? w[r0] : 0.0, acc);
                else
                    io.y[r0] = q;
            }
        }
    }
    if constexpr (K > 0)
        reduce_point<KA>(acc, red, g, G);
}

// ------------------------------------------------ sliced-layout products

// Column indices of the lane's row: absolute int32 (-1 = padding), 16-bit
// offsets from the row (SELL_PAD = padding) four to a load, or the slice's
// slot offsets (one per slice and slot, the same for every lane) with the
// row's mask of present slots.
template <int COLS>
struct SliceCols {
    const int32_t *__restrict__ col;   // COLS_INT32: sell_col + e0 + lane
    const short4 *__restrict__ off4;   // COLS_OFF16: sell_off4 + sell_ptr4[s] + lane
    int slot;                          // COLS_SLOTS: lane l holds slot offset l of the slice
    uint32_t mask;                     // COLS_SLOTS: dg_mask[row]
    int row;
    int safe_row;                      // min(row, n - 1): an address every lane may read
};

// The loads behind the columns of entries k .. k+U-1 (COLS_INT32: the
// columns themselves; COLS_OFF16: the packed offsets; COLS_SLOTS: none, the
// slice's slot offsets and the row's mask are loaded once per slice).
template <int U, int COLS>
struct ColsRaw {
    int32_t c[COLS == COLS_INT32 ? U : 1];
    short4 o[COLS == COLS_OFF16 ? (U + 3) / 4 : 1];
};

// Phase 1: issue those loads (k a multiple of U, U a multiple of 4 for
// 16-bit offsets); entries past width are not read.
template <int U, int COLS, bool NT>
__device__ __forceinline__ void cols_issue(const SliceCols<COLS> &sc, int k, int width, ColsRaw<U, COLS> &r)
{
    if constexpr (COLS == COLS_OFF16) {
        static_assert(U % 4 == 0, "16-bit offsets come four to a load");
#pragma unroll
        for (int j = 0; j < U / 4; ++j) {
            r.o[j] = make_short4(SELL_PAD, SELL_PAD, SELL_PAD, SELL_PAD);
            if (k + 4 * j < width)
                r.o[j] = load_stream<NT>(sc.off4 + (size_t)(k / 4 + j) * SLICE);
        }
    } else if constexpr (COLS == COLS_INT32) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            r.c[u] = k + u < width ? load_stream<NT>(sc.col + (size_t)(k + u) * SLICE) : -1;
    }
}

// Phase 2: the columns of entries k .. k+U-1, -1 for padding and past width.
template <int U, int COLS>
__device__ __forceinline__ void cols_decode(const SliceCols<COLS> &sc, int k, int width, const ColsRaw<U, COLS> &r,
                                            int (&c)[U])
{
    if constexpr (COLS == COLS_SLOTS) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = -1;
            if (k + u < width) {
                const int off = __builtin_amdgcn_readlane(sc.slot, k + u);  // slot k+u, to every lane
                if (((sc.mask >> (k + u)) & 1u) != 0u)
                    c[u] = sc.row + off;
            }
        }
    } else if constexpr (COLS == COLS_OFF16) {
#pragma unroll
        for (int j = 0; j < U / 4; ++j) {
            const int16_t os[4] = {r.o[j].x, r.o[j].y, r.o[j].z, r.o[j].w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
                c[4 * j + i] = (k + 4 * j + i < width && os[i] != SELL_PAD) ? sc.row + (int)os[i] : -1;
        }
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
            c[u] = r.c[u];
    }
}

// The vector a sliced product multiplies, read where the row gathers it.
// VecOf: a stored vector.  The fused BiCGStab products below take sources
// that recompute the vector from others at each gathered index instead.
template <typename T>
struct VecOf {
    const T *__restrict__ v;
    __device__ __forceinline__ T at(int c) const { return v[c]; }
};

// Entries k .. k+U-1 of one row of a slice, added to q left to right (the
// row's CSR order).  The column loads and the value loads are all issued
// before the first is waited for; then the U gathers; then the sums.
// width is uniform over the wave, so every test on it is a scalar branch.
// Padding only follows a row's last nonzero and is skipped.
template <typename T, int U, int COLS, bool NT, typename SRC>
__device__ __forceinline__ void slice_row_chunk(const SliceCols<COLS> &cols, const T *__restrict__ vals,
                                                const SRC &v, int k, int width, T &q)
{
    ColsRaw<U, COLS> raw;
    cols_issue<U, COLS, NT>(cols, k, width, raw);
    // Every load below is unconditional, so the chunk is straight-line code
    // and the compiler waits for exactly the loads it needs: entries past
    // width re-read the slice's last entry (a cache hit) and a padding
    // entry gathers the lane's own, clamped row; neither product is added.
    T a[U], x[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
        a[u] = load_stream<NT>(vals + (size_t)min(k + u, width - 1) * SLICE);
    int c[U];
    cols_decode<U, COLS>(cols, k, width, raw, c);
#pragma unroll
    for (int u = 0; u < U; ++u)
        x[u] = v.at(c[u] >= 0 ? c[u] : cols.safe_row);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const T t = q + a[u] * x[u];
        q = c[u] >= 0 ? t : q;
    }
}

// One row of a slice summed left to right: the lane's entries k = 0 ..
// width-1 sit SLICE apart.  A slice of at most U entries per row (every
// stencil here) takes one straight-line chunk, so the compiler can count
// the loads in flight exactly; wider slices loop over chunks of U.
template <typename T, int U, int COLS, bool NT, typename SRC>
__device__ __forceinline__ T slice_row_sum(const SliceCols<COLS> &cols, const T *__restrict__ vals,
                                           const SRC &v, int width)
{
    T q = T(0);
    if constexpr (COLS == COLS_SLOTS) {
        // at most DG_MAX_SLOTS slots: a fixed sequence of chunks, no loop
#pragma unroll
        for (int k = 0; k < DG_MAX_SLOTS; k += U)
            if (k < width)
                slice_row_chunk<T, U, COLS, NT>(cols, vals, v, k, width, q);
    } else {
        for (int k = 0; k < width; k += U)
            slice_row_chunk<T, U, COLS, NT>(cols, vals, v, k, width, q);
    }
    return q;
}


// Start and width of slice sl, read once per wave and held as uniform values.
__device__ __forceinline__ void slice_extent(const DevCsr &A, int sl, int &e0, int &width)
{
    e0 = __builtin_amdgcn_readfirstlane(A.sell_ptr[sl]);
    const int e1 = __builtin_amdgcn_readfirstlane(A.sell_ptr[sl + 1]);
    width = (e1 - e0) / SLICE;
}

// The slices the calling wave takes: first, first + step, ... below end
// (DevCsr::sweep).  Workgroups are dealt to the eight XCDs round robin, so
// blockIdx.x & 7 is the workgroup's XCD; in sweep mode the grid is a
// multiple of 8 and no larger than what is resident at once, so each XCD's
// waves form one window of consecutive slices that advances through the
// XCD's eighth of the matrix: the gathers of a slice's neighbouring planes
// (rows +- n^2 for a 3D stencil) find them in the XCD's own L2, fetched by
// the window a moment earlier or later.
__device__ __forceinline__ void slice_range(const DevCsr &A, int &first, int &end, int &step)
{
    constexpr int WPG = WG / SLICE;  // waves per workgroup
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / SLICE));
    if (A.sweep) {
        const int g8 = gridDim.x >> 3;
        const int x = blockIdx.x & 7;
        const int per = (A.nslices + 7) >> 3;
        first = x * per + (int)(blockIdx.x >> 3) * WPG + wave;
        end = min(A.nslices, (x + 1) * per);
        step = g8 * WPG;
    } else {
        first = logical_wg() * WPG + wave;
        end = A.nslices;
        step = gridDim.x * WPG;
    }
}

// The column form of slice sl for the lane's row.
template <int COLS>
__device__ __forceinline__ SliceCols<COLS> slice_cols_of(const DevCsr &A, int sl, int e0, int lane, int row)
{
    SliceCols<COLS> c{nullptr, nullptr, 0, 0u, row, min(row, A.n - 1)};
    if constexpr (COLS == COLS_INT32)
        c.col = A.sell_col + e0 + lane;
    else if constexpr (COLS == COLS_OFF16)
        c.off4 = A.sell_off4 + __builtin_amdgcn_readfirstlane(A.sell_ptr4[sl]) + lane;
    else {
        // one coalesced load of the slice's slot offsets (width <= 32 lanes;
        // lanes past width read the last slot and do not use it)
        // (the caller skips empty slices, so width >= 1 here)
        const int width = (__builtin_amdgcn_readfirstlane(A.sell_ptr[sl + 1]) - e0) / SLICE;
        c.slot = A.dg_off[e0 / SLICE + min(lane, width - 1)];
        c.mask = A.dg_mask[row];  // sized for every row of every slice
    }
    return c;
}

// The products of k_csr_rows on the sliced layout: one wave per slice, one
// lane per row, no LDS staging and no barrier before the reduction point.
// Wave w of the grid (logical workgroup order) takes slices w, w + W, ...
// for W waves: at any moment the chip streams one contiguous window of the
// slices, each XCD a contiguous eighth of it.  Row sums, epilogues and the
// reduction are those of k_csr_rows, so y is bitwise identical to it.
// NT: the matrix loads non-temporal (DevCsr::stream; a template parameter,
// not a branch, so that each kernel keeps the registers of one path).
// SU: entries requested together, from the widest slice: 5 or 7 slots (the
// slot layout), 4 entries (the other sliced layouts), else FK_SELL_UNROLL;
// a chunk wider than the matrix's slices costs a predicated entry on every
// row (192^3: 110 against 105 us per product with 8 and 7 slots).
template <int MODE, int DOTS, int COLS, bool NT, int SU = FK_SELL_UNROLL>
__global__ __launch_bounds__(WG, FK_SPMV_MIN_WAVES) void k_sell_rows(DevCsr A, RowIo io, RedArgs red)
{
    if (!runs(red))
        return;
    constexpr int K = (MODE != ROW_SPMV) ? 2 : popc3(DOTS);
    constexpr int KA = K > 0 ? K : 1;
    constexpr bool NEED_V = MODE == ROW_SPMV && (DOTS & D_YV) != 0;
    constexpr bool NEED_W = MODE != ROW_SPMV || (DOTS & D_YW) != 0;
    const int G = gridDim.x;
    const int g = logical_wg();
    const int lane = threadIdx.x & (SLICE - 1);
    int sl0, sl_end, sl_step;
    slice_range(A, sl0, sl_end, sl_step);

    dd acc[KA];
#pragma unroll
    for (int k = 0; k < KA; ++k)
        acc[k] = dd{0.0, 0.0};

    for (int sl = sl0; sl < sl_end; sl += sl_step) {
        int e0, width;
        slice_extent(A, sl, e0, width);
        const int row = sl * SLICE + lane;
        const bool live = row < A.n;
        const int srow = min(row, A.n - 1);  // read by every lane, used by live ones
        double vrow = 0.0, wrow = 0.0;
        if constexpr (NEED_V)
            vrow = io.v[srow];
        if constexpr (NEED_W)
            wrow = io.w[srow];
        // (Three double-double accumulators leave room for fewer entries in
        // 64 VGPRs: 4 with int32 columns, 6 with slots.)
        constexpr int U = COLS == COLS_SLOTS ? (KA < 3 || SU < 6 ? SU : 6)
                          : SU < FK_SELL_UNROLL ? SU
                          : KA < 3 ? FK_SELL_UNROLL
                          : COLS == COLS_INT32 ? FK_SELL_UNROLL / 2 : FK_SELL_UNROLL;
        double q = 0.0;
        if (width > 0) {  // uniform: a slice of empty rows reads nothing
            const SliceCols<COLS> cols = slice_cols_of<COLS>(A, sl, e0, lane, row);
            q = slice_row_sum<double, U, COLS, NT>(cols, A.sell_vals + e0 + lane, VecOf<double>{io.v}, width);
        }
        if (live) {
            if constexpr (K > 0)
                row_epilogue<MODE, DOTS, KA>(io, row, q, vrow, wrow, acc);
            else
                io.y[row] = q;
        }
    }
    if constexpr (K > 0)
        reduce_point<KA>(acc, red, g, G);
}

// out[e] = vals[map[e]], or 0 where map[e] < 0: the values of the sliced
// layout gathered once from the CSR values.
__global__ __launch_bounds__(WG) void k_gather_vals(int64_t n, double *__restrict__ out,
                                                     const double *__restrict__ vals,
                                                     const int32_t *__restrict__ map)
{
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
        const int32_t j = map[i];
        out[i] = j >= 0 ? vals[j] : 0.0;
    }
}

// ------------------------------------------- BiCGStab in two kernels
//
// Algorithm 4 with each vector update folded into the product that follows
// it: wherever the product gathers the vector it multiplies, it recomputes
// that vector's entry from the vectors of the update, with the update's own
// expression, so the product sees bitwise the vector the four-kernel
// schedule would have stored.  Two launches per iteration instead of four,
// one full reduction each:
//   k_*_bicg_sas: s_i = r_i - alpha_i A p_i (formed for the own rows and at
//     gathered columns, never stored); A s_i; <As,s>, <As,As>, <As,r0*>,
//     <s,s> (FIN_B_SS_OMEGA: half-step test, omega_i, beta_i, expanded rr,
//     decision);
//   k_*_bicg_xap: x_{i+1}, r_{i+1} = s_i - omega_i A s_i and
//     p_{i+1} = r_{i+1} + beta_i (p_i - omega_i A p_i) for the own rows
//     (s_i formed again from r_i and A p_i), p_{i+1} recomputed at gathered
//     columns; A p_{i+1}; <Ap,r0*>, <r,r0*>, <r,r> (FIN_B_XRP_ALPHA:
//     rho_{i+1}, alpha_{i+1}).
// The product of p_{i+1} gathers r_i, p_i and A p_i while it writes r_{i+1},
// p_{i+1} and A p_{i+1}, so those three alternate between two buffers by
// the parity of i (the device's iteration count, so graph replays and
// batches agree).  After a decision (half step, converged, budget,
// breakdown) the xap launch only finishes x and r, and its own reduction
// ends the solve (FIN_B_XRP_PUB).

#ifndef FK_FUSED_MIN_WAVES
#define FK_FUSED_MIN_WAVES 4
#endif
// Entries of a row requested together by the fused products (each entry
// gathers two or four vectors).
#ifndef FK_FUSED_UNROLL
#define FK_FUSED_UNROLL 5
#endif
#ifndef FK_FUSED_UNROLL_CG
#define FK_FUSED_UNROLL_CG 7
#endif

// s_i = r_i - alpha_i A p_i, as k_bicg_s writes it.
struct VecS {
    const double *__restrict__ r;
    const double *__restrict__ ap;
    double alpha;
    __device__ __forceinline__ double at(int c) const { return r[c] - alpha * ap[c]; }
};

// p_{i+1} = (s_i - omega_i A s_i) + beta_i (p_i - omega_i A p_i) with
// s_i = r_i - alpha_i A p_i, as k_bicg_s and k_bicg_xrp write them.
struct VecP {
    const double *__restrict__ r;
    const double *__restrict__ as;
    const double *__restrict__ p;
    const double *__restrict__ ap;
    double alpha, omega, beta;
    __device__ __forceinline__ double at(int c) const
    {
        const double si = r[c] - alpha * ap[c];
        const double ri = si - omega * as[c];
        return ri + beta * (p[c] - omega * ap[c]);
    }
};

// The s, A s step: own-row inputs, loaded before the row sum.
struct BicgSas {
    static constexpr int K = 4;
    static constexpr int U = FK_FUSED_UNROLL;  // entries requested together (two gathers each)
    Bicg2Io io;
    VecS src;
    struct Own {
        double s, rs;
    };
    __device__ __forceinline__ Own load(int srow) const { return Own{src.at(srow), io.rs[srow]}; }
    __device__ __forceinline__ void row(int row, double q, const Own &o, dd (&acc)[K]) const
    {
        io.as[row] = q;
        dd_fma(acc[0], q, o.s);
        dd_fma(acc[1], q, q);
        dd_fma(acc[2], q, o.rs);
        dd_fma(acc[3], o.s, o.s);
    }
};

// The x, r, p, A p step.
struct BicgXap {
    static constexpr int K = 3;
    static constexpr int U = FK_FUSED_UNROLL;  // (four gathers each)
    Bicg2Io io;
    VecP src;
    double *__restrict__ r_new;
    double *__restrict__ p_new;
    double *__restrict__ ap_new;
    struct Own {
        double x, r, p, as, ap, rs;
    };
    __device__ __forceinline__ Own load(int srow) const
    {
        return Own{io.x[srow], src.r[srow], src.p[srow], src.as[srow], src.ap[srow], io.rs[srow]};
    }
    __device__ __forceinline__ void row(int row, double q, const Own &o, dd (&acc)[K]) const
    {
        const double si = o.r - src.alpha * o.ap;
        io.x[row] = o.x + src.alpha * o.p + src.omega * si;
        const double ri = si - src.omega * o.as;
        r_new[row] = ri;
        p_new[row] = ri + src.beta * (o.p - src.omega * o.ap);
        ap_new[row] = q;
        dd_fma(acc[0], q, o.rs);
        dd_fma(acc[1], ri, o.rs);
        dd_fma(acc[2], ri, ri);
    }
};

// CG in one kernel per iteration (Algorithm 2): the x, r, p update of
// iteration i folded into the product A p_i the same way.  The product
// recomputes p_i = (r_{i-1} - alpha A p_{i-1}) + beta p_{i-1} at every
// gathered column, as k_cg_update writes it.
struct VecCgP {
    const double *__restrict__ r;
    const double *__restrict__ ap;
    const double *__restrict__ p;
    double alpha, beta;
    __device__ __forceinline__ double at(int c) const
    {
        const double ri = r[c] - alpha * ap[c];
        return ri + beta * p[c];
    }
};

// UW: entries requested together (three gathers each): 5 for slices of at
// most 5 entries per row (2D 5-point stencils, one chunk with nothing
// wasted), else 7 (the 7-point stencil in one chunk).
template <int UW>
struct CgXap {
    static constexpr int K = 3;
    static constexpr int U = UW;
    Cg1Io io;
    VecCgP src;
    double *__restrict__ r_new;
    double *__restrict__ p_new;
    double *__restrict__ ap_new;
    struct Own {
        double x, r, p, ap;
    };
    __device__ __forceinline__ Own load(int srow) const
    {
        return Own{io.x[srow], src.r[srow], src.p[srow], src.ap[srow]};
    }
    // {<p_i,Ap_i>, <Ap_i,Ap_i>, <r_i,r_i>}, the dots of FIN_CG_RR_ALPHA
    __device__ __forceinline__ void row(int row, double q, const Own &o, dd (&acc)[K]) const
    {
        io.x[row] = o.x + src.alpha * o.p;
        const double ri = o.r - src.alpha * o.ap;
        r_new[row] = ri;
        const double pi = ri + src.beta * o.p;
        p_new[row] = pi;
        ap_new[row] = q;
        dd_fma(acc[0], q, pi);
        dd_fma(acc[1], q, q);
        dd_fma(acc[2], ri, ri);
    }
};

// r_{i-1}, p_{i-1}, A p_{i-1} sit in buffer (i-1) & 1 and r_i, p_i, A p_i go
// to i & 1 (all three are gathered while the launch writes the new ones);
// the device's count holds i - 1 when the launch starts.
template <int UW>
__device__ __forceinline__ CgXap<UW> cg_xap_of(const Cg1Io &io, const DevState *st)
{
    const int old = st->it & 1, nw = (st->it + 1) & 1;
    return CgXap<UW>{io, VecCgP{io.r[old], io.ap[old], io.p[old], st->alpha, st->beta}, io.r[nw], io.p[nw],
                     io.ap[nw]};
}

// The step's policy from the solver state: the buffers of p_i, A p_i by the
// parity of the iteration count and the scalars of the last reductions.
__device__ __forceinline__ BicgSas bicg_sas_of(const Bicg2Io &io, const DevState *st)
{
    const int cur = st->it & 1;
    return BicgSas{io, VecS{io.r[cur], io.ap[cur], st->alpha}};
}

// (the s step's reduction has counted iteration i + 1 already)
__device__ __forceinline__ BicgXap bicg_xap_of(const Bicg2Io &io, const DevState *st)
{
    const int old = (st->it - 1) & 1, nw = st->it & 1;
    return BicgXap{io, VecP{io.r[old], io.as, io.p[old], io.ap[old], st->alpha, st->omega, st->beta},
                   io.r[nw], io.p[nw], io.ap[nw]};
}

// After a decision: x_{i+1} = x_i + alpha_i p_i and r_{i+1} = s_i (half step),
// or x_{i+1}, r_{i+1} of the full step; the last reduction of the solve
// (FIN_B_XRP_PUB with <r,r0*>, <r,r>) then sets the final status.
__device__ void bicg2_finish(const Bicg2Io &io, int64_t n, const RedArgs &red)
{
    const DevState *st = red.st;
    const bool half = st->status == ST_HALF;
    const double alpha = st->alpha, omega = st->omega;
    // the buffers of iteration i: the count not yet advanced after the half
    // step, one ahead after a decision
    const int cur = half ? (st->it & 1) : ((st->it - 1) & 1);
    const double *__restrict__ p = io.p[cur];
    const double *__restrict__ ap = io.ap[cur];
    double *__restrict__ r = io.r[cur];  // r_{i+1} replaces r_i element by element
    dd acc[2] = {dd{0.0, 0.0}, dd{0.0, 0.0}};
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
        const double si = r[i] - alpha * ap[i];
        if (half) {
            io.x[i] = io.x[i] + alpha * p[i];
            r[i] = si;
        } else {
            io.x[i] = io.x[i] + alpha * p[i] + omega * si;
            const double ri = si - omega * io.as[i];
            r[i] = ri;
            dd_fma(acc[0], ri, io.rs[i]);
            dd_fma(acc[1], ri, ri);
        }
    }
    RedArgs rd = red;
    rd.fin = FIN_B_XRP_PUB;
    reduce_point<2>(acc, rd, blockIdx.x, gridDim.x);
}


// A fused step on the sliced layouts: one wave per slice, one lane per row,
// as k_sell_rows.
template <typename POL, int COLS, bool NT>
__device__ __forceinline__ void sell_fused(const DevCsr &A, const POL &pol, const RedArgs &red)
{
    const int G = gridDim.x;
    const int g = logical_wg();
    const int lane = threadIdx.x & (SLICE - 1);
    int sl0, sl_end, sl_step;
    slice_range(A, sl0, sl_end, sl_step);
    dd acc[POL::K];
#pragma unroll
    for (int k = 0; k < POL::K; ++k)
        acc[k] = dd{0.0, 0.0};
    for (int sl = sl0; sl < sl_end; sl += sl_step) {
        int e0, width;
        slice_extent(A, sl, e0, width);
        const int row = sl * SLICE + lane;
        const typename POL::Own own = pol.load(min(row, A.n - 1));
        double q = 0.0;
        if (width > 0) {
            // (16-bit offsets come four to a load)
            constexpr int U = COLS == COLS_OFF16 ? (POL::U + 3) / 4 * 4 : POL::U;
            const SliceCols<COLS> cols = slice_cols_of<COLS>(A, sl, e0, lane, row);
            q = slice_row_sum<double, U, COLS, NT>(cols, A.sell_vals + e0 + lane, pol.src, width);
        }
        if (row < A.n)
            pol.row(row, q, own, acc);
    }
    reduce_point<POL::K>(acc, red, g, G);
}

// The same on row blocks (as k_csr_rows: products staged in LDS, one
// thread sums a row left to right; a row longer than NNZ_MAX by a fixed
// tree over the workgroup).
template <typename POL>
__device__ __forceinline__ void csr_fused(const DevCsr &A, const POL &pol, const RedArgs &red)
{
    __shared__ double prod[NNZ_MAX];
    __shared__ int32_t rptr[WG + 1];
    __shared__ double red_lds[WAVES];
    const int G = gridDim.x;
    const int g = logical_wg();
    const int b_begin = (int)(((int64_t)A.nblocks * g) / G);
    const int b_end = (int)(((int64_t)A.nblocks * (g + 1)) / G);
    const int tid = threadIdx.x;
    dd acc[POL::K];
#pragma unroll
    for (int k = 0; k < POL::K; ++k)
        acc[k] = dd{0.0, 0.0};
    for (int blk = b_begin; blk < b_end; ++blk) {
        const int r0 = A.blocks[blk];
        const int r1 = A.blocks[blk + 1];
        const int j0 = A.block_j0[blk];
        const int nrows = r1 - r0;
        const int nz = A.block_j0[blk + 1] - j0;
        if (nz <= NNZ_MAX) {
            typename POL::Own own{};
            if (tid < nrows) {
                own = pol.load(r0 + tid);
                rptr[tid] = A.row_ptr[r0 + tid] - j0;
            }
            if (tid == 0)
                rptr[nrows] = nz;
            int ci[ITEMS];
            double va[ITEMS];
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int e = tid + i * WG;
                if (e < nz) {
                    ci[i] = A.col_idx[j0 + e];
                    va[i] = A.vals[j0 + e];
                }
            }
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int e = tid + i * WG;
                if (e < nz)
                    prod[e] = va[i] * pol.src.at(ci[i]);
            }
            __syncthreads();
            if (tid < nrows) {
                const int e0 = rptr[tid], e1 = rptr[tid + 1];
                double q = 0.0;
                for (int e = e0; e < e1; ++e)
                    q = q + prod[e];
                pol.row(r0 + tid, q, own, acc);
            }
            __syncthreads();
        } else {
            double part = 0.0;
            for (int e = tid; e < nz; e += WG)
                part = part + A.vals[j0 + e] * pol.src.at(A.col_idx[j0 + e]);
            const double q = block_sum(part, red_lds);
            if (tid == 0)
                pol.row(r0, q, pol.load(r0), acc);
        }
    }
    reduce_point<POL::K>(acc, red, g, G);
}

template <int COLS, bool NT>
__global__ __launch_bounds__(WG, FK_FUSED_MIN_WAVES) void k_sell_bicg_sas(DevCsr A, Bicg2Io io, RedArgs red)
{
    if (!runs(red))
        return;
    sell_fused<BicgSas, COLS, NT>(A, bicg_sas_of(io, red.st), red);
}

template <int COLS, bool NT>
__global__ __launch_bounds__(WG, FK_FUSED_MIN_WAVES) void k_sell_bicg_xap(DevCsr A, Bicg2Io io, RedArgs red)
{
    if (!runs(red))
        return;
    if (red.st->status != ST_RUNNING) {  // uniform: the state is read-only here
        bicg2_finish(io, A.n, red);
        return;
    }
    sell_fused<BicgXap, COLS, NT>(A, bicg_xap_of(io, red.st), red);
}

__global__ __launch_bounds__(WG, FK_FUSED_MIN_WAVES) void k_csr_bicg_sas(DevCsr A, Bicg2Io io, RedArgs red)
{
    if (!runs(red))
        return;
    csr_fused<BicgSas>(A, bicg_sas_of(io, red.st), red);
}

__global__ __launch_bounds__(WG, FK_FUSED_MIN_WAVES) void k_csr_bicg_xap(DevCsr A, Bicg2Io io, RedArgs red)
{
    if (!runs(red))
        return;
    if (red.st->status != ST_RUNNING) {
        bicg2_finish(io, A.n, red);
        return;
    }
    csr_fused<BicgXap>(A, bicg_xap_of(io, red.st), red);
}

template <int COLS, bool NT, int UW>
__global__ __launch_bounds__(WG, FK_FUSED_MIN_WAVES) void k_sell_cg_xap(DevCsr A, Cg1Io io, RedArgs red)
{
    if (!runs(red))
        return;
    sell_fused<CgXap<UW>, COLS, NT>(A, cg_xap_of<UW>(io, red.st), red);
}

__global__ __launch_bounds__(WG, FK_FUSED_MIN_WAVES) void k_csr_cg_xap(DevCsr A, Cg1Io io, RedArgs red)
{
    if (!runs(red))
        return;
    csr_fused<CgXap<FK_FUSED_UNROLL_CG>>(A, cg_xap_of<FK_FUSED_UNROLL_CG>(io, red.st), red);
}

// --------------------------------------------------- fused vector updates

// Algorithm 2: x_i = x_{i-1} + alpha p_{i-1}; r_i = r_{i-1} - alpha A p_{i-1};
// p_i = r_i + beta p_{i-1}; first stage of <r_i, r_i>.
__global__ __launch_bounds__(WG) void k_cg_update(int64_t n, double *__restrict__ x,
                                                   double *__restrict__ r, double *__restrict__ p,
                                                   const double *__restrict__ ap, RedArgs red)
{
    if (!runs(red))
        return;
    const double alpha = red.st->alpha;
    const double beta = red.st->beta;
    dd acc[1] = {dd{0.0, 0.0}};
    const int64_t stride = (int64_t)gridDim.x * WG;
#pragma unroll FK_VEC_UNROLL
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
        const double pi = p[i];
        x[i] = x[i] + alpha * pi;
        const double ri = r[i] - alpha * ap[i];
        r[i] = ri;
        p[i] = ri + beta * pi;
        dd_fma(acc[0], ri, ri);
    }
    reduce_point<1>(acc, red, blockIdx.x, gridDim.x);
}

// Algorithm 4: s_i = r_i - alpha_i A p_i; first stage of <s_i, s_i>.
__global__ __launch_bounds__(WG) void k_bicg_s(int64_t n, const double *__restrict__ r,
                                                const double *__restrict__ ap,
                                                double *__restrict__ s, RedArgs red)
{
    if (!runs(red))
        return;
    const double alpha = red.st->alpha;
    dd acc[1] = {dd{0.0, 0.0}};
    const int64_t stride = (int64_t)gridDim.x * WG;
#pragma unroll FK_VEC_UNROLL
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
        const double si = r[i] - alpha * ap[i];
        s[i] = si;
        dd_fma(acc[0], si, si);
    }
    reduce_point<1>(acc, red, blockIdx.x, gridDim.x);
}

// Algorithm 4: x_{i+1} = x_i + alpha p_i + omega s_i; r_{i+1} = s_i - omega A s_i;
// p_{i+1} = r_{i+1} + beta (p_i - omega A p_i); first stages of <r_{i+1}, r0*>
// and (for free, r is in registers) <r_{i+1}, r_{i+1}>.  After a half-step
// exit: x_{i+1} = x_i + alpha p_i and r_{i+1} = s_i.
__global__ __launch_bounds__(WG) void k_bicg_xrp(int64_t n, double *__restrict__ x,
                                                  double *__restrict__ r, double *__restrict__ p,
                                                  const double *__restrict__ s,
                                                  const double *__restrict__ as,
                                                  const double *__restrict__ ap,
                                                  const double *__restrict__ rs, RedArgs red)
{
    if (!runs(red))
        return;
    const int32_t status = red.st->status;
    const bool half = status == ST_HALF;
    const double alpha = red.st->alpha;
    const double omega = red.st->omega;
    const double beta = red.st->beta;
    // While the solve runs, <r,r0*>, <r,r> are published for the next
    // product's reduction (FIN_B_RHO_ALPHA); after a decision (half step or
    // iteration i+1 decided) this launch finishes the solve itself.
    RedArgs rd = red;
    if (red.fin == FIN_B_XRP_PUB && status == ST_RUNNING) {
        rd.fin = FIN_PUBLISH;
        if (blockIdx.x == 0 && threadIdx.x == 0)
            red.st->rho_pub = 1;
    }
    dd acc[2] = {dd{0.0, 0.0}, dd{0.0, 0.0}};
    const int64_t stride = (int64_t)gridDim.x * WG;
    if (half) {
#pragma unroll FK_VEC_UNROLL
        for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
            x[i] = x[i] + alpha * p[i];
            r[i] = s[i];
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
            const double si = s[i];
            const double pi = p[i];
            x[i] = x[i] + alpha * pi + omega * si;
            const double ri = si - omega * as[i];
            r[i] = ri;
            p[i] = ri + beta * (pi - omega * ap[i]);
            dd_fma(acc[0], ri, rs[i]);
            dd_fma(acc[1], ri, ri);
        }
    }
    reduce_point<2>(acc, rd, blockIdx.x, gridDim.x);
}

// ------------------------------------------- classical building blocks

// First stage of <a,b> (and <a,c> when NDOT == 2).
// <a, b>, and <a, c>, <a, e> for NDOT = 2, 3: the dots of the classical
// forms, and the separate dot kernels of the split variants of Sections 3.1
// and 3.2 (the product's dots computed in a kernel of their own).
template <int NDOT>
__global__ __launch_bounds__(WG) void k_dot(int64_t n, const double *__restrict__ a,
                                             const double *__restrict__ b,
                                             const double *__restrict__ c,
                                             const double *__restrict__ e, RedArgs red)
{
    if (!runs(red))
        return;
    dd acc[NDOT];
#pragma unroll
    for (int k = 0; k < NDOT; ++k)
        acc[k] = dd{0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
        const double ai = a[i];
        dd_fma(acc[0], ai, b[i]);
        if constexpr (NDOT >= 2)
            dd_fma(acc[1], ai, c[i]);
        if constexpr (NDOT >= 3)
            dd_fma(acc[2], ai, e[i]);
    }
    reduce_point<NDOT>(acc, red, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(WG) void k_axpy(int64_t n, double *__restrict__ out,
                                              const double *y, const double *__restrict__ x,
                                              int which, int negative, const DevState *st,
                                              uint32_t run_mask)
{
    if (((1u << st->status) & run_mask) == 0u)
        return;
    const double c = which == 0 ? st->alpha : st->omega;
    const int64_t stride = (int64_t)gridDim.x * WG;
    if (negative) {
        for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride)
            out[i] = y[i] - c * x[i];
    } else {
        for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride)
            out[i] = y[i] + c * x[i];
    }
}

__global__ __launch_bounds__(WG) void k_xpay(int64_t n, double *__restrict__ p,
                                              const double *__restrict__ r,
                                              const double *__restrict__ v, const DevState *st,
                                              uint32_t run_mask)
{
    if (((1u << st->status) & run_mask) == 0u)
        return;
    const double beta = st->beta;
    const double omega = st->omega;
    const int64_t stride = (int64_t)gridDim.x * WG;
    if (v) {
        for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride)
            p[i] = r[i] + beta * (p[i] - omega * v[i]);
    } else {
        for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride)
            p[i] = r[i] + beta * p[i];
    }
}

// dst = src, then the finalize step `red.fin` on one thread (no inner products).
__global__ __launch_bounds__(WG) void k_copy_fin(int64_t n, double *__restrict__ dst,
                                                  const double *__restrict__ src, RedArgs red)
{
    if (!runs(red))
        return;
    for (int64_t i = threadIdx.x; i < n; i += WG)
        dst[i] = src[i];
    if (threadIdx.x == 0)
        finalize(red.st, red.fin, nullptr, 0, red.hist, red.scal);
}

__global__ __launch_bounds__(WG) void k_zero(double *__restrict__ x, int64_t n,
                                              const DevState *st, uint32_t run_mask)
{
    if (((1u << st->status) & run_mask) == 0u)
        return;
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride)
        x[i] = 0.0;
}

// x[0 .. n) = 0 unconditionally (scratch that must start at zero).
__global__ __launch_bounds__(WG) void k_clear(double *__restrict__ x, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride)
        x[i] = 0.0;
}

// The reduction scratch before its first use: partial slots empty, the
// published partials zero.
__global__ __launch_bounds__(WG) void k_red_init(double *__restrict__ part)
{
    const double empty = __longlong_as_double((long long)RED_EMPTY);
    for (size_t i = (size_t)blockIdx.x * WG + threadIdx.x; i < RED_SCRATCH_DOUBLES; i += (size_t)gridDim.x * WG)
        part[i] = i < RED_PUB_OFFSET ? empty : 0.0;
}

// The state a multi-kernel solve starts from, written by the device (every
// field zero except these).
__global__ __launch_bounds__(64) void k_state_init(DevState *st, double rtol, int32_t max_iter,
                                                    int32_t hist_cap)
{
    if (threadIdx.x != 0)
        return;
    DevState s{};
    s.status = ST_RUNNING;
    s.rtol = rtol;
    s.max_iter = max_iter;
    s.hist_cap = hist_cap;
    *st = s;
}

// ------------------------------------- mixed precision: FP32 inner solver

// Fixed-order workgroup sum of one float (long CSR rows of the FP32 product).
__device__ __forceinline__ float block_sum_f(float v, float *lds)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = v + __shfl_xor(v, off, 64);
    if (lane == 0)
        lds[wave] = v;
    __syncthreads();
    float s = lds[0];
    for (int w = 1; w < WAVES; ++w)
        s = s + lds[w];
    __syncthreads();
    return s;
}

// The two dot accumulators of the FP32 products: exact (the product of two
// floats is exact in FP64, summed in double-double as on the FP64 path, so
// independent of the launch shape) or FP32 (product rounded to FP32, added
// to an FP32 sum).
template <bool F32ACC>
struct Dots32 {
    using ACC = AccDD;
    dd a[2] = {dd{0.0, 0.0}, dd{0.0, 0.0}};
    __device__ void add(float q, float vrow)
    {
        dd_fma(a[0], (double)q, (double)vrow);
        dd_fma(a[1], (double)q, (double)q);
    }
};

template <>
struct Dots32<true> {
    using ACC = AccF32;
    float a[2] = {0.0f, 0.0f};
    __device__ void add(float q, float vrow)
    {
        const float qv = q * vrow;
        const float qq = q * q;
        a[0] = a[0] + qv;
        a[1] = a[1] + qq;
    }
};

// y = A v in FP32 storage and arithmetic (values rounded to FP32 once, when
// the solver is created), each row summed left to right in FP32, fused with
// the first stage of <y, v>, <y, y> (Dots32<F32ACC>): the product kernel of
// the inner pipelined CG of the mixed-precision methods.
template <bool F32ACC>
__global__ __launch_bounds__(WG, FK_SPMV_MIN_WAVES) void k_csr_rows32(DevCsr A, const float *vals32,
                                                                       const float *v, float *y,
                                                                       RedArgs red)
{
    if (!runs(red))
        return;
    __shared__ float prod[NNZ_MAX];
    __shared__ int32_t rptr[WG + 1];
    __shared__ float red_lds[WAVES];
    const int G = gridDim.x;
    const int g = logical_wg();
    const int b_begin = (int)(((int64_t)A.nblocks * g) / G);
    const int b_end = (int)(((int64_t)A.nblocks * (g + 1)) / G);
    const int tid = threadIdx.x;
    Dots32<F32ACC> acc;
    for (int blk = b_begin; blk < b_end; ++blk) {
        const int r0 = A.blocks[blk];
        const int r1 = A.blocks[blk + 1];
        const int j0 = A.block_j0[blk];
        const int nrows = r1 - r0;
        const int nz = A.block_j0[blk + 1] - j0;
        if (nz <= NNZ_MAX) {
            float vrow = 0.f;
            if (tid < nrows) {
                vrow = v[r0 + tid];
                rptr[tid] = A.row_ptr[r0 + tid] - j0;
            }
            if (tid == 0)
                rptr[nrows] = nz;
            int ci[ITEMS];
            float va[ITEMS];
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int e = tid + i * WG;
                if (e < nz) {
                    ci[i] = A.col_idx[j0 + e];
                    va[i] = vals32[j0 + e];
                }
            }
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int e = tid + i * WG;
                if (e < nz)
                    prod[e] = va[i] * v[ci[i]];
            }
            __syncthreads();
            if (tid < nrows) {
                const int e0 = rptr[tid], e1 = rptr[tid + 1];
                float q = 0.f;
                for (int e = e0; e < e1; ++e)
                    q = q + prod[e];
                y[r0 + tid] = q;
                acc.add(q, vrow);
            }
            __syncthreads();
        } else {
            float part = 0.f;
            for (int e = tid; e < nz; e += WG)
                part = part + vals32[j0 + e] * v[A.col_idx[j0 + e]];
            const float q = block_sum_f(part, red_lds);
            if (tid == 0) {
                y[r0] = q;
                acc.add(q, v[r0]);
            }
        }
    }
    reduce_point<2, typename Dots32<F32ACC>::ACC>(acc.a, red, g, G);
}

// k_csr_rows32 on the sliced layout (vals32 in slice order).
template <int COLS, bool F32ACC, bool NT, int SU = FK_SELL_UNROLL>
__global__ __launch_bounds__(WG, FK_SPMV_MIN_WAVES) void k_sell_rows32(DevCsr A, const float *vals32,
                                                                        const float *v, float *y,
                                                                        RedArgs red)
{
    if (!runs(red))
        return;
    const int G = gridDim.x;
    const int g = logical_wg();
    const int lane = threadIdx.x & (SLICE - 1);
    int sl0, sl_end, sl_step;
    slice_range(A, sl0, sl_end, sl_step);
    Dots32<F32ACC> acc;
    for (int sl = sl0; sl < sl_end; sl += sl_step) {
        int e0, width;
        slice_extent(A, sl, e0, width);
        const int row = sl * SLICE + lane;
        const bool live = row < A.n;
        const float vrow = v[min(row, A.n - 1)];
        float q = 0.f;
        if (width > 0) {  // uniform: a slice of empty rows reads nothing
            const SliceCols<COLS> cols = slice_cols_of<COLS>(A, sl, e0, lane, row);
            q = slice_row_sum<float, COLS == COLS_SLOTS ? SU : FK_SELL_UNROLL, COLS, NT>(cols, vals32 + e0 + lane,
                                                                                     VecOf<float>{v}, width);
        }
        if (live) {
            y[row] = q;
            acc.add(q, vrow);
        }
    }
    reduce_point<2, typename Dots32<F32ACC>::ACC>(acc.a, red, g, G);
}

// Inner FP32 update of Algorithm 2 (alpha, beta held in FP32):
// d += alpha p; r -= alpha A p; p = r + beta p; first stage of <r, r>
// (Dots32<F32ACC>: both slots take <r, r>, the first is reduced).
template <bool F32ACC>
__global__ __launch_bounds__(WG) void k_cg_update32(int64_t n, float *__restrict__ d,
                                                     float *__restrict__ r, float *__restrict__ p,
                                                     const float *__restrict__ ap, RedArgs red)
{
    if (!runs(red))
        return;
    const float alpha = (float)red.st->alpha;
    const float beta = (float)red.st->beta;
    typename Dots32<F32ACC>::ACC::T acc[1] = {Dots32<F32ACC>::ACC::zero()};
    const int64_t stride = (int64_t)gridDim.x * WG;
#pragma unroll FK_VEC_UNROLL
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
        const float pi = p[i];
        d[i] = d[i] + alpha * pi;
        const float ri = r[i] - alpha * ap[i];
        r[i] = ri;
        p[i] = ri + beta * pi;
        if constexpr (F32ACC) {
            const float rr = ri * ri;
            acc[0] = acc[0] + rr;
        } else {
            dd_fma(acc[0], (double)ri, (double)ri);
        }
    }
    reduce_point<1, typename Dots32<F32ACC>::ACC>(acc, red, blockIdx.x, gridDim.x);
}

// Inner start (d0 = 0): p = r, d = 0, first stage of <r, r> (reported twice,
// as the residual norm and as the norm of the inner right-hand side).
template <bool F32ACC>
__global__ __launch_bounds__(WG) void k_inner_setup32(int64_t n, const float *__restrict__ r,
                                                       float *__restrict__ p, float *__restrict__ d,
                                                       RedArgs red)
{
    if (!runs(red))
        return;
    Dots32<F32ACC> acc;
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride) {
        const float ri = r[i];
        p[i] = ri;
        d[i] = 0.f;
        acc.add(ri, ri);
    }
    reduce_point<2, typename Dots32<F32ACC>::ACC>(acc.a, red, blockIdx.x, gridDim.x);
}

// out = alpha x + beta y.
// (out may alias x or y: each element is read before it is written)
__global__ __launch_bounds__(WG) void k_axpby(int64_t n, double alpha, const double *x, double beta,
                                               const double *y, double *out)
{
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride)
        out[i] = alpha * x[i] + beta * y[i];
}

// x += d in FP64 (the refinement's correction).
__global__ __launch_bounds__(WG) void k_add32(int64_t n, double *__restrict__ x,
                                               const float *__restrict__ d)
{
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride)
        x[i] = x[i] + (double)d[i];
}

// FP64 values rounded to FP32.
__global__ __launch_bounds__(WG) void k_to_f32(int64_t n, float *__restrict__ out,
                                                const double *__restrict__ in)
{
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += stride)
        out[i] = (float)in[i];
}


// -------------------------------------------------------------- GMRES(m)

__device__ __forceinline__ bool runs_mask(const DevState *st, uint32_t mask)
{
    return ((1u << st->status) & mask) != 0u;
}

// out = in / rho0 (out may be in: each element is read before it is written).
__global__ __launch_bounds__(WG) void k_gm_scale(int64_t n, double *out, const double *in, DevState *st,
                                                  uint32_t mask)
{
    if (!runs_mask(st, mask))
        return;
    const double rho0 = st->rho0;
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x; t < n; t += stride)
        out[t] = in[t] / rho0;
}

// First stage of R[j][i] = <v_j, w> for j0 <= j < j1, all from the same w
// (classical Gram-Schmidt).  Workgroup g owns a contiguous chunk of rows and
// keeps GM_JT double-double accumulators at a time; a thread requests GM_RU
// of its rows (and their GM_JT basis entries) at once, then adds them in row
// order.  Its partials go to part[j][g]; k_gm_multidot_fin does the second
// stage.
constexpr int GM_JT = 8;
constexpr int GM_RU = 4;
__global__ __launch_bounds__(WG) void k_gm_multidot(int64_t n, const double *__restrict__ V,
                                                     const double *__restrict__ w, int j0, int j1,
                                                     double *part, DevState *st, uint32_t mask)
{
    if (!runs_mask(st, mask))
        return;
    __shared__ dd lds[WAVES][KMAX];
    const int G = gridDim.x, g = blockIdx.x;
    const int64_t lo = n * g / G, hi = n * (g + 1) / G;
    for (int jt = j0; jt < j1; jt += GM_JT) {
        dd acc[GM_JT];
#pragma unroll
        for (int q = 0; q < GM_JT; ++q)
            acc[q] = dd{0.0, 0.0};
        for (int64_t t0 = lo + threadIdx.x; t0 < hi; t0 += GM_RU * WG) {
            double wt[GM_RU], vv[GM_RU][GM_JT];
#pragma unroll
            for (int u = 0; u < GM_RU; ++u) {
                const int64_t t = t0 + (int64_t)u * WG;
                wt[u] = t < hi ? w[t] : 0.0;
#pragma unroll
                for (int q = 0; q < GM_JT; ++q)
                    vv[u][q] = (t < hi && jt + q < j1) ? V[(size_t)(jt + q) * n + t] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < GM_RU; ++u) {
                if (t0 + (int64_t)u * WG < hi) {
#pragma unroll
                    for (int q = 0; q < GM_JT; ++q)
                        if (jt + q < j1)
                            dd_fma(acc[q], vv[u][q], wt[u]);
                }
            }
        }
        // block sums, KMAX at a time
#pragma unroll
        for (int q0 = 0; q0 < GM_JT; q0 += KMAX) {
            dd v4[KMAX];
#pragma unroll
            for (int q = 0; q < KMAX; ++q)
                v4[q] = acc[q0 + q];
            block_reduce<KMAX>(v4, lds);
            if (threadIdx.x == 0) {
#pragma unroll
                for (int q = 0; q < KMAX; ++q) {
                    const int j = jt + q0 + q;
                    if (j < j1) {
                        double *slot = part + 2 * ((size_t)j * GM_GRID + g);
                        slot[0] = v4[q].hi;
                        slot[1] = v4[q].lo;
                    }
                }
            }
        }
    }
}

// Second stage: workgroup b sums dot j = j0 + b over the G partials of
// k_gm_multidot (thread t takes partials t, t + WG, ..., then a fixed tree)
// and writes R[j][i].
__global__ __launch_bounds__(WG) void k_gm_multidot_fin(int G, int j0, int i, double *R, int m1,
                                                         const double *__restrict__ part, DevState *st,
                                                         uint32_t mask)
{
    if (!runs_mask(st, mask))
        return;
    __shared__ dd lds[WAVES][KMAX];
    const int j = j0 + (int)blockIdx.x;
    dd a[1] = {dd{0.0, 0.0}};
    for (int g = threadIdx.x; g < G; g += WG) {
        const double *slot = part + 2 * ((size_t)j * GM_GRID + g);
        a[0] = dd_add(a[0], dd{slot[0], slot[1]});
    }
    block_reduce<1>(a, lds);
    if (threadIdx.x == 0)
        R[(size_t)j * m1 + i] = a[0].hi + a[0].lo;
}

// w -= sum_{j=1}^{i-1} R[j][i] v_j (j in order); first stage of <w, w>.
// A thread updates GM_RU of its elements at once (independent chains, their
// loads together), then adds them to <w, w> in element order.
__global__ __launch_bounds__(WG) void k_gm_update(int64_t n, double *__restrict__ w,
                                                   const double *__restrict__ V, int i, int m1, RedArgs red)
{
    if (!runs(red))
        return;
    const double *R = red.scal;
    dd acc[1] = {dd{0.0, 0.0}};
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t t0 = (int64_t)blockIdx.x * WG + threadIdx.x; t0 < n; t0 += GM_RU * stride) {
        double wt[GM_RU];
#pragma unroll
        for (int u = 0; u < GM_RU; ++u) {
            const int64_t t = t0 + u * stride;
            wt[u] = t < n ? w[t] : 0.0;
        }
        for (int j = 1; j < i; ++j) {
            const double rj = R[(size_t)j * m1 + i];
#pragma unroll
            for (int u = 0; u < GM_RU; ++u) {
                const int64_t t = t0 + u * stride;
                if (t < n)
                    wt[u] = wt[u] - rj * V[(size_t)j * n + t];
            }
        }
#pragma unroll
        for (int u = 0; u < GM_RU; ++u) {
            const int64_t t = t0 + u * stride;
            if (t < n) {
                w[t] = wt[u];
                dd_fma(acc[0], wt[u], wt[u]);
            }
        }
    }
    reduce_point<1>(acc, red, blockIdx.x, gridDim.x);
}

// v_i = w / R[i][i] (in place); first stage of <r, v_i>.
__global__ __launch_bounds__(WG) void k_gm_normalize(int64_t n, double *__restrict__ v,
                                                      const double *__restrict__ r, int i, int m1, RedArgs red)
{
    if (!runs(red))
        return;
    const double rii = red.scal[(size_t)i * m1 + i];
    dd acc[1] = {dd{0.0, 0.0}};
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x; t < n; t += stride) {
        const double vt = v[t] / rii;
        v[t] = vt;
        dd_fma(acc[0], r[t], vt);
    }
    reduce_point<1>(acc, red, blockIdx.x, gridDim.x);
}

// r -= xi_i v_i (xi_i in row 0 of R).  Runs after the step was counted,
// so it checks the step index rather than the status.
__global__ __launch_bounds__(WG) void k_gm_rupdate(int64_t n, double *__restrict__ r,
                                                    const double *__restrict__ v, int i,
                                                    const double *__restrict__ R, DevState *st, uint32_t mask)
{
    if (!runs_mask(st, mask) || st->gi != i + 1)
        return;
    const double xi = R[i];
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x; t < n; t += stride)
        r[t] = r[t] - xi * v[t];
}

// x += rho0 (eta_1 v_0 + sum_{j=2}^{used} eta_j v_{j-1}), the sum in j order.
__global__ __launch_bounds__(WG) void k_gm_xupdate(int64_t n, double *__restrict__ x,
                                                    const double *__restrict__ V,
                                                    const double *__restrict__ eta, int used,
                                                    const DevState *st)
{
    const double rho0 = st->rho0;
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x; t < n; t += stride) {
        double s = eta[1] * V[t];
        for (int j = 2; j <= used; ++j)
            s = s + eta[j] * V[(size_t)(j - 1) * n + t];
        x[t] = x[t] + rho0 * s;
    }
}

// ------------------------------------------- single-workgroup solver

// A whole pipelined CG or BiCGStab solve in one workgroup of SWG threads,
// for systems small enough that one CU holds them: the launch latency of the
// multi-kernel iteration would dominate (Section 2.1's latency barrier), and
// with one workgroup every global synchronisation of the iteration becomes a
// workgroup barrier.  Thread t owns rows t, t + SWG, ... (RPT of them) and
// keeps their vector entries in registers; the vectors the products gather
// (p, and s for BiCGStab) live in LDS; the matrix is read from global memory
// (it stays in the caches).  Rows are summed left to right and inner
// products accumulated in double-double exactly as in the grid kernels, and
// the scalar steps are the same `finalize` cases applied in the same order,
// so the iterates are those of the multi-kernel path.  Because one
// workgroup sees every partial at once, the inner products that the grid
// path reduces at separate points are reduced together: one reduction per
// CG iteration ({<r_i,r_i>, <p_i,Ap_i>, <Ap_i,Ap_i>}), two per BiCGStab
// iteration.  The iteration count is bounded by max_iter.
constexpr int SWG = 1024;  // the most threads (and rows per thread: 4) it takes

// The matrix as the single-workgroup solver reads it: from LDS when it was
// staged there at the start of the solve, else from global memory.
struct SmallCsr {
    const int32_t *rp;
    const int32_t *ci;
    const double *va;
};

__device__ __forceinline__ double row_sum(const SmallCsr &A, int i, const double *v)
{
    const int j0 = A.rp[i], j1 = A.rp[i + 1];
    double q = 0.0;
    for (int j = j0; j < j1; ++j)
        q = q + A.va[j] * v[A.ci[j]];
    return q;
}

// Bytes of LDS the matrix takes when staged: vals, col_idx, row_ptr.
__host__ __device__ constexpr size_t small_csr_bytes(int64_t n, int64_t nnz)
{
    return (size_t)nnz * 12 + (size_t)(n + 1) * 4;
}

// Copy the matrix into LDS behind the vectors (8-byte aligned start).
template <int WGS>
__device__ __forceinline__ SmallCsr stage_csr(const DevCsr &A, char *base)
{
    double *va = reinterpret_cast<double *>(base);
    int32_t *ci = reinterpret_cast<int32_t *>(va + A.nnz);
    int32_t *rp = ci + A.nnz;
    for (int j = threadIdx.x; j < A.nnz; j += WGS) {
        va[j] = A.vals[j];
        ci[j] = A.col_idx[j];
    }
    for (int j = threadIdx.x; j <= A.n; j += WGS)
        rp[j] = A.row_ptr[j];
    return SmallCsr{rp, ci, va};
}

// Workgroup reduction of K double-doubles (each wave by its DPP tree, then
// the NW wave results by shuffles in wave 0, a fixed tree), followed by the
// finalize steps fins[0..nf) on thread 0, each taking its slice of the
// rounded sums and applied only while the solve is in state needs[f].  Ends
// past a barrier, so every thread sees the updated state.
template <int K, int NW>
__device__ __forceinline__ void small_reduce(dd (&v)[K], dd (*lds)[KMAX], DevState &s,
                                             const int *fins, const int *ks, const int *needs,
                                             int nf, double *hist, double *scal)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k)
        v[k] = wave_reduce(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            lds[wave][k] = v[k];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            dd t = lane < NW ? lds[lane][k] : dd{0.0, 0.0};
            v[k] = lanes_sum(t, NW);
        }
        if (lane == 0) {
            double d[K];
#pragma unroll
            for (int k = 0; k < K; ++k)
                d[k] = v[k].hi + v[k].lo;
            int off = 0;
            for (int f = 0; f < nf; ++f) {
                if (s.status == needs[f])
                    finalize(&s, fins[f], d + off, ks[f], hist, scal);
                off += ks[f];
            }
        }
    }
    __syncthreads();
}

template <int RPT, bool STAGE, int WGS>
__global__ __launch_bounds__(WGS) void k_small_cg(DevCsr Ag, const double *__restrict__ b,
                                                  double *__restrict__ x, DevState *gst,
                                                  double *hist, double *scal)
{
    extern __shared__ double pv[];  // p (first x0) for the gathers, n entries; then the matrix
    __shared__ DevState s;
    __shared__ dd lds[WGS / 64][KMAX];
    const int tid = threadIdx.x;
    const int n = Ag.n;
    if (tid == 0)
        s = *gst;
    const SmallCsr A = STAGE ? stage_csr<WGS>(Ag, reinterpret_cast<char *>(pv + n))
                             : SmallCsr{Ag.row_ptr, Ag.col_idx, Ag.vals};
    double xr[RPT], rr[RPT], pr[RPT], apr[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * WGS;
        xr[k] = rr[k] = pr[k] = apr[k] = 0.0;
        if (i < n) {
            xr[k] = x[i];
            pv[i] = xr[k];
        }
    }
    __syncthreads();
    {   // r0 = b - A x0, p0 = r0, <r0,r0>, <b,b>
        dd acc[2] = {dd{0.0, 0.0}, dd{0.0, 0.0}};
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + k * WGS;
            if (i < n) {
                const double bi = b[i];
                const double ri = bi - row_sum(A, i, pv);
                rr[k] = ri;
                pr[k] = ri;
                dd_fma(acc[0], ri, ri);
                dd_fma(acc[1], bi, bi);
            }
        }
        const int fins[1] = {FIN_SETUP}, ks[1] = {2}, needs[1] = {ST_RUNNING};
        small_reduce<2, WGS / 64>(acc, lds, s, fins, ks, needs, 1, hist, scal);
    }
    if (s.status == ST_RUNNING) {  // A p0, alpha_0, beta_0
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + k * WGS;
            if (i < n)
                pv[i] = pr[k];
        }
        __syncthreads();
        dd acc[2] = {dd{0.0, 0.0}, dd{0.0, 0.0}};
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + k * WGS;
            if (i < n) {
                const double q = row_sum(A, i, pv);
                apr[k] = q;
                dd_fma(acc[0], q, pr[k]);
                dd_fma(acc[1], q, q);
            }
        }
        const int fins[1] = {FIN_CG_ALPHA}, ks[1] = {2}, needs[1] = {ST_RUNNING};
        small_reduce<2, WGS / 64>(acc, lds, s, fins, ks, needs, 1, hist, scal);
    }
    while (s.status == ST_RUNNING) {
        const double alpha = s.alpha, beta = s.beta;
        dd acc[3] = {dd{0.0, 0.0}, dd{0.0, 0.0}, dd{0.0, 0.0}};
        // x_i, r_i, p_i and <r_i, r_i>
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + k * WGS;
            if (i < n) {
                const double pi = pr[k];
                xr[k] = xr[k] + alpha * pi;
                const double ri = rr[k] - alpha * apr[k];
                rr[k] = ri;
                const double pn = ri + beta * pi;
                pr[k] = pn;
                pv[i] = pn;
                dd_fma(acc[0], ri, ri);
            }
        }
        __syncthreads();
        // A p_i, <p_i, A p_i>, <A p_i, A p_i>
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + k * WGS;
            if (i < n) {
                const double q = row_sum(A, i, pv);
                apr[k] = q;
                dd_fma(acc[1], q, pr[k]);
                dd_fma(acc[2], q, q);
            }
        }
        const int fins[2] = {FIN_CG_RR, FIN_CG_ALPHA}, ks[2] = {1, 2},
                  needs[2] = {ST_RUNNING, ST_RUNNING};
        small_reduce<3, WGS / 64>(acc, lds, s, fins, ks, needs, 2, hist, scal);
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * WGS;
        if (i < n)
            x[i] = xr[k];
    }
    if (tid == 0)
        *gst = s;
}

template <int RPT, bool STAGE, int WGS>
__global__ __launch_bounds__(WGS) void k_small_bicgstab(DevCsr Ag, const double *__restrict__ b,
                                                        double *__restrict__ x, DevState *gst,
                                                        double *hist, double *scal)
{
    extern __shared__ double lv[];  // p (first x0) and s for the gathers, 2n entries; then the matrix
    const int n = Ag.n;
    double *pv = lv;
    double *sv = lv + n;
    __shared__ DevState s;
    __shared__ dd lds[WGS / 64][KMAX];
    const int tid = threadIdx.x;
    if (tid == 0)
        s = *gst;
    const SmallCsr A = STAGE ? stage_csr<WGS>(Ag, reinterpret_cast<char *>(lv + 2 * n))
                             : SmallCsr{Ag.row_ptr, Ag.col_idx, Ag.vals};
    double xr[RPT], rr[RPT], pr[RPT], apr[RPT], rsr[RPT], sr[RPT], asr[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * WGS;
        xr[k] = rr[k] = pr[k] = apr[k] = rsr[k] = sr[k] = asr[k] = 0.0;
        if (i < n) {
            xr[k] = x[i];
            pv[i] = xr[k];
        }
    }
    __syncthreads();
    {   // r0 = b - A x0, r0* = r0, p0 = r0, <r0,r0>, <b,b>
        dd acc[2] = {dd{0.0, 0.0}, dd{0.0, 0.0}};
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + k * WGS;
            if (i < n) {
                const double bi = b[i];
                const double ri = bi - row_sum(A, i, pv);
                rr[k] = rsr[k] = pr[k] = ri;
                dd_fma(acc[0], ri, ri);
                dd_fma(acc[1], bi, bi);
            }
        }
        const int fins[1] = {FIN_SETUP}, ks[1] = {2}, needs[1] = {ST_RUNNING};
        small_reduce<2, WGS / 64>(acc, lds, s, fins, ks, needs, 1, hist, scal);
    }
    // <r, r0*> and <r, r> of the last update, reduced with the next <Ap, r0*>
    dd carry[2] = {dd{0.0, 0.0}, dd{0.0, 0.0}};
    bool first = true;
    while (s.status == ST_RUNNING && s.it < s.max_iter) {
        // A p_i and <A p_i, r0*> (with the previous update's inner products)
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + k * WGS;
            if (i < n)
                pv[i] = pr[k];
        }
        __syncthreads();
        dd acc1[3] = {carry[0], carry[1], dd{0.0, 0.0}};
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + k * WGS;
            if (i < n) {
                const double q = row_sum(A, i, pv);
                apr[k] = q;
                dd_fma(acc1[2], q, rsr[k]);
            }
        }
        {
            const int fins[2] = {first ? FIN_NONE : FIN_B_XRP, FIN_B_ALPHA}, ks[2] = {2, 1},
                      needs[2] = {ST_RUNNING, ST_RUNNING};
            small_reduce<3, WGS / 64>(acc1, lds, s, fins, ks, needs, 2, hist, scal);
        }
        first = false;
        if (s.status != ST_RUNNING)
            break;
        // s_i = r_i - alpha A p_i, A s_i, and four inner products
        const double alpha = s.alpha;
        dd acc2[4] = {dd{0.0, 0.0}, dd{0.0, 0.0}, dd{0.0, 0.0}, dd{0.0, 0.0}};
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + k * WGS;
            if (i < n) {
                const double si = rr[k] - alpha * apr[k];
                sr[k] = si;
                sv[i] = si;
                dd_fma(acc2[0], si, si);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + k * WGS;
            if (i < n) {
                const double q = row_sum(A, i, sv);
                asr[k] = q;
                dd_fma(acc2[1], q, sr[k]);
                dd_fma(acc2[2], q, q);
                dd_fma(acc2[3], q, rsr[k]);
            }
        }
        {
            const int fins[2] = {FIN_B_SS, FIN_B_OMEGA}, ks[2] = {1, 3},
                      needs[2] = {ST_RUNNING, ST_RUNNING};
            small_reduce<4, WGS / 64>(acc2, lds, s, fins, ks, needs, 2, hist, scal);
        }
        if (s.status == ST_HALF) {
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                xr[k] = xr[k] + alpha * pr[k];
                rr[k] = sr[k];
            }
            if (tid == 0)
                finalize(&s, FIN_B_XRP, nullptr, 0, hist, scal);
            __syncthreads();
            break;
        }
        if (s.status != ST_RUNNING)
            break;
        const double omega = s.omega, beta = s.beta;
        carry[0] = carry[1] = dd{0.0, 0.0};
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + k * WGS;
            if (i < n) {
                const double si = sr[k];
                const double pi = pr[k];
                xr[k] = xr[k] + alpha * pi + omega * si;
                const double ri = si - omega * asr[k];
                rr[k] = ri;
                pr[k] = ri + beta * (pi - omega * apr[k]);
                dd_fma(carry[0], ri, rsr[k]);
                dd_fma(carry[1], ri, ri);
            }
        }
        // The last update's inner products are reduced with the next A p;
        // when that one cannot run any more, reduce them now.
        if (s.it + 1 >= s.max_iter) {
            dd fin2[2] = {carry[0], carry[1]};
            const int fins[1] = {FIN_B_XRP}, ks[1] = {2}, needs[1] = {ST_RUNNING};
            small_reduce<2, WGS / 64>(fin2, lds, s, fins, ks, needs, 1, hist, scal);
            break;
        }
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int i = tid + k * WGS;
        if (i < n)
            x[i] = xr[k];
    }
    if (tid == 0)
        *gst = s;
}

// Streaming copy with 16-byte accesses, four in flight per thread
// (bandwidth calibration).
__global__ __launch_bounds__(WG) void k_copy16(int4 *__restrict__ dst, const int4 *__restrict__ src,
                                                int64_t n16)
{
    const int64_t stride = (int64_t)gridDim.x * WG;
    int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const int4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n16; i += stride)
        dst[i] = src[i];
}

__global__ void k_copy_tail(char *__restrict__ dst, const char *__restrict__ src, int64_t n)
{
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
        dst[i] = src[i];
}

thread_local hipEvent_t t_start = nullptr;
thread_local hipEvent_t t_stop = nullptr;

template <typename... KArgs, typename... Args>
hipError_t launch_shm(void (*kernel)(KArgs...), int grid, int block, size_t shm, hipStream_t s,
                      Args... args)
{
    if (t_start) {
        hipEvent_t a = t_start, b = t_stop;
        t_start = t_stop = nullptr;
        hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), (uint32_t)shm, s, a, b, 0,
                              static_cast<KArgs>(args)...);
    } else {
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), (uint32_t)shm, s,
                           static_cast<KArgs>(args)...);
    }
    return hipGetLastError();
}

template <typename... KArgs, typename... Args>
hipError_t launch(void (*kernel)(KArgs...), int grid, int block, hipStream_t s, Args... args)
{
    return launch_shm(kernel, grid, block, 0, s, args...);
}

}  // namespace

// ------------------------------------------------------ launch wrappers

void set_launch_timing(hipEvent_t start, hipEvent_t stop)
{
    t_start = start;
    t_stop = stop;
}

// The product kernel of A's layout.
template <int MODE, int DOTS, bool NT>
static hipError_t launch_sell(const DevCsr &A, const RowIo &io, const RedArgs &red, int grid, hipStream_t s)
{
    if (A.dg_mask) {
        if (A.max_width <= 5)
            return launch(k_sell_rows<MODE, DOTS, COLS_SLOTS, NT, 5>, grid, WG, s, A, io, red);
        if (A.max_width <= 7)
            return launch(k_sell_rows<MODE, DOTS, COLS_SLOTS, NT, 7>, grid, WG, s, A, io, red);
        return launch(k_sell_rows<MODE, DOTS, COLS_SLOTS, NT>, grid, WG, s, A, io, red);
    }
    if (A.sell_off4) {
        if (A.max_width <= 4)
            return launch(k_sell_rows<MODE, DOTS, COLS_OFF16, NT, 4>, grid, WG, s, A, io, red);
        return launch(k_sell_rows<MODE, DOTS, COLS_OFF16, NT>, grid, WG, s, A, io, red);
    }
    if (A.max_width <= 4)
        return launch(k_sell_rows<MODE, DOTS, COLS_INT32, NT, 4>, grid, WG, s, A, io, red);
    return launch(k_sell_rows<MODE, DOTS, COLS_INT32, NT>, grid, WG, s, A, io, red);
}

template <int MODE, int DOTS>
static hipError_t launch_rows(const DevCsr &A, const RowIo &io, const RedArgs &red, int grid,
                              hipStream_t s)
{
    if (A.nslices > 0 && A.stream)
        return launch_sell<MODE, DOTS, true>(A, io, red, grid, s);
    if (A.nslices > 0)
        return launch_sell<MODE, DOTS, false>(A, io, red, grid, s);
    return launch(k_csr_rows<MODE, DOTS>, grid, WG, s, A, io, red);
}

hipError_t launch_spmv_dots(const DevCsr &A, const double *v, double *y, const double *w,
                            int dots, const RedArgs &red, int grid, hipStream_t s)
{
    RowIo io{v, y, w, nullptr, nullptr, nullptr};
    switch (dots) {
    case 0: return launch_rows<ROW_SPMV, 0>(A, io, red, grid, s);
    case D_YV: return launch_rows<ROW_SPMV, D_YV>(A, io, red, grid, s);
    case D_YV | D_YY: return launch_rows<ROW_SPMV, D_YV | D_YY>(A, io, red, grid, s);
    case D_YW: return launch_rows<ROW_SPMV, D_YW>(A, io, red, grid, s);
    case D_YV | D_YY | D_YW: return launch_rows<ROW_SPMV, D_YV | D_YY | D_YW>(A, io, red, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_residual0(const DevCsr &A, const double *b, const double *x, double *r,
                            double *p, double *rs, const RedArgs &red, int grid, hipStream_t s)
{
    RowIo io{x, r, b, p, rs, nullptr};
    return launch_rows<ROW_RESID, 0>(A, io, red, grid, s);
}

template <bool XAP, int COLS, bool NT>
static auto bicg2_kernel()
{
    if constexpr (XAP)
        return k_sell_bicg_xap<COLS, NT>;
    else
        return k_sell_bicg_sas<COLS, NT>;
}

template <bool XAP, bool NT>
static hipError_t launch_bicg2_sell(const DevCsr &A, const Bicg2Io &io, const RedArgs &red, int grid,
                                    hipStream_t s)
{
    if (A.dg_mask)
        return launch(bicg2_kernel<XAP, COLS_SLOTS, NT>(), grid, WG, s, A, io, red);
    if (A.sell_off4)
        return launch(bicg2_kernel<XAP, COLS_OFF16, NT>(), grid, WG, s, A, io, red);
    return launch(bicg2_kernel<XAP, COLS_INT32, NT>(), grid, WG, s, A, io, red);
}

// Workgroups of one fused step resident per compute unit (the occupancy of
// the kernel its launch would take), 0 when the query fails.
template <typename KS, typename KC>
static int fused_occupancy(const DevCsr &A, KS sell_slots, KS sell_off16, KS sell_int32, KC csr)
{
    int n = 0;
    hipError_t e;
    if (A.nslices > 0 && A.dg_mask)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sell_slots, WG, 0);
    else if (A.nslices > 0 && A.sell_off4)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sell_off16, WG, 0);
    else if (A.nslices > 0)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sell_int32, WG, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, csr, WG, 0);
    return e == hipSuccess ? n : 0;
}

int fused_per_cu(const DevCsr &A, int step)
{
    const bool nt = A.stream != 0;
    switch (step) {
    case FUSED_BICG_SAS:
        return nt ? fused_occupancy(A, k_sell_bicg_sas<COLS_SLOTS, true>, k_sell_bicg_sas<COLS_OFF16, true>,
                                    k_sell_bicg_sas<COLS_INT32, true>, k_csr_bicg_sas)
                  : fused_occupancy(A, k_sell_bicg_sas<COLS_SLOTS, false>, k_sell_bicg_sas<COLS_OFF16, false>,
                                    k_sell_bicg_sas<COLS_INT32, false>, k_csr_bicg_sas);
    case FUSED_BICG_XAP:
        return nt ? fused_occupancy(A, k_sell_bicg_xap<COLS_SLOTS, true>, k_sell_bicg_xap<COLS_OFF16, true>,
                                    k_sell_bicg_xap<COLS_INT32, true>, k_csr_bicg_xap)
                  : fused_occupancy(A, k_sell_bicg_xap<COLS_SLOTS, false>, k_sell_bicg_xap<COLS_OFF16, false>,
                                    k_sell_bicg_xap<COLS_INT32, false>, k_csr_bicg_xap);
    case FUSED_CG_XAP:
        if (A.max_width <= 5)
            return nt ? fused_occupancy(A, k_sell_cg_xap<COLS_SLOTS, true, 5>, k_sell_cg_xap<COLS_OFF16, true, 5>,
                                        k_sell_cg_xap<COLS_INT32, true, 5>, k_csr_cg_xap)
                      : fused_occupancy(A, k_sell_cg_xap<COLS_SLOTS, false, 5>, k_sell_cg_xap<COLS_OFF16, false, 5>,
                                        k_sell_cg_xap<COLS_INT32, false, 5>, k_csr_cg_xap);
        return nt ? fused_occupancy(A, k_sell_cg_xap<COLS_SLOTS, true, 7>, k_sell_cg_xap<COLS_OFF16, true, 7>,
                                    k_sell_cg_xap<COLS_INT32, true, 7>, k_csr_cg_xap)
                  : fused_occupancy(A, k_sell_cg_xap<COLS_SLOTS, false, 7>, k_sell_cg_xap<COLS_OFF16, false, 7>,
                                    k_sell_cg_xap<COLS_INT32, false, 7>, k_csr_cg_xap);
    default:
        return 0;
    }
}

template <bool NT, int UW>
static hipError_t launch_cg1_sell(const DevCsr &A, const Cg1Io &io, const RedArgs &red, int grid, hipStream_t s)
{
    if (A.dg_mask)
        return launch(k_sell_cg_xap<COLS_SLOTS, NT, UW>, grid, WG, s, A, io, red);
    if (A.sell_off4)
        return launch(k_sell_cg_xap<COLS_OFF16, NT, UW>, grid, WG, s, A, io, red);
    return launch(k_sell_cg_xap<COLS_INT32, NT, UW>, grid, WG, s, A, io, red);
}

// Measured on 2D Poisson 511^2 (5 entries per row): 5 entries per chunk
// 63,500 iterations/s against 57,500 with 7; on 3D 128^3 (7) the reverse.
hipError_t launch_cg1_xap(const DevCsr &A, const Cg1Io &io, const RedArgs &red, int grid, hipStream_t s)
{
    if (A.nslices > 0 && A.max_width <= 5)
        return A.stream ? launch_cg1_sell<true, 5>(A, io, red, grid, s) : launch_cg1_sell<false, 5>(A, io, red, grid, s);
    if (A.nslices > 0)
        return A.stream ? launch_cg1_sell<true, 7>(A, io, red, grid, s) : launch_cg1_sell<false, 7>(A, io, red, grid, s);
    return launch(k_csr_cg_xap, grid, WG, s, A, io, red);
}

hipError_t launch_bicg2_sas(const DevCsr &A, const Bicg2Io &io, const RedArgs &red, int grid, hipStream_t s)
{
    if (A.nslices > 0)
        return A.stream ? launch_bicg2_sell<false, true>(A, io, red, grid, s)
                        : launch_bicg2_sell<false, false>(A, io, red, grid, s);
    return launch(k_csr_bicg_sas, grid, WG, s, A, io, red);
}

hipError_t launch_bicg2_xap(const DevCsr &A, const Bicg2Io &io, const RedArgs &red, int grid, hipStream_t s)
{
    if (A.nslices > 0)
        return A.stream ? launch_bicg2_sell<true, true>(A, io, red, grid, s)
                        : launch_bicg2_sell<true, false>(A, io, red, grid, s);
    return launch(k_csr_bicg_xap, grid, WG, s, A, io, red);
}

hipError_t launch_gather_vals(int64_t n, double *out, const double *vals, const int32_t *map,
                              int grid, hipStream_t s)
{
    return launch(k_gather_vals, grid, WG, s, n, out, vals, map);
}

hipError_t launch_gm_scale(int64_t n, double *out, const double *in, DevState *st, uint32_t run_mask, int grid,
                           hipStream_t s)
{
    return launch(k_gm_scale, grid, WG, s, n, out, in, st, run_mask);
}

hipError_t launch_gm_multidot(int64_t n, const double *V, const double *w, int j0, int j1, double *part,
                              DevState *st, uint32_t run_mask, hipStream_t s)
{
    return launch(k_gm_multidot, GM_GRID, WG, s, n, V, w, j0, j1, part, st, run_mask);
}

hipError_t launch_gm_multidot_fin(int j0, int j1, int i, double *R, int m1, const double *part, DevState *st,
                                  uint32_t run_mask, hipStream_t s)
{
    return launch(k_gm_multidot_fin, j1 - j0, WG, s, GM_GRID, j0, i, R, m1, part, st, run_mask);
}

hipError_t launch_gm_update(int64_t n, double *w, const double *V, int i, int m1, const RedArgs &red, int grid,
                            hipStream_t s)
{
    return launch(k_gm_update, grid, WG, s, n, w, V, i, m1, red);
}

hipError_t launch_gm_normalize(int64_t n, double *v, const double *r, int i, int m1, const RedArgs &red,
                               int grid, hipStream_t s)
{
    return launch(k_gm_normalize, grid, WG, s, n, v, r, i, m1, red);
}

hipError_t launch_gm_rupdate(int64_t n, double *r, const double *v, int i, const double *R, DevState *st,
                             uint32_t run_mask, int grid, hipStream_t s)
{
    return launch(k_gm_rupdate, grid, WG, s, n, r, v, i, R, st, run_mask);
}

hipError_t launch_gm_xupdate(int64_t n, double *x, const double *V, const double *eta, int used,
                             const DevState *st, int grid, hipStream_t s)
{
    return launch(k_gm_xupdate, grid, WG, s, n, x, V, eta, used, st);
}

hipError_t launch_residual32(const DevCsr &A, const double *b, const double *x, float *r32,
                             const RedArgs &red, int grid, hipStream_t s)
{
    RowIo io{x, nullptr, b, nullptr, nullptr, r32};
    return launch_rows<ROW_RESID32, 0>(A, io, red, grid, s);
}

template <bool F32ACC, bool NT>
static hipError_t launch_sell32(const DevCsr &A, const float *vals32, const float *v, float *y,
                                const RedArgs &red, int grid, hipStream_t s)
{
    if (A.dg_mask) {
        if (A.max_width <= 5)
            return launch(k_sell_rows32<COLS_SLOTS, F32ACC, NT, 5>, grid, WG, s, A, vals32, v, y, red);
        if (A.max_width <= 7)
            return launch(k_sell_rows32<COLS_SLOTS, F32ACC, NT, 7>, grid, WG, s, A, vals32, v, y, red);
        return launch(k_sell_rows32<COLS_SLOTS, F32ACC, NT>, grid, WG, s, A, vals32, v, y, red);
    }
    if (A.sell_off4)
        return launch(k_sell_rows32<COLS_OFF16, F32ACC, NT>, grid, WG, s, A, vals32, v, y, red);
    return launch(k_sell_rows32<COLS_INT32, F32ACC, NT>, grid, WG, s, A, vals32, v, y, red);
}

template <bool F32ACC>
static hipError_t launch_spmv32_t(const DevCsr &A, const float *vals32, const float *v, float *y,
                                  const RedArgs &red, int grid, hipStream_t s)
{
    if (A.nslices > 0)
        return A.stream ? launch_sell32<F32ACC, true>(A, vals32, v, y, red, grid, s)
                        : launch_sell32<F32ACC, false>(A, vals32, v, y, red, grid, s);
    return launch(k_csr_rows32<F32ACC>, grid, WG, s, A, vals32, v, y, red);
}

hipError_t launch_spmv32(const DevCsr &A, const float *vals32, const float *v, float *y,
                         const RedArgs &red, int grid, hipStream_t s, bool f32acc)
{
    return f32acc ? launch_spmv32_t<true>(A, vals32, v, y, red, grid, s)
                  : launch_spmv32_t<false>(A, vals32, v, y, red, grid, s);
}

hipError_t launch_cg_update32(int64_t n, float *d, float *r, float *p, const float *ap,
                              const RedArgs &red, int grid, hipStream_t s, bool f32acc)
{
    if (f32acc)
        return launch(k_cg_update32<true>, grid, WG, s, n, d, r, p, ap, red);
    return launch(k_cg_update32<false>, grid, WG, s, n, d, r, p, ap, red);
}

hipError_t launch_inner_setup32(int64_t n, const float *r, float *p, float *d, const RedArgs &red,
                                int grid, hipStream_t s, bool f32acc)
{
    if (f32acc)
        return launch(k_inner_setup32<true>, grid, WG, s, n, r, p, d, red);
    return launch(k_inner_setup32<false>, grid, WG, s, n, r, p, d, red);
}

hipError_t launch_axpby(int64_t n, double alpha, const double *x, double beta, const double *y,
                        double *out, int grid, hipStream_t s)
{
    return launch(k_axpby, grid, WG, s, n, alpha, x, beta, y, out);
}

hipError_t launch_add32(int64_t n, double *x, const float *d, int grid, hipStream_t s)
{
    return launch(k_add32, grid, WG, s, n, x, d);
}

hipError_t launch_to_f32(int64_t n, float *out, const double *in, int grid, hipStream_t s)
{
    return launch(k_to_f32, grid, WG, s, n, out, in);
}

hipError_t launch_cg_update(int64_t n, double *x, double *r, double *p, const double *ap,
                            const RedArgs &red, int grid, hipStream_t s)
{
    return launch(k_cg_update, grid, WG, s, n, x, r, p, ap, red);
}

hipError_t launch_bicg_s(int64_t n, const double *r, const double *ap, double *sv,
                         const RedArgs &red, int grid, hipStream_t s)
{
    return launch(k_bicg_s, grid, WG, s, n, r, ap, sv, red);
}

hipError_t launch_bicg_xrp(int64_t n, double *x, double *r, double *p, const double *sv,
                           const double *as, const double *ap, const double *rs,
                           const RedArgs &red, int grid, hipStream_t s)
{
    return launch(k_bicg_xrp, grid, WG, s, n, x, r, p, sv, as, ap, rs, red);
}

hipError_t launch_dot(int64_t n, const double *a, const double *b, const double *c, int ndots,
                      const RedArgs &red, int grid, hipStream_t s, const double *e)
{
    if (ndots == 1)
        return launch(k_dot<1>, grid, WG, s, n, a, b, c, e, red);
    if (ndots == 2)
        return launch(k_dot<2>, grid, WG, s, n, a, b, c, e, red);
    if (ndots == 3)
        return launch(k_dot<3>, grid, WG, s, n, a, b, c, e, red);
    return hipErrorInvalidValue;
}

hipError_t launch_axpy(int64_t n, double *out, const double *y, const double *x, int which,
                       int negative, DevState *st, uint32_t run_mask, int grid, hipStream_t s)
{
    return launch(k_axpy, grid, WG, s, n, out, y, x, which, negative, st, run_mask);
}

hipError_t launch_xpay(int64_t n, double *p, const double *r, const double *v, DevState *st,
                       uint32_t run_mask, int grid, hipStream_t s)
{
    return launch(k_xpay, grid, WG, s, n, p, r, v, st, run_mask);
}

hipError_t launch_copy_fin(int64_t n, double *dst, const double *src, const RedArgs &red,
                           hipStream_t s)
{
    return launch(k_copy_fin, 1, WG, s, n, dst, src, red);
}

hipError_t launch_zero(double *x, int64_t n, DevState *st, uint32_t run_mask, int grid,
                       hipStream_t s)
{
    return launch(k_zero, grid, WG, s, x, n, st, run_mask);
}

hipError_t launch_red_init(double *partials, hipStream_t s)
{
    return launch(k_red_init, 64, WG, s, partials);
}

hipError_t launch_clear(double *x, int64_t n, int grid, hipStream_t s)
{
    return launch(k_clear, grid, WG, s, x, n);
}

hipError_t launch_state_init(DevState *st, double rtol, int32_t max_iter, int32_t hist_cap, hipStream_t s)
{
    return launch(k_state_init, 1, 64, s, st, rtol, max_iter, hist_cap);
}

size_t small_lds_bytes(int method_bicg, int64_t n)
{
    return (size_t)(method_bicg ? 2 : 1) * (size_t)n * sizeof(double);
}

size_t small_staged_lds_bytes(int method_bicg, int64_t n, int64_t nnz)
{
    return small_lds_bytes(method_bicg, n) + small_csr_bytes(n, nnz);
}

int small_rows_per_thread(int64_t n)
{
    const int64_t r = (n + SWG - 1) / SWG;
    return r <= 1 ? 1 : r <= 2 ? 2 : r <= 4 ? 4 : 0;
}

// Threads of the single-workgroup solver for n rows: the fewest of 256,
// 512 and 1024 that keep at most two rows per thread, else 1024 (up to
// four).  Every thread joins each reduction's double-double butterfly, so
// for small systems fewer, fuller waves finish an iteration sooner
// (measured on 32^2: 1024 threads 5.8 us, 512 threads 4.6 us per CG
// iteration; on 63^2, 1024 threads stay ahead).
static int small_threads(int64_t n)
{
    return n <= 512 ? 256 : n <= 1024 ? 512 : SWG;
}

template <bool STAGE, int WGS>
static hipError_t launch_small_w(int method_bicg, const DevCsr &A, const double *b, double *x,
                                 DevState *st, double *hist, double *scal, size_t shm, hipStream_t s)
{
    const int64_t r = (A.n + WGS - 1) / WGS;
    const int rpt = r <= 1 ? 1 : r <= 2 ? 2 : r <= 4 ? 4 : 0;
    switch (rpt * 2 + (method_bicg ? 1 : 0)) {
    case 2: return launch_shm(k_small_cg<1, STAGE, WGS>, 1, WGS, shm, s, A, b, x, st, hist, scal);
    case 4: return launch_shm(k_small_cg<2, STAGE, WGS>, 1, WGS, shm, s, A, b, x, st, hist, scal);
    case 3: return launch_shm(k_small_bicgstab<1, STAGE, WGS>, 1, WGS, shm, s, A, b, x, st, hist, scal);
    case 5: return launch_shm(k_small_bicgstab<2, STAGE, WGS>, 1, WGS, shm, s, A, b, x, st, hist, scal);
    default: break;
    }
    if constexpr (WGS == SWG) {
        switch (rpt * 2 + (method_bicg ? 1 : 0)) {
        case 8: return launch_shm(k_small_cg<4, STAGE, WGS>, 1, WGS, shm, s, A, b, x, st, hist, scal);
        default: break;
        }
    }
    return hipErrorInvalidValue;
}

template <bool STAGE>
static hipError_t launch_small_t(int method_bicg, const DevCsr &A, const double *b, double *x,
                                 DevState *st, double *hist, double *scal, size_t shm, hipStream_t s)
{
    switch (small_threads(A.n)) {
    case 256: return launch_small_w<STAGE, 256>(method_bicg, A, b, x, st, hist, scal, shm, s);
    case 512: return launch_small_w<STAGE, 512>(method_bicg, A, b, x, st, hist, scal, shm, s);
    default: return launch_small_w<STAGE, SWG>(method_bicg, A, b, x, st, hist, scal, shm, s);
    }
}

hipError_t launch_small(int method_bicg, const DevCsr &A, const double *b, double *x, DevState *st,
                        double *hist, double *scal, bool stage, hipStream_t s)
{
    if (stage)
        return launch_small_t<true>(method_bicg, A, b, x, st, hist, scal,
                                    small_staged_lds_bytes(method_bicg, A.n, A.nnz), s);
    return launch_small_t<false>(method_bicg, A, b, x, st, hist, scal,
                                 small_lds_bytes(method_bicg, A.n), s);
}

hipError_t launch_copy(void *dst, const void *src, int64_t n_bytes, int grid, hipStream_t s)
{
    const int64_t n16 = n_bytes / 16;
    if (n16 > 0) {
        hipError_t e = launch(k_copy16, grid, WG, s, reinterpret_cast<int4 *>(dst),
                              reinterpret_cast<const int4 *>(src), n16);
        if (e != hipSuccess)
            return e;
    }
    const int64_t tail = n_bytes - n16 * 16;
    if (tail > 0)
        return launch(k_copy_tail, 1, 64, s, reinterpret_cast<char *>(dst) + n16 * 16,
                      reinterpret_cast<const char *>(src) + n16 * 16, tail);
    return hipSuccess;
}

}  // namespace fk
