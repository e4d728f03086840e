// Batched solves: many independent SPD systems of uneven size in one
// persistent launch (the many small-to-medium systems of Section 1), each
// solved by FP64 iterative refinement around the FP32 pipelined CG of
// Algorithm 2 with the beta recurrence of Eq. (3), and the C ABI of
// include/fk.h (fk_batch_*).
//
// The batch is one block-diagonal CSR matrix; system s owns the rows
// [sys_ptr[s], sys_ptr[s+1]).  Systems are claimed from a largest-first
// order and each is solved, whole refinement included, before the claimant
// takes the next.
//  - Single workgroups: all reductions are inside the workgroup and no
//    workgroup waits for another.  A system with at most lds_rows rows keeps
//    its four FP32 work vectors in LDS; larger ones keep them in device
//    memory (the same workgroup writes and reads them between barriers).
//  - Teams (optional): `team` resident workgroups solve one system
//    together, each a contiguous chunk of its rows, and meet at team
//    barriers and all-reduces through device memory.  Teams claim from the
//    large end of the order and single workgroups from the small end, so
//    the two meet where their work balances.  The arithmetic is that of the single-system mixed
// method (FK_CG_MIXED): rows summed left to right, inner products of exact
// products in double-double rounded once, alpha and beta in FP64 rounded to
// FP32 for the updates.  One inner iteration has one reduction: the update
// of d, r, p and the product A p are separated by a barrier, and <r,r>,
// <p,Ap>, <Ap,Ap> are reduced together; the convergence test on <r,r> comes
// first, so the product computed on the last iteration is simply unused.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "fk.h"
#include "fk_dd.hpp"
#include "fk_internal.hpp"

namespace fk {
namespace batch {

enum BStatus : int32_t { B_CONVERGED = 0, B_NOT_CONVERGED = 1, B_BREAKDOWN = 2, B_UNSOLVED = 3 };

constexpr int TEAM_MAX = 64;                      // workgroups per team
constexpr int TEAM_DEFAULT = 16;                  // measured best on the 512-system batch
constexpr uint32_t TEAM_SPIN_DEFAULT = 1u << 22;  // polls of one team wait (seconds)

struct BatchArgs {
    const int32_t *sys_ptr;   // [count + 1]
    const int32_t *order;     // systems, largest first
    int32_t count;
    const int32_t *row_ptr, *col_idx;
    const double *vals;
    const float *vals32;
    const double *b;
    double *x;
    float *r32, *p32, *ap32, *d32;  // device work vectors, indexed by global row
    uint64_t *deque;  // systems claimed from the front (low word) and back (high word) of order
    int32_t *status, *iters, *sweeps;
    double *rel;
    double rtol, inner_rtol;
    int32_t max_iter;  // <= 0: 10 n_s per system
    int32_t max_outer;
    int32_t lds_rows;
    // teams: workgroups [0, team * nteams) form nteams teams of `team`
    int32_t team, nteams;
    uint32_t *team_cnt;   // [nteams][CNT_STRIDE] arrivals, counting up within a launch
    double *team_slots;   // [nteams][2][team][KMAX] double-double partials
    int32_t *team_sys;    // [nteams] the system a team is solving
    int32_t *abort_flag;  // set when a team wait runs out of patience
    uint32_t spin_limit;  // polls a team wait makes before it gives up
};

// Device-coherent accesses (agent scope) for the vectors that several
// workgroups of a team share: p of the inner solve and x.
template <typename T>
__device__ __forceinline__ T ld_coh(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_coh(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Claim the next system: from the front of `order` (largest first) or from
// its back.  One 64-bit word counts both ends, so a system is claimed once
// and the two ends stop where they meet.  -1 when none is left.  Lock-free:
// a failed exchange means another claim succeeded.
__device__ __forceinline__ int claim(const BatchArgs &a, bool front)
{
    uint64_t old = ld_coh(a.deque);
    for (;;) {
        const uint32_t f = (uint32_t)old, b = (uint32_t)(old >> 32);
        if ((int64_t)f + (int64_t)b >= (int64_t)a.count)
            return -1;
        const uint64_t want = front ? old + 1u : old + (uint64_t(1) << 32);
        if (__hip_atomic_compare_exchange_strong(a.deque, &old, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return a.order[front ? (int)f : a.count - 1 - (int)b];
    }
}

// A workgroup's place in its team; `epoch` counts the team's meetings.
struct Team {
    int t, j, T;
    uint32_t epoch;
};

// Thread 0: arrive at the team's counter for this epoch and wait until all
// T members have.  The wait is bounded: after spin_limit polls, or when
// another wait has already given up, it sets the abort flag and returns
// false.  The caller's stores must be complete (s_waitcnt) before it.
__device__ bool team_arrive_wait(const BatchArgs &a, const Team &tm)
{
    uint32_t *cnt = a.team_cnt + (size_t)tm.t * CNT_STRIDE;
    __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t target = (uint32_t)tm.T * (tm.epoch + 1u);
    for (uint32_t polls = 0;; ++polls) {
        if (ld_coh(cnt) >= target)
            return true;
        if (polls >= a.spin_limit || ((polls & 15u) == 15u && ld_coh(a.abort_flag) != 0)) {
            st_coh(a.abort_flag, 1);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// The team's double-double partials of one meeting: member jj's slot.
__device__ __forceinline__ double *team_slot(const BatchArgs &a, const Team &tm, int jj)
{
    return a.team_slots + (((size_t)tm.t * 2 + (tm.epoch & 1u)) * tm.T + jj) * (2 * KMAX);
}

// Team barrier: every member's earlier stores are visible to every member
// after it.  false if the team gave up.
__device__ bool team_barrier(const BatchArgs &a, Team &tm, double *bcast)
{
    __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have completed
    __syncthreads();
    if (threadIdx.x == 0)
        bcast[0] = team_arrive_wait(a, tm) ? 1.0 : 0.0;
    __syncthreads();
    const bool ok = bcast[0] != 0.0;
    __syncthreads();
    tm.epoch++;
    return ok;
}

// Team all-reduce of K double-double values: each member sums its
// workgroup (waves in order), publishes the sum, meets the others, and adds
// the T sums in member order, so every member gets the same rounded totals.
// After the barrier wave 0 alone finishes: its lanes add the wave sums and
// later the T members' sums, which lanes 0 .. T-1 fetch at once, by
// butterflies (a fixed order, so every member rounds the same totals);
// lane 0 publishes and waits in between.  It is also a team barrier.
// false if the team gave up.
template <int K, int NW>
__device__ bool team_reduce(const BatchArgs &a, Team &tm, dd (&v)[K], double (&out)[K], dd (*lds)[NW],
                            double *bcast)
{
    static_assert(K < 4 && K <= KMAX, "broadcast words");
    __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have completed
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k)
        v[k] = wave_reduce(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            lds[k][wave] = v[k];
    }
    __syncthreads();
    if (wave == 0) {
        dd w[K];
#pragma unroll
        for (int k = 0; k < K; ++k)
            w[k] = lanes_sum(lane < NW ? lds[k][lane] : dd{0.0, 0.0}, NW);
        int ok = 1;
        if (lane == 0) {
            double *mine = team_slot(a, tm, tm.j);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                st_coh(mine + 2 * k, w[k].hi);
                st_coh(mine + 2 * k + 1, w[k].lo);
            }
            __builtin_amdgcn_s_waitcnt(0);
            ok = team_arrive_wait(a, tm) ? 1 : 0;
        }
        ok = __builtin_amdgcn_readfirstlane(ok);
        if (ok) {
            dd m[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                m[k] = dd{0.0, 0.0};
                if (lane < tm.T) {
                    const double *o = team_slot(a, tm, lane);
                    m[k] = dd{ld_coh(o + 2 * k), ld_coh(o + 2 * k + 1)};
                }
            }
            int width = 1;
            while (width < tm.T)
                width <<= 1;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const dd sum = lanes_sum(m[k], width);
                if (lane == 0)
                    bcast[k] = sum.hi + sum.lo;
            }
        }
        if (lane == 0)
            bcast[3] = ok ? 1.0 : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k)
        out[k] = bcast[k];
    const bool ok = bcast[3] != 0.0;
    __syncthreads();
    tm.epoch++;
    return ok;
}

// Sum K double-double values over the workgroup and return the rounded
// totals to every thread (wave order, then a fixed tree: reproducible).
template <int K, int NW>
__device__ __forceinline__ void wg_reduce(dd (&v)[K], double (&out)[K], dd (*lds)[NW], double *bcast)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k)
        v[k] = wave_reduce(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            lds[k][wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < K) {
        dd a = lds[threadIdx.x][0];
        for (int w = 1; w < NW; ++w)
            a = dd_add(a, lds[threadIdx.x][w]);
        bcast[threadIdx.x] = a.hi + a.lo;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k)
        out[k] = bcast[k];
    __syncthreads();
}

// One CSR row summed left to right, with the column indices and values of
// up to RB nonzeros requested together and their gathers next, so a thread
// has many loads in flight instead of a dependent chain per nonzero.
constexpr int RB = 8;

template <typename T, typename V, bool COH = false>
__device__ __forceinline__ T row_sum(const int32_t *__restrict__ col, const T *__restrict__ vals,
                                     const V *__restrict__ x, int j0, int j1, int shift)
{
    T q = T(0);
    for (int j = j0; j < j1; j += RB) {
        int c[RB];
        T v[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k)
            if (j + k < j1) {
                c[k] = col[j + k] - shift;
                v[k] = vals[j + k];
            }
        T g[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k)
            if (j + k < j1)
                g[k] = (T)(COH ? ld_coh(x + c[k]) : x[c[k]]);
#pragma unroll
        for (int k = 0; k < RB; ++k)
            if (j + k < j1)
                q = q + v[k] * g[k];
    }
    return q;
}

// Two rows summed left to right at once (each in its own order, as
// row_sum): up to RB2 indices and values of each, then their gathers, are
// requested together, so a thread has more loads in flight.  (With 1024
// threads this spills a few registers; measured, the wider requests still
// win: 868 -> 704 us per inner iteration of a 512^2 system alone.)
constexpr int RB2 = 6;
template <typename T, typename V, bool COH>
__device__ __forceinline__ void row_sum2(const int32_t *__restrict__ col, const T *__restrict__ vals,
                                         const V *__restrict__ x, int a0, int a1, int b0, int b1, int shift,
                                         T &qa, T &qb)
{
    qa = T(0);
    qb = T(0);
    const int la = a1 - a0, lb = b1 - b0;
    const int len = la > lb ? la : lb;
    for (int j = 0; j < len; j += RB2) {
        int ca[RB2], cb[RB2];
        T va[RB2], vb[RB2];
#pragma unroll
        for (int k = 0; k < RB2; ++k) {
            if (j + k < la) {
                ca[k] = col[a0 + j + k] - shift;
                va[k] = vals[a0 + j + k];
            }
            if (j + k < lb) {
                cb[k] = col[b0 + j + k] - shift;
                vb[k] = vals[b0 + j + k];
            }
        }
        T ga[RB2], gb[RB2];
#pragma unroll
        for (int k = 0; k < RB2; ++k) {
            if (j + k < la)
                ga[k] = (T)(COH ? ld_coh(x + ca[k]) : x[ca[k]]);
            if (j + k < lb)
                gb[k] = (T)(COH ? ld_coh(x + cb[k]) : x[cb[k]]);
        }
#pragma unroll
        for (int k = 0; k < RB2; ++k) {
            if (j + k < la)
                qa = qa + va[k] * ga[k];
            if (j + k < lb)
                qb = qb + vb[k] * gb[k];
        }
    }
}

template <bool COH>
__device__ __forceinline__ float ldp(const float *p)
{
    return COH ? ld_coh(p) : *p;
}

template <bool COH>
__device__ __forceinline__ void stp(float *p, float v)
{
    if constexpr (COH)
        st_coh(p, v);
    else
        *p = v;
}

// The inner update d += alpha p, r -= alpha Ap, p = r + beta p over one
// thread's rows i0, i0 + WGS, ... < i1, two rows per step with their loads
// together; <r,r> accumulates in row order.  COH: p is shared by a team.
template <int WGS, bool COH>
__device__ __forceinline__ void inner_update(float *R, float *P, const float *AP, float *D, int i0, int i1,
                                             float af, float bf, dd &rr)
{
    int i = i0;
    for (; i + WGS < i1; i += 2 * WGS) {
        const int i2 = i + WGS;
        const float pa = ldp<COH>(P + i), pb = ldp<COH>(P + i2);
        const float da = D[i], db = D[i2];
        const float ra = R[i], rb = R[i2];
        const float ya = AP[i], yb = AP[i2];
        D[i] = da + af * pa;
        D[i2] = db + af * pb;
        const float sa = ra - af * ya, sb = rb - af * yb;
        R[i] = sa;
        R[i2] = sb;
        stp<COH>(P + i, sa + bf * pa);
        stp<COH>(P + i2, sb + bf * pb);
        dd_fma(rr, (double)sa, (double)sa);
        dd_fma(rr, (double)sb, (double)sb);
    }
    if (i < i1) {
        const float pi = ldp<COH>(P + i);
        D[i] = D[i] + af * pi;
        const float ri = R[i] - af * AP[i];
        R[i] = ri;
        stp<COH>(P + i, ri + bf * pi);
        dd_fma(rr, (double)ri, (double)ri);
    }
}

// The inner product Ap over one thread's rows (two per step, as above) with
// <p,Ap> and <Ap,Ap> accumulated in row order.
template <int WGS, bool COH>
__device__ __forceinline__ void inner_product(const BatchArgs &a, int r0, const float *P, float *AP, int i0,
                                              int i1, dd &pap, dd &apap)
{
    int i = i0;
    for (; i + WGS < i1; i += 2 * WGS) {
        const int i2 = i + WGS;
        float qa, qb;
        row_sum2<float, float, COH>(a.col_idx, a.vals32, P, a.row_ptr[r0 + i], a.row_ptr[r0 + i + 1],
                                    a.row_ptr[r0 + i2], a.row_ptr[r0 + i2 + 1], r0, qa, qb);
        AP[i] = qa;
        AP[i2] = qb;
        dd_fma(pap, (double)qa, (double)ldp<COH>(P + i));
        dd_fma(apap, (double)qa, (double)qa);
        dd_fma(pap, (double)qb, (double)ldp<COH>(P + i2));
        dd_fma(apap, (double)qb, (double)qb);
    }
    if (i < i1) {
        const float q = row_sum<float, float, COH>(a.col_idx, a.vals32, P, a.row_ptr[r0 + i],
                                                   a.row_ptr[r0 + i + 1], r0);
        AP[i] = q;
        dd_fma(pap, (double)q, (double)ldp<COH>(P + i));
        dd_fma(apap, (double)q, (double)q);
    }
}

// One system of the batch, solved by the whole workgroup.  IN_LDS: its four
// FP32 work vectors live in the workgroup's LDS (n <= lds_rows), else in
// global memory.
template <int WGS, bool IN_LDS>
__device__ __forceinline__ void solve_one(const BatchArgs &a, int s, float *vlds, dd (*red)[WGS / 64],
                                          double *bcast)
{
    constexpr int NW = WGS / 64;
    const int tid = threadIdx.x;
    const int r0 = a.sys_ptr[s];
    const int n = a.sys_ptr[s + 1] - r0;
    // IN_LDS is a compile-time choice, so each vector has one address
    // space and compiles to ds_* or global_* accesses (not flat).
    float *R = IN_LDS ? vlds : a.r32 + r0;
    float *P = IN_LDS ? vlds + a.lds_rows : a.p32 + r0;
    float *AP = IN_LDS ? vlds + 2 * a.lds_rows : a.ap32 + r0;
    float *D = IN_LDS ? vlds + 3 * a.lds_rows : a.d32 + r0;
    const int64_t max_iter = a.max_iter > 0 ? a.max_iter : 10 * (int64_t)n;
    int64_t used = 0;
    int32_t sweeps = 0, st = B_NOT_CONVERGED;
    double bnorm = 0.0, tol = 0.0, rel = 0.0;
    for (;;) {
        // r_j = b - A x_j (FP64, rows left to right); r32 = (float) r_j
        dd acc[2] = {dd{0.0, 0.0}, dd{0.0, 0.0}};
        for (int i = tid; i < n; i += WGS) {
            const int gi = r0 + i;
            const double q = row_sum<double, double>(a.col_idx, a.vals, a.x, a.row_ptr[gi],
                                                     a.row_ptr[gi + 1], 0);
            const double ri = a.b[gi] - q;
            R[i] = (float)ri;
            dd_fma(acc[0], ri, ri);
            if (sweeps == 0)
                dd_fma(acc[1], a.b[gi], a.b[gi]);
        }
        double rr[2];
        wg_reduce<2, NW>(acc, rr, red, bcast);
        if (sweeps == 0) {
            if (rr[1] == 0.0) {  // b = 0: x = 0
                for (int i = tid; i < n; i += WGS)
                    a.x[r0 + i] = 0.0;
                st = B_CONVERGED;
                rel = 0.0;
                break;
            }
            bnorm = sqrt(rr[1]);
            tol = a.rtol * bnorm;
        }
        rel = sqrt(rr[0]) / bnorm;
        if (!isfinite(rr[0])) {
            st = B_BREAKDOWN;
            break;
        }
        if (sqrt(rr[0]) <= tol) {
            st = B_CONVERGED;
            break;
        }
        if (sweeps >= a.max_outer || used >= max_iter) {
            st = B_NOT_CONVERGED;
            break;
        }
        // Inner solve A d = r32, d_0 = 0, by FP32 pipelined CG.
        const int64_t cap = max_iter - used;
        dd ai[1] = {dd{0.0, 0.0}};
        for (int i = tid; i < n; i += WGS) {
            const float ri = R[i];
            P[i] = ri;
            D[i] = 0.f;
            dd_fma(ai[0], (double)ri, (double)ri);
        }
        double rri[1];
        wg_reduce<1, NW>(ai, rri, red, bcast);
        double rrin = rri[0];
        int64_t k = 0;
        int ist = B_NOT_CONVERGED;
        const double tol_in = a.inner_rtol * sqrt(rrin);
        if (rrin == 0.0 || (isfinite(rrin) && sqrt(rrin) <= tol_in)) {
            ist = B_CONVERGED;  // no step
        } else if (!isfinite(rrin)) {
            ist = B_BREAKDOWN;
        } else {
            double alpha = 0.0, beta = 0.0;
            bool first = true;
            for (int64_t it = 0;; ++it) {
                // it == 0: product only; it >= 1: update, then product.
                dd acc3[3] = {dd{0.0, 0.0}, dd{0.0, 0.0}, dd{0.0, 0.0}};
                if (!first) {
                    inner_update<WGS, false>(R, P, AP, D, tid, n, (float)alpha, (float)beta, acc3[0]);
                    __syncthreads();  // p complete before the product
                }
                inner_product<WGS, false>(a, r0, P, AP, tid, n, acc3[1], acc3[2]);
                double d3[3];
                wg_reduce<3, NW>(acc3, d3, red, bcast);
                if (!first) {
                    rrin = d3[0];
                    k = it;
                    if (!isfinite(rrin)) {
                        ist = B_BREAKDOWN;
                        break;
                    }
                    if (sqrt(rrin) <= tol_in) {
                        ist = B_CONVERGED;
                        break;
                    }
                    if (it == cap)
                        break;
                }
                const double pap = d3[1], apap = d3[2];
                if (!(pap > 0.0) || !isfinite(pap) || !isfinite(apap)) {
                    ist = B_BREAKDOWN;
                    break;
                }
                alpha = rrin / pap;
                beta = alpha * alpha * apap / rrin - 1.0;  // Eq. (3)
                first = false;
            }
        }
        used += k;
        if (ist == B_BREAKDOWN) {
            st = B_BREAKDOWN;
            break;
        }
        if (k == 0) {
            st = B_NOT_CONVERGED;
            break;
        }
        for (int i = tid; i < n; i += WGS)
            a.x[r0 + i] = a.x[r0 + i] + (double)D[i];
        sweeps++;
        __syncthreads();  // x complete before the next residual
    }
    if (tid == 0) {
        a.status[s] = st;
        a.iters[s] = (int32_t)used;
        a.sweeps[s] = sweeps;
        a.rel[s] = rel;
    }
}

// One system solved by a team: the steps, arithmetic and decisions of
// solve_one, with member j taking rows [j c, (j+1) c) of the system
// (c = ceil(n / T)) and every workgroup reduction replaced by a team
// all-reduce.  p and x are read and written through device-coherent
// accesses (other members gather them); r, Ap and d are only ever touched by
// the member that owns the row.  Every member takes every decision on the
// same reduced values, so all meet the same number of times.  false: the
// team gave up waiting (the system keeps status B_UNSOLVED).
template <int WGS>
__device__ bool solve_team(const BatchArgs &a, int s, Team &tm, dd (*red)[WGS / 64], double *bcast)
{
    constexpr int NW = WGS / 64;
    const int tid = threadIdx.x;
    const int r0 = a.sys_ptr[s];
    const int n = a.sys_ptr[s + 1] - r0;
    const int chunk = (n + tm.T - 1) / tm.T;
    const int lo = min(n, tm.j * chunk), hi = min(n, lo + chunk);
    float *R = a.r32 + r0, *P = a.p32 + r0, *AP = a.ap32 + r0, *D = a.d32 + r0;
    double *X = a.x + r0;
    const int64_t max_iter = a.max_iter > 0 ? a.max_iter : 10 * (int64_t)n;
    int64_t used = 0;
    int32_t sweeps = 0, st = B_NOT_CONVERGED;
    double bnorm = 0.0, tol = 0.0, rel = 0.0;
    for (;;) {
        // r_j = b - A x_j (FP64, rows left to right); r32 = (float) r_j
        dd acc[2] = {dd{0.0, 0.0}, dd{0.0, 0.0}};
        for (int i = lo + tid; i < hi; i += WGS) {
            const int gi = r0 + i;
            const double q = row_sum<double, double, true>(a.col_idx, a.vals, a.x, a.row_ptr[gi],
                                                           a.row_ptr[gi + 1], 0);
            const double ri = a.b[gi] - q;
            R[i] = (float)ri;
            dd_fma(acc[0], ri, ri);
            if (sweeps == 0)
                dd_fma(acc[1], a.b[gi], a.b[gi]);
        }
        double rr[2];
        if (!team_reduce<2, NW>(a, tm, acc, rr, red, bcast))
            return false;
        if (sweeps == 0) {
            if (rr[1] == 0.0) {  // b = 0: x = 0
                for (int i = lo + tid; i < hi; i += WGS)
                    st_coh(X + i, 0.0);
                st = B_CONVERGED;
                rel = 0.0;
                break;
            }
            bnorm = sqrt(rr[1]);
            tol = a.rtol * bnorm;
        }
        rel = sqrt(rr[0]) / bnorm;
        if (!isfinite(rr[0])) {
            st = B_BREAKDOWN;
            break;
        }
        if (sqrt(rr[0]) <= tol) {
            st = B_CONVERGED;
            break;
        }
        if (sweeps >= a.max_outer || used >= max_iter) {
            st = B_NOT_CONVERGED;
            break;
        }
        // Inner solve A d = r32, d_0 = 0, by FP32 pipelined CG.
        const int64_t cap = max_iter - used;
        dd ai[1] = {dd{0.0, 0.0}};
        for (int i = lo + tid; i < hi; i += WGS) {
            const float ri = R[i];
            st_coh(P + i, ri);
            D[i] = 0.f;
            dd_fma(ai[0], (double)ri, (double)ri);
        }
        double rri[1];
        if (!team_reduce<1, NW>(a, tm, ai, rri, red, bcast))  // also: p complete
            return false;
        double rrin = rri[0];
        int64_t k = 0;
        int ist = B_NOT_CONVERGED;
        const double tol_in = a.inner_rtol * sqrt(rrin);
        if (rrin == 0.0 || (isfinite(rrin) && sqrt(rrin) <= tol_in)) {
            ist = B_CONVERGED;  // no step
        } else if (!isfinite(rrin)) {
            ist = B_BREAKDOWN;
        } else {
            double alpha = 0.0, beta = 0.0;
            bool first = true;
            for (int64_t it = 0;; ++it) {
                // it == 0: product only; it >= 1: update, then product.
                dd acc3[3] = {dd{0.0, 0.0}, dd{0.0, 0.0}, dd{0.0, 0.0}};
                if (!first) {
                    inner_update<WGS, true>(R, P, AP, D, lo + tid, hi, (float)alpha, (float)beta, acc3[0]);
                    if (!team_barrier(a, tm, bcast))  // p complete before the product
                        return false;
                }
                inner_product<WGS, true>(a, r0, P, AP, lo + tid, hi, acc3[1], acc3[2]);
                double d3[3];
                if (!team_reduce<3, NW>(a, tm, acc3, d3, red, bcast))
                    return false;
                if (!first) {
                    rrin = d3[0];
                    k = it;
                    if (!isfinite(rrin)) {
                        ist = B_BREAKDOWN;
                        break;
                    }
                    if (sqrt(rrin) <= tol_in) {
                        ist = B_CONVERGED;
                        break;
                    }
                    if (it == cap)
                        break;
                }
                const double pap = d3[1], apap = d3[2];
                if (!(pap > 0.0) || !isfinite(pap) || !isfinite(apap)) {
                    ist = B_BREAKDOWN;
                    break;
                }
                alpha = rrin / pap;
                beta = alpha * alpha * apap / rrin - 1.0;  // Eq. (3)
                first = false;
            }
        }
        used += k;
        if (ist == B_BREAKDOWN) {
            st = B_BREAKDOWN;
            break;
        }
        if (k == 0) {
            st = B_NOT_CONVERGED;
            break;
        }
        for (int i = lo + tid; i < hi; i += WGS)
            st_coh(X + i, ld_coh(X + i) + (double)D[i]);
        sweeps++;
        if (!team_barrier(a, tm, bcast))  // x complete before the next residual
            return false;
    }
    if (tm.j == 0 && tid == 0) {
        a.status[s] = st;
        a.iters[s] = (int32_t)used;
        a.sweeps[s] = sweeps;
        a.rel[s] = rel;
    }
    return true;
}

// A single workgroup's life: claim a system, solve it alone (in LDS when
// it fits), claim again.  `first`, if not negative, is a system already
// claimed.
template <int WGS>
__device__ void single_loop(const BatchArgs &a, bool front, int first, float *vlds, dd (*red)[WGS / 64],
                            double *bcast, int32_t *s_sys)
{
    for (int s = first;;) {
        if (s < 0) {
            if (threadIdx.x == 0)
                *s_sys = claim(a, front);
            __syncthreads();
            s = *s_sys;
            __syncthreads();
            if (s < 0)
                return;
        }
        const int n = a.sys_ptr[s + 1] - a.sys_ptr[s];
        if (n <= a.lds_rows)
            solve_one<WGS, true>(a, s, vlds, red, bcast);
        else
            solve_one<WGS, false>(a, s, vlds, red, bcast);
        __syncthreads();
        s = -1;
    }
}

// A team's life: its first member claims the largest remaining system and
// announces it at a team barrier; the team solves it and claims again.  A
// system that fits one workgroup's LDS is not worth a team, and none after
// it is larger: the team then dissolves, its first member solves that
// system alone and every member goes on as a single workgroup.
template <int WGS>
__device__ void team_loop(const BatchArgs &a, Team tm, float *vlds, dd (*red)[WGS / 64], double *bcast,
                          int32_t *s_sys)
{
    for (;;) {
        if (threadIdx.x == 0 && tm.j == 0)
            st_coh(a.team_sys + tm.t, claim(a, true));
        if (!team_barrier(a, tm, bcast))
            return;
        if (threadIdx.x == 0)
            *s_sys = ld_coh(a.team_sys + tm.t);
        __syncthreads();
        const int s = *s_sys;
        __syncthreads();
        if (s < 0)
            return;
        if (a.sys_ptr[s + 1] - a.sys_ptr[s] <= a.lds_rows) {
            single_loop<WGS>(a, true, tm.j == 0 ? s : -1, vlds, red, bcast, s_sys);
            return;
        }
        if (!solve_team<WGS>(a, s, tm, red, bcast))
            return;
    }
}

template <int WGS>
__global__ __launch_bounds__(WGS) void k_batch_mixed(BatchArgs a)
{
    constexpr int NW = WGS / 64;
    extern __shared__ __align__(16) float vlds[];  // 4 * lds_rows floats
    __shared__ dd red[3][NW];
    __shared__ double bcast[4];
    __shared__ int32_t s_sys;
    if ((int)blockIdx.x < a.team * a.nteams) {
        team_loop<WGS>(a, Team{(int)blockIdx.x / a.team, (int)blockIdx.x % a.team, a.team, 0u}, vlds, red,
                       bcast, &s_sys);
        return;
    }
    // Single workgroups: largest first, or smallest first beside teams.
    single_loop<WGS>(a, a.nteams == 0, -1, vlds, red, bcast, &s_sys);
}

// Before each launch: both claim counts, the team counters and the abort
// flag to zero, every status to B_UNSOLVED (a kernel, so that a captured
// graph holds no memset node).
__global__ __launch_bounds__(256) void k_batch_reset(BatchArgs a)
{
    const int i = (int)(blockIdx.x * 256 + threadIdx.x);
    if (i == 0) {
        *a.deque = 0;
        *a.abort_flag = 0;
    }
    if (i < a.nteams)
        a.team_cnt[(size_t)i * CNT_STRIDE] = 0u;
    for (int s = i; s < a.count; s += (int)(gridDim.x * 256))
        a.status[s] = B_UNSOLVED;
}

__global__ __launch_bounds__(256) void k_to_f32_batch(int64_t n, float *out, const double *in)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = (float)in[i];
}

}  // namespace batch
}  // namespace fk

// =================================================================== host

using namespace fk;
using namespace fk::batch;

struct fk_batch_s {
    int32_t count = 0;
    int64_t n = 0, nnz = 0;
    int device = 0;
    int32_t *sys_ptr = nullptr, *order = nullptr, *row_ptr = nullptr, *col_idx = nullptr;
    double *vals = nullptr;
    float *vals32 = nullptr, *r32 = nullptr, *p32 = nullptr, *ap32 = nullptr, *d32 = nullptr;
    uint64_t *deque = nullptr;
    int32_t *status = nullptr, *iters = nullptr, *sweeps = nullptr;
    double *rel = nullptr;
    int32_t max_rows = 0;
    // team scratch, grown on demand: counters, partial slots, announced
    // systems for up to team_cap_n teams of up to team_cap_t members
    uint32_t *team_cnt = nullptr;
    double *team_slots = nullptr;
    int32_t *team_sys = nullptr, *abort_flag = nullptr;
    int team_cap_n = 0, team_cap_t = 0;
    bool solved = false;
    // graph of the last launch configuration
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    BatchArgs gargs{};
    int gwgs = 0;
    size_t glds = 0;
    int ggrid = 0;
};

namespace {

template <typename T>
void dfree(T *&p)
{
    if (p)
        (void)hipFree(p);
    p = nullptr;
}

template <typename T>
hipError_t dalloc(T **p, size_t count)
{
    return hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(count, 1) * sizeof(T));
}

void release(fk_batch B)
{
    dfree(B->sys_ptr);
    dfree(B->order);
    dfree(B->row_ptr);
    dfree(B->col_idx);
    dfree(B->vals);
    dfree(B->vals32);
    dfree(B->r32);
    dfree(B->p32);
    dfree(B->ap32);
    dfree(B->d32);
    dfree(B->deque);
    dfree(B->team_cnt);
    dfree(B->team_slots);
    dfree(B->team_sys);
    dfree(B->abort_flag);
    B->team_cap_n = B->team_cap_t = 0;
    dfree(B->status);
    dfree(B->iters);
    dfree(B->sweeps);
    dfree(B->rel);
    if (B->exec)
        (void)hipGraphExecDestroy(B->exec);
    if (B->graph)
        (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
}

// Resident workgroups of the batch kernel per CU (registers, LDS, waves).
hipError_t occupancy(int wgs, size_t lds, int *per_cu)
{
    switch (wgs) {
    case 256:
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch_mixed<256>, 256, lds);
    case 512:
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch_mixed<512>, 512, lds);
    default:
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch_mixed<1024>, 1024, lds);
    }
}

hipError_t launch(const BatchArgs &a, int wgs, int grid, size_t lds, hipStream_t s)
{
    const int rgrid = std::max(1, std::min(64, (std::max(a.count, a.nteams) + 255) / 256));
    hipLaunchKernelGGL(k_batch_reset, dim3(rgrid), dim3(256), 0, s, a);
    switch (wgs) {
    case 256:
        hipLaunchKernelGGL(k_batch_mixed<256>, dim3(grid), dim3(256), lds, s, a);
        break;
    case 512:
        hipLaunchKernelGGL(k_batch_mixed<512>, dim3(grid), dim3(512), lds, s, a);
        break;
    default:
        hipLaunchKernelGGL(k_batch_mixed<1024>, dim3(grid), dim3(1024), lds, s, a);
        break;
    }
    return hipGetLastError();
}

}  // namespace

extern "C" fk_status fk_batch_create(int32_t count, const int64_t *sys_ptr, int64_t nnz, const int32_t *row_ptr,
                                     const int32_t *col_idx, const double *vals, int32_t ptr_kind,
                                     void *hip_stream, fk_batch *out)
{
    if (!out)
        return internal_fail(FK_E_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || !sys_ptr)
        return internal_fail(FK_E_ARG, "count must be >= 1 and sys_ptr given");
    if (sys_ptr[0] != 0)
        return internal_fail(FK_E_CSR, "sys_ptr[0] = %lld, expected 0", (long long)sys_ptr[0]);
    for (int32_t s = 0; s < count; ++s)
        if (sys_ptr[s + 1] <= sys_ptr[s])
            return internal_fail(FK_E_CSR, "system %d is empty or sys_ptr decreases", s);
    const int64_t n = sys_ptr[count];
    if (n >= INT32_MAX || nnz < 0 || nnz > INT32_MAX)
        return internal_fail(FK_E_ARG, "n = %lld or nnz = %lld out of range", (long long)n, (long long)nnz);
    if (!row_ptr || (nnz > 0 && (!col_idx || !vals)))
        return internal_fail(FK_E_ARG, "NULL CSR array");
    if (ptr_kind != FK_PTR_HOST && ptr_kind != FK_PTR_DEVICE)
        return internal_fail(FK_E_ARG, "ptr_kind = %d", ptr_kind);
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<int32_t> h_rp, h_ci;
    const int32_t *rp = row_ptr, *ci = col_idx;
    try {
        if (ptr_kind == FK_PTR_DEVICE) {
            h_rp.resize((size_t)n + 1);
            h_ci.resize((size_t)std::max<int64_t>(nnz, 1));
            if (hipMemcpy(h_rp.data(), row_ptr, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost) != hipSuccess ||
                (nnz > 0 && hipMemcpy(h_ci.data(), col_idx, (size_t)nnz * 4, hipMemcpyDeviceToHost) != hipSuccess))
                return internal_fail(FK_E_HIP, "copying the CSR arrays back failed");
            rp = h_rp.data();
            ci = h_ci.data();
        }
    } catch (const std::bad_alloc &) {
        return internal_fail(FK_E_OOM, "host allocation failed");
    }
    // CSR conventions, and every row of system s referencing only system s.
    if (rp[0] != 0 || (int64_t)rp[n] != nnz)
        return internal_fail(FK_E_CSR, "row_ptr[0] must be 0 and row_ptr[n] = nnz");
    int32_t max_rows = 0;
    std::vector<int64_t> sys_nnz((size_t)count);
    for (int32_t s = 0; s < count; ++s) {
        const int64_t lo = sys_ptr[s], hi = sys_ptr[s + 1];
        max_rows = std::max<int32_t>(max_rows, (int32_t)(hi - lo));
        for (int64_t i = lo; i < hi; ++i) {
            if (rp[i + 1] < rp[i])
                return internal_fail(FK_E_CSR, "row_ptr decreases at row %lld", (long long)i);
            for (int64_t j = rp[i]; j < rp[i + 1]; ++j)
                if (ci[j] < lo || ci[j] >= hi)
                    return internal_fail(FK_E_CSR, "row %lld of system %d references column %d outside it",
                                         (long long)i, s, ci[j]);
        }
        sys_nnz[(size_t)s] = rp[hi] - rp[lo];
    }
    // Largest systems first (ties by index), so the longest solves start early.
    std::vector<int32_t> order((size_t)count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return sys_nnz[(size_t)x] > sys_nnz[(size_t)y]; });
    std::vector<int32_t> sp32((size_t)count + 1);
    for (int32_t s = 0; s <= count; ++s)
        sp32[(size_t)s] = (int32_t)sys_ptr[s];

    fk_batch B = new (std::nothrow) fk_batch_s;
    if (!B)
        return internal_fail(FK_E_OOM, "host allocation failed");
    B->count = count;
    B->n = n;
    B->nnz = nnz;
    B->max_rows = max_rows;
    (void)hipGetDevice(&B->device);
    const hipMemcpyKind kind = ptr_kind == FK_PTR_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipError_t e = dalloc(&B->sys_ptr, (size_t)count + 1);
    e = e ? e : dalloc(&B->order, (size_t)count);
    e = e ? e : dalloc(&B->row_ptr, (size_t)n + 1);
    e = e ? e : dalloc(&B->col_idx, (size_t)nnz);
    e = e ? e : dalloc(&B->vals, (size_t)nnz);
    e = e ? e : dalloc(&B->vals32, (size_t)nnz);
    e = e ? e : dalloc(&B->r32, (size_t)n);
    e = e ? e : dalloc(&B->p32, (size_t)n);
    e = e ? e : dalloc(&B->ap32, (size_t)n);
    e = e ? e : dalloc(&B->d32, (size_t)n);
    e = e ? e : dalloc(&B->deque, 1);
    e = e ? e : dalloc(&B->abort_flag, 1);
    e = e ? e : dalloc(&B->status, (size_t)count);
    e = e ? e : dalloc(&B->iters, (size_t)count);
    e = e ? e : dalloc(&B->sweeps, (size_t)count);
    e = e ? e : dalloc(&B->rel, (size_t)count);
    e = e ? e : hipMemcpyAsync(B->sys_ptr, sp32.data(), sp32.size() * 4, hipMemcpyHostToDevice, st);
    e = e ? e : hipMemcpyAsync(B->order, order.data(), order.size() * 4, hipMemcpyHostToDevice, st);
    e = e ? e : hipMemcpyAsync(B->row_ptr, row_ptr, (size_t)(n + 1) * 4, kind, st);
    if (nnz > 0) {
        e = e ? e : hipMemcpyAsync(B->col_idx, col_idx, (size_t)nnz * 4, kind, st);
        e = e ? e : hipMemcpyAsync(B->vals, vals, (size_t)nnz * 8, kind, st);
    }
    if (e == hipSuccess && nnz > 0)
        hipLaunchKernelGGL(k_to_f32_batch, dim3(2048), dim3(256), 0, st, nnz, B->vals32, B->vals);
    e = e ? e : hipGetLastError();
    e = e ? e : hipStreamSynchronize(st);
    if (e != hipSuccess) {
        release(B);
        delete B;
        return e == hipErrorOutOfMemory ? internal_fail(FK_E_OOM, "batch: out of device memory")
                                        : internal_fail(FK_E_HIP, "fk_batch_create: %s", hipGetErrorString(e));
    }
    *out = B;
    return FK_OK;
}

extern "C" fk_status fk_batch_destroy(fk_batch B)
{
    if (!B)
        return internal_fail(FK_E_ARG, "NULL batch");
    (void)hipDeviceSynchronize();
    release(B);
    delete B;
    return FK_OK;
}

extern "C" fk_status fk_batch_solve(fk_batch B, const fk_batch_opts *o, const double *b, double *x,
                                    void *hip_stream)
{
    if (!B || !o || !b || !x)
        return internal_fail(FK_E_ARG, "NULL argument");
    if (!(o->rtol >= 0.0) || !std::isfinite(o->rtol) || !(o->inner_rtol >= 0.0) || !std::isfinite(o->inner_rtol))
        return internal_fail(FK_E_ARG, "rtol and inner_rtol must be finite and >= 0");
    if (o->max_iter < 0 || o->max_outer < 0)
        return internal_fail(FK_E_ARG, "max_iter and max_outer must be >= 0");
    const int wgs = o->workgroup == 0 ? 1024 : o->workgroup;
    if (wgs != 256 && wgs != 512 && wgs != 1024)
        return internal_fail(FK_E_ARG, "workgroup must be 0, 256, 512 or 1024");
    if (o->flags & ~FK_FLAG_GRAPH)
        return internal_fail(FK_E_ARG, "unknown flags 0x%x", o->flags);
    if (o->team < 0 || o->team > TEAM_MAX || o->teams < 0 || o->spin_limit < 0)
        return internal_fail(FK_E_ARG, "team must be in [0, %d], teams and spin_limit >= 0", TEAM_MAX);
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, B->device) != hipSuccess)
        lds_max = 65536;
    // static LDS of the kernel: reduction slots and the broadcast words
    const int static_lds = 3 * (wgs / 64) * 16 + 64;
    const int lds_cap = std::max(0, (lds_max - static_lds) / 16);
    int lds_rows = o->lds_rows == 0 ? std::min(6144, lds_cap) : o->lds_rows;
    if (lds_rows < 0)
        lds_rows = 0;
    if (lds_rows > lds_cap)
        return internal_fail(FK_E_ARG, "lds_rows = %d exceeds the %d rows that fit in LDS", lds_rows, lds_cap);
    lds_rows = std::min(lds_rows, B->max_rows);
    hipStream_t s = (hipStream_t)hip_stream;

    BatchArgs a{};
    a.sys_ptr = B->sys_ptr;
    a.order = B->order;
    a.count = B->count;
    a.row_ptr = B->row_ptr;
    a.col_idx = B->col_idx;
    a.vals = B->vals;
    a.vals32 = B->vals32;
    a.b = b;
    a.x = x;
    a.r32 = B->r32;
    a.p32 = B->p32;
    a.ap32 = B->ap32;
    a.d32 = B->d32;
    a.deque = B->deque;
    a.abort_flag = B->abort_flag;
    a.status = B->status;
    a.iters = B->iters;
    a.sweeps = B->sweeps;
    a.rel = B->rel;
    a.rtol = o->rtol;
    a.inner_rtol = o->inner_rtol == 0.0 ? 1e-4 : o->inner_rtol;
    a.max_iter = o->max_iter;
    a.max_outer = o->max_outer == 0 ? 50 : o->max_outer;
    a.lds_rows = lds_rows;
    const size_t lds = (size_t)lds_rows * 16;
    // One workgroup per CU slot the LDS allows, never more than the systems.
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B->device) != hipSuccess || cus < 1)
        cus = 256;
    const int per_cu = std::max(1, std::min(2048 / wgs, lds > 0 ? (int)(lds_max / (lds + static_lds)) : 2048 / wgs));
    int grid = std::max(1, std::min(B->count, cus * per_cu));

    // Teams wait for one another, so every member must be resident at once:
    // the kernel's occupancy bounds them, and the remaining resident slots
    // go to single workgroups.  Teams take the lowest workgroup ids, which
    // are dispatched first.
    //  Default (team = 0): teams of TEAM_DEFAULT over every resident
    //  workgroup when some system does not fit in LDS, else none.
    const int team = o->team == 0 ? (B->max_rows > lds_rows ? TEAM_DEFAULT : 1) : o->team;
    int nteams = 0;
    if (team > 1) {
        int occ = 0;
        if (occupancy(wgs, lds, &occ) != hipSuccess || occ < 1)
            return internal_fail(FK_E_HIP, "batch: occupancy query failed");
        const int resident = cus * occ;
        nteams = o->teams > 0 ? o->teams : resident / team;
        nteams = std::min({nteams, resident / team, B->count});
        if (nteams < 1)
            return internal_fail(FK_E_ARG, "team = %d exceeds the %d resident workgroups", team, resident);
        grid = nteams * team + std::max(0, std::min(B->count, resident - nteams * team));
        if (nteams > B->team_cap_n || team > B->team_cap_t) {
            dfree(B->team_cnt);
            dfree(B->team_slots);
            dfree(B->team_sys);
            B->team_cap_n = B->team_cap_t = 0;
            hipError_t e = dalloc(&B->team_cnt, (size_t)nteams * CNT_STRIDE);
            e = e ? e : dalloc(&B->team_slots, (size_t)nteams * 2 * team * KMAX * 2);
            e = e ? e : dalloc(&B->team_sys, (size_t)nteams);
            if (e != hipSuccess)
                return e == hipErrorOutOfMemory ? internal_fail(FK_E_OOM, "batch: out of device memory")
                                                : internal_fail(FK_E_HIP, "batch: %s", hipGetErrorString(e));
            B->team_cap_n = nteams;
            B->team_cap_t = team;
        }
    }
    a.team = team;
    a.nteams = nteams;
    a.team_cnt = B->team_cnt;
    a.team_slots = B->team_slots;
    a.team_sys = B->team_sys;
    const uint32_t spin_limit = o->spin_limit > 0 ? (uint32_t)o->spin_limit : TEAM_SPIN_DEFAULT;
    a.spin_limit = spin_limit;

    const bool graph = (o->flags & FK_FLAG_GRAPH) != 0 && s != nullptr;
    if (graph) {
        const bool same = B->exec && B->gwgs == wgs && B->glds == lds && B->ggrid == grid &&
                          std::memcmp(&B->gargs, &a, sizeof a) == 0;
        if (!same) {
            if (B->exec)
                (void)hipGraphExecDestroy(B->exec);
            if (B->graph)
                (void)hipGraphDestroy(B->graph);
            B->exec = nullptr;
            B->graph = nullptr;
            hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess)
                return internal_fail(FK_E_HIP, "capture: %s", hipGetErrorString(e));
            hipError_t el = launch(a, wgs, grid, lds, s);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(s, &g);
            if (el != hipSuccess || e != hipSuccess) {
                if (g)
                    (void)hipGraphDestroy(g);
                return internal_fail(FK_E_HIP, "capture: %s", hipGetErrorString(el != hipSuccess ? el : e));
            }
            e = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                return internal_fail(FK_E_HIP, "instantiate: %s", hipGetErrorString(e));
            }
            B->graph = g;
            B->gargs = a;
            B->gwgs = wgs;
            B->glds = lds;
            B->ggrid = grid;
        }
        hipError_t e = hipGraphLaunch(B->exec, s);
        if (e != hipSuccess)
            return internal_fail(FK_E_HIP, "graph launch: %s", hipGetErrorString(e));
    } else {
        hipError_t e = launch(a, wgs, grid, lds, s);
        if (e != hipSuccess)
            return internal_fail(FK_E_HIP, "batch launch: %s", hipGetErrorString(e));
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return internal_fail(FK_E_HIP, "batch solve: %s", hipGetErrorString(e));
    B->solved = true;
    if (nteams > 0) {
        int32_t aborted = 0;
        e = hipMemcpy(&aborted, B->abort_flag, sizeof aborted, hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return internal_fail(FK_E_HIP, "batch solve: %s", hipGetErrorString(e));
        if (aborted)
            return internal_fail(FK_E_HIP, "batch: a team wait exceeded %u polls; systems with status 3 were "
                                 "not solved", spin_limit);
    }
    return FK_OK;
}

extern "C" fk_status fk_batch_results(fk_batch B, int32_t *status, int32_t *iterations, int32_t *sweeps,
                                      double *rel_res)
{
    if (!B)
        return internal_fail(FK_E_ARG, "NULL batch");
    if (!B->solved)
        return internal_fail(FK_E_STATE, "no completed solve");
    const size_t c = (size_t)B->count;
    hipError_t e = hipSuccess;
    if (status)
        e = e ? e : hipMemcpy(status, B->status, c * 4, hipMemcpyDeviceToHost);
    if (iterations)
        e = e ? e : hipMemcpy(iterations, B->iters, c * 4, hipMemcpyDeviceToHost);
    if (sweeps)
        e = e ? e : hipMemcpy(sweeps, B->sweeps, c * 4, hipMemcpyDeviceToHost);
    if (rel_res)
        e = e ? e : hipMemcpy(rel_res, B->rel, c * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return internal_fail(FK_E_HIP, "fk_batch_results: %s", hipGetErrorString(e));
    return FK_OK;
}

extern "C" fk_status fk_batch_shape(fk_batch B, int32_t *count, int64_t *n, int64_t *nnz)
{
    if (!B || !count || !n || !nnz)
        return internal_fail(FK_E_ARG, "NULL argument");
    *count = B->count;
    *n = B->n;
    *nnz = B->nnz;
    return FK_OK;
}
