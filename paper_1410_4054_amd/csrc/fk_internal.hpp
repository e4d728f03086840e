// Internal declarations shared by the kernels (fk_kernels.hip) and the host
// driver / C ABI (fk_capi.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fk.h"

namespace fk {

// Workgroup shape of every kernel: four wave64 wavefronts.
constexpr int WG = 256;
constexpr int WAVES = WG / 64;
// Products staged in LDS per row block; rows longer than this are "long rows".
constexpr int NNZ_MAX = 2048;
constexpr int ITEMS = NNZ_MAX / WG;  // staged products per thread per block
// Largest number of inner products reduced together at one reduction point.
constexpr int KMAX = 4;
// Upper bound on workgroups of one launch (size of the partial-sum buffer).
constexpr int GMAX = 4096;
// The second reduction stage is a two-level tree: workgroups form groups
// of RGROUP; the last of each group sums the group, the last group's
// leader sums the group sums.
constexpr int RGROUP = 64;
constexpr int RNGROUPS_MAX = GMAX / RGROUP;
constexpr int CNT_STRIDE = 32;  // uint32 per arrival counter (one 128-byte line each)
// Published first-stage partials (FIN_PUBLISH) of at most this many dots.
constexpr int KPUB = 2;
// Layout of the reduction scratch (doubles): level-1 partials [KMAX][GMAX]
// double-double, level-2 partials [KMAX][RNGROUPS_MAX] double-double (both
// holding RED_EMPTY between launches: launch_red_init writes it, the
// leaders put it back), then published partials [KPUB][GMAX]
// double-double.
constexpr size_t RED_L2_OFFSET = (size_t)2 * KMAX * GMAX;
constexpr size_t RED_PUB_OFFSET = RED_L2_OFFSET + (size_t)2 * KMAX * RNGROUPS_MAX;
constexpr size_t RED_SCRATCH_DOUBLES = RED_PUB_OFFSET + (size_t)2 * KPUB * GMAX;
// The bits of an empty partial slot: a signalling NaN, which no
// floating-point operation returns.
constexpr uint64_t RED_EMPTY = 0x7ff40000deadbeefull;

// Solver state kept on the device; only the last workgroup of a reduction
// writes it, every kernel reads `status` first and returns unless it is one
// of the states in its run mask.
enum DevStatus : int32_t {
    ST_RUNNING = 0,
    ST_HALF = 1,          // BiCGStab: ||s_i|| met the tolerance; x_{i+1} = x_i + alpha p_i pending
    ST_CONVERGED = 2,
    ST_NOT_CONVERGED = 3, // iteration budget used up
    ST_BREAKDOWN = 4,
    ST_ZERO_RHS = 5,      // b = 0: x = 0, k = 0
    ST_CYCLE_DONE = 6,    // GMRES: the current restart cycle has ended
    // Pipelined BiCGStab: iteration i+1 is decided (converged, budget used
    // up, breakdown after the step), its x, r, p update still to run; that
    // update then sets the matching final state.
    ST_FINAL_CONVERGED = 7,
    ST_FINAL_NOT_CONVERGED = 8,
    ST_FINAL_BREAKDOWN = 9,
};

constexpr uint32_t RUN_ACTIVE = 1u << ST_RUNNING;
constexpr uint32_t RUN_ACTIVE_OR_HALF = (1u << ST_RUNNING) | (1u << ST_HALF);
constexpr uint32_t RUN_HALF = 1u << ST_HALF;
constexpr uint32_t RUN_BICG_UPDATE = RUN_ACTIVE_OR_HALF | (1u << ST_FINAL_CONVERGED) |
                                     (1u << ST_FINAL_NOT_CONVERGED) | (1u << ST_FINAL_BREAKDOWN);
constexpr uint32_t RUN_ALWAYS = 0xffffffffu;

struct alignas(128) DevState {
    double alpha, beta, omega;
    double rr;        // <r_i, r_i> (CG) / last direct <r,r> (BiCGStab, diagnostic)
    double rho;       // <r_i, r0*>
    double apr;       // <A p_i, r0*>
    double ss;        // <s_i, s_i>
    double rr_next;   // BiCGStab: expanded <r_{i+1}, r_{i+1}>
    double bnorm, tol, rtol;
    double last_rel;  // ||r_k|| / ||b|| of the last completed iteration
    double dots[KMAX];  // rounded results of the last reduction
    double rho0;      // GMRES: ||r0|| of the current cycle
    double zeta2;     // GMRES: (norm estimate / rho0)^2
    int32_t it;       // completed iterations k
    int32_t status;
    int32_t max_iter;
    int32_t hist_cap; // entries of hist / 4-tuples of scal available
    int32_t gi;       // GMRES: step of the current cycle (1-based, next to do)
    int32_t gm;       // GMRES: restart length m
    int32_t rho_pub;  // BiCGStab: <r,r0*>, <r,r> published by the last update
    int32_t red_fault;  // a reduction point gave up waiting (the solve is void)
};

// What the last workgroup does with the reduced inner products.
enum Fin : int32_t {
    FIN_NONE = 0,       // keep the rounded dots in state->dots only
    FIN_SETUP,          // d = {<r0,r0>, <b,b>}
    FIN_CG_ALPHA,       // d = {<p,Ap>, <Ap,Ap>}: alpha_i, beta_i (Eq. (3))
    FIN_CG_RR,          // d = {<r_i,r_i>}: k, convergence
    FIN_B_ALPHA,        // d = {<Ap,r0*>}: alpha_i
    FIN_B_SS,           // d = {<s,s>}: half-step test
    FIN_B_OMEGA,        // d = {<As,s>, <As,As>, <As,r0*>}: omega, beta, expanded rr
    FIN_B_XRP,          // d = {<r,r0*>, <r,r>}: rho, k, convergence (pipelined)
    FIN_C_CG_ALPHA,     // classical CG: d = {<p,q>}
    FIN_C_CG_BETA,      // classical CG: d = {<r,r>}
    FIN_C_B_OMEGA,      // classical BiCGStab: d = {<t,s>, <t,t>}
    FIN_C_B_RR,         // classical BiCGStab: d = {<r,r>}
    FIN_C_B_RHO,        // classical BiCGStab: d = {<r,r0*>}
    FIN_HALF_DONE,      // BiCGStab half-step exit bookkeeping (no dots)
    FIN_MIX_OUTER,      // mixed precision: d = {<r,r>, <b,b>} of the FP64 true residual
    FIN_GM_SETUP,       // GMRES cycle start: d = {<r0,r0>, <b,b>}
    FIN_GM_R1,          // GMRES: d = {<v_{i-1}, w>} -> R[i-1][i]
    FIN_GM_NORM,        // GMRES: d = {<w,w>} -> R[i][i]
    FIN_GM_XI,          // GMRES: d = {<r, v_i>} -> xi_i, norm estimate, step done
    FIN_PUBLISH,        // first stage only: store the workgroup partials for the
                        // next reduction point to fold in (no second stage here)
    FIN_CG_RR_ALPHA,    // d = {<p_i,Ap_i>, <Ap_i,Ap_i>, <r_i,r_i>} (the last one
                        // published by the update): FIN_CG_RR, then FIN_CG_ALPHA
    FIN_B_SS_OMEGA,     // d = {<As,s>, <As,As>, <As,r0*>, <s,s>} (the last one
                        // published by the s update): FIN_B_SS, then FIN_B_OMEGA,
                        // then the convergence decision on the expanded rr
    FIN_B_RHO_ALPHA,    // d = {<Ap,r0*>, <r,r0*>, <r,r>} (the last two published by
                        // the previous update, if any): rho, then FIN_B_ALPHA
    FIN_B_XRP_PUB,      // the x, r, p update: publishes <r,r0*>, <r,r> while the
                        // solve runs; after a decision, finalizes (FIN_B_XRP role)
    // The FP32-accumulating inner solver: the dots arrive as FP32 values and
    // the scalars of Algorithm 2 are formed in FP32 (held in the state's
    // doubles, which represent them exactly).
    FIN_SETUP32,        // d = {<r0,r0>, <r0,r0>}: FIN_SETUP with an FP32 tolerance
    FIN_CG_ALPHA32,     // d = {<p,Ap>, <Ap,Ap>}: alpha_i, beta_i (Eq. (3)) in FP32
    FIN_CG_RR_ALPHA32,  // d = {<p,Ap>, <Ap,Ap>, <r,r>}: FIN_CG_RR_ALPHA in FP32
    FIN_B_XRP_ALPHA,    // d = {<Ap,r0*>, <r,r0*>, <r,r>} of one launch (the x, r, p
                        // update fused with the next product): rho, then FIN_B_ALPHA
};

// Everything a reduction point needs.
struct RedArgs {
    DevState *st;
    double *partials;  // reduction scratch, RED_SCRATCH_DOUBLES (zeroed once)
    double *hist;      // ||r_i||/||b|| or nullptr
    double *scal;      // 4 scalars per iteration or nullptr
    int32_t fin;
    uint32_t run_mask;
    // Published partials folded into this reduction point: `npub` workgroup
    // partials of `kpub` dots (0: none), appended after the kernel's own dots.
    int32_t npub = 0;
    int32_t kpub = 0;
};

// Rows per slice of the sliced layout: one wave64, one row per lane.
constexpr int SLICE = 64;

// CSR matrix on the device plus the layout its products read.
//  - Row blocks (nslices == 0): the CSR arrays themselves, cut into blocks
//    of consecutive rows whose products are staged in LDS.
//  - Sliced (nslices > 0): the same nonzeros regrouped once, when the
//    matrix is created, into slices of SLICE consecutive rows.  Slice s
//    holds width_s = (sell_ptr[s+1] - sell_ptr[s]) / SLICE entries per row,
//    stored entry-major: the k-th nonzero of row s*SLICE + l is at
//    sell_ptr[s] + k*SLICE + l, in the row's CSR order; rows shorter than
//    width_s are padded with column -1 and value 0.  One lane sums one row
//    left to right, so every row sum is rounded exactly as in CSR order.
struct DevCsr {
    int32_t n;
    int32_t nnz;
    int32_t nblocks;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *vals;
    const int32_t *blocks;    // row index where block b starts; blocks[nblocks] = n
    const int32_t *block_j0;  // row_ptr[blocks[b]] (first nonzero of block b)
    int32_t nslices;          // 0: row blocks; > 0: sliced layout, ceil(n / SLICE) slices
    const int32_t *sell_ptr;  // nslices + 1 entry offsets
    const int32_t *sell_col;  // column of each entry, -1 for padding
    const double *sell_vals;  // value of each entry, 0 for padding
    // Narrow sliced layout (when non-null, read instead of sell_col): the
    // column of each entry as a 16-bit offset from its row, SELL_PAD for
    // padding, packed four entries per lane: entries 4j .. 4j+3 of row
    // s*SLICE + l are the short4 at sell_off4[sell_ptr4[s] + j*SLICE + l]
    // (the last group of a slice padded to four).
    const int32_t *sell_ptr4;
    const short4 *sell_off4;
    // Slot sliced layout (when non-null, read instead of both): slice s
    // stores w_s = (sell_ptr[s+1] - sell_ptr[s]) / SLICE slots, one per
    // distinct column offset (column - row) of its rows, in ascending order;
    // slot k of row s*SLICE + l holds the value of column row + dg_off[
    // sell_ptr[s]/SLICE + k] when bit k of dg_mask[row] is set (else 0).
    const int32_t *dg_off;
    const uint32_t *dg_mask;
    // Order in which the waves of a sliced product take the slices:
    // 0 = wave w of W takes slices w, w + W, ... (grid stride, XCD-major
    // workgroup numbering); 1 = sweep: the x-th eighth of the slices belongs
    // to XCD x, whose waves take consecutive slices side by side and move
    // through the eighth together (a sliding window; the grid then holds no
    // more workgroups than are resident at once).
    int32_t sweep;
    // 1: the sliced products load the matrix data non-temporally (the
    // matrix and the vectors of an iteration exceed the Infinity Cache, so
    // the matrix comes from HBM every launch anyway); 0: ordinary loads.
    int32_t stream;
    // Sliced layouts: the most entries (or slots) per row of any slice.
    int32_t max_width;
};

// Column forms of the sliced products.
constexpr int COLS_INT32 = 0;  // sell_col
constexpr int COLS_OFF16 = 1;  // sell_off4
constexpr int COLS_SLOTS = 2;  // dg_off + dg_mask
constexpr int DG_MAX_SLOTS = 32;  // slots per slice (bits of a row mask)

constexpr int16_t SELL_PAD = -32768;

// Dot selection bits for the fused product kernel y = A v.
enum DotBits : int32_t {
    D_YV = 1,  // <y, v>
    D_YY = 2,  // <y, y>
    D_YW = 4,  // <y, w>
};

// Profiling: when set, the next kernel launched by a wrapper below carries
// these two HIP events, stamped by the device when that kernel itself starts
// and ends (hipExtLaunchKernel), so the measured time is the kernel's own
// duration.  Cleared by that launch.
void set_launch_timing(hipEvent_t start, hipEvent_t stop);

// Host-side launch wrappers (fk_kernels.hip).
hipError_t launch_spmv_dots(const DevCsr &A, const double *v, double *y, const double *w,
                            int dots, const RedArgs &red, int grid, hipStream_t s);
hipError_t launch_residual0(const DevCsr &A, const double *b, const double *x, double *r,
                            double *p, double *rs, const RedArgs &red, int grid, hipStream_t s);
hipError_t launch_cg_update(int64_t n, double *x, double *r, double *p, const double *ap,
                            const RedArgs &red, int grid, hipStream_t s);
hipError_t launch_bicg_s(int64_t n, const double *r, const double *ap, double *sv,
                         const RedArgs &red, int grid, hipStream_t s);
hipError_t launch_bicg_xrp(int64_t n, double *x, double *r, double *p, const double *sv,
                           const double *as, const double *ap, const double *rs,
                           const RedArgs &red, int grid, hipStream_t s);
// The two-kernel BiCGStab iteration (updates folded into the products; see
// fk_kernels.hip): the vectors, with r_i, p_i and A p_i in two buffers
// each, selected by the parity of the device's iteration count (s_i is
// never stored: both steps recompute it from r_i and A p_i).
struct Bicg2Io {
    double *x;
    double *r[2];
    double *as;
    const double *rs;  // r0*
    double *p[2];
    double *ap[2];
};
hipError_t launch_bicg2_sas(const DevCsr &A, const Bicg2Io &io, const RedArgs &red, int grid, hipStream_t s);
// CG in one kernel per iteration: the x, r, p update of iteration i folded
// into A p_i (r, p, A p in two buffers each, by the parity of the count).
struct Cg1Io {
    double *x;
    double *r[2];
    double *p[2];
    double *ap[2];
};
hipError_t launch_cg1_xap(const DevCsr &A, const Cg1Io &io, const RedArgs &red, int grid, hipStream_t s);
// Workgroups of a fused step resident per compute unit.
enum FusedStep : int { FUSED_BICG_SAS = 0, FUSED_BICG_XAP = 1, FUSED_CG_XAP = 2 };
int fused_per_cu(const DevCsr &A, int step);
hipError_t launch_bicg2_xap(const DevCsr &A, const Bicg2Io &io, const RedArgs &red, int grid, hipStream_t s);
// Classical (unfused) building blocks.
// <a,b> (ndots 1); <a,b>, <a,c> (2); <a,b>, <a,c>, <a,e> (3).
hipError_t launch_dot(int64_t n, const double *a, const double *b, const double *c,
                      int ndots, const RedArgs &red, int grid, hipStream_t s, const double *e = nullptr);
// out = y + coef * x (negative = 0) or y - coef * x (negative = 1),
// coef = state->alpha (which = 0) or state->omega (which = 1)
hipError_t launch_axpy(int64_t n, double *out, const double *y, const double *x, int which,
                       int negative, DevState *st, uint32_t run_mask, int grid, hipStream_t s);
// p = r + beta * (p - omega * v) when v != nullptr, else p = r + beta * p
hipError_t launch_xpay(int64_t n, double *p, const double *r, const double *v,
                       DevState *st, uint32_t run_mask, int grid, hipStream_t s);
// dst = src when state->status is in run_mask; then runs `fin` on one thread.
hipError_t launch_copy_fin(int64_t n, double *dst, const double *src, const RedArgs &red,
                           hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, int64_t n_bytes, int grid, hipStream_t s);
// out = alpha x + beta y
hipError_t launch_axpby(int64_t n, double alpha, const double *x, double beta, const double *y,
                        double *out, int grid, hipStream_t s);

// Mixed precision (FP32 inner pipelined CG inside FP64 iterative refinement).
// r32 = (float)(b - A x) with FP64 <r,r>, <b,b> (FIN_MIX_OUTER).
hipError_t launch_residual32(const DevCsr &A, const double *b, const double *x, float *r32,
                             const RedArgs &red, int grid, hipStream_t s);
// y = A32 v with the FP32 dots <y,v>, <y,y> (FIN_CG_ALPHA or FIN_CG_ALPHA32
// on the inner state), accumulated exactly (double-double) or, with
// f32acc, in FP32.  vals32 holds the FP32 values in the layout A's products
// read: CSR order (nnz entries) for row blocks, slice order
// (sell_ptr[nslices] entries) for the sliced layout.
hipError_t launch_spmv32(const DevCsr &A, const float *vals32, const float *v, float *y,
                         const RedArgs &red, int grid, hipStream_t s, bool f32acc);
// out[e] = map[e] >= 0 ? vals[map[e]] : 0 (the values of the sliced layout).
hipError_t launch_gather_vals(int64_t n, double *out, const double *vals, const int32_t *map,
                              int grid, hipStream_t s);
hipError_t launch_cg_update32(int64_t n, float *d, float *r, float *p, const float *ap,
                              const RedArgs &red, int grid, hipStream_t s, bool f32acc);
// p = r, d = 0, FP32 <r,r> twice (FIN_SETUP / FIN_SETUP32 on the inner state).
hipError_t launch_inner_setup32(int64_t n, const float *r, float *p, float *d, const RedArgs &red,
                                int grid, hipStream_t s, bool f32acc);
hipError_t launch_add32(int64_t n, double *x, const float *d, int grid, hipStream_t s);
hipError_t launch_to_f32(int64_t n, float *out, const double *in, int grid, hipStream_t s);

// GMRES(m) (Algorithms 5 and 6).  The basis V holds m+1 vectors of n
// doubles (v_0 = r0 / rho0, v_1..v_m orthonormal); R is (m+1) x (m+1)
// row-major, row 0 holding xi_1..xi_m.  In `red`, scal points to R.
constexpr int GM_MAX = 64;          // largest restart length
#ifndef FK_GM_GRID
#define FK_GM_GRID 1024
#endif
constexpr int GM_GRID = FK_GM_GRID;  // workgroups of the multi-dot kernel
// Multi-dot scratch (doubles): double-double partials [GM_MAX][GM_GRID].
constexpr size_t GM_PART_DOUBLES = (size_t)2 * GM_MAX * GM_GRID;
// out = in / rho0 (the cycle's first basis vector)
hipError_t launch_gm_scale(int64_t n, double *out, const double *in, DevState *st, uint32_t run_mask, int grid,
                           hipStream_t s);
// R[j][i] = <v_j, w> for j0 <= j < j1: first stage (per-workgroup partials
// into part), then the second stage, one workgroup per dot, writing R.
hipError_t launch_gm_multidot(int64_t n, const double *V, const double *w, int j0, int j1, double *part,
                              DevState *st, uint32_t run_mask, hipStream_t s);
hipError_t launch_gm_multidot_fin(int j0, int j1, int i, double *R, int m1, const double *part, DevState *st,
                                  uint32_t run_mask, hipStream_t s);
// w -= sum_{j=1}^{i-1} R[j][i] v_j; first stage of <w,w> (FIN_GM_NORM)
hipError_t launch_gm_update(int64_t n, double *w, const double *V, int i, int m1, const RedArgs &red, int grid,
                            hipStream_t s);
// v_i = w / R[i][i] in place; first stage of <r, v_i> (FIN_GM_XI)
hipError_t launch_gm_normalize(int64_t n, double *v, const double *r, int i, int m1, const RedArgs &red,
                               int grid, hipStream_t s);
// r -= xi_i v_i (the classical form's residual update)
hipError_t launch_gm_rupdate(int64_t n, double *r, const double *v, int i, const double *R, DevState *st,
                             uint32_t run_mask, int grid, hipStream_t s);
// x += rho0 (eta_1 v_0 + sum_{j=2}^{used} eta_j v_{j-1})
hipError_t launch_gm_xupdate(int64_t n, double *x, const double *V, const double *eta, int used,
                             const DevState *st, int grid, hipStream_t s);

// Single-workgroup solver (whole solve in one launch) for small systems.
// Rows per thread: 1, 2, 4 or 8 (0 = too large); LDS bytes it needs.
// `stage`: copy the matrix into LDS first (needs small_staged_lds_bytes).
int small_rows_per_thread(int64_t n);
size_t small_lds_bytes(int method_bicg, int64_t n);
size_t small_staged_lds_bytes(int method_bicg, int64_t n, int64_t nnz);
hipError_t launch_small(int method_bicg, const DevCsr &A, const double *b, double *x, DevState *st,
                        double *hist, double *scal, bool stage, hipStream_t s);
hipError_t launch_zero(double *x, int64_t n, DevState *st, uint32_t run_mask, int grid,
                       hipStream_t s);
// x[0 .. n) = 0, unconditionally.
hipError_t launch_clear(double *x, int64_t n, int grid, hipStream_t s);
// A reduction scratch of RED_SCRATCH_DOUBLES ready for its first use: the
// partial slots empty (RED_EMPTY), the published partials zero.
hipError_t launch_red_init(double *partials, hipStream_t s);
// *st = the state a multi-kernel solve starts from (running, rtol, max_iter,
// hist_cap, everything else zero), written by a one-thread kernel.
hipError_t launch_state_init(DevState *st, double rtol, int32_t max_iter, int32_t hist_cap, hipStream_t s);

// Shared by the C ABI sources: record the thread's error message and
// return `s`; the device view of a matrix handle.
fk_status internal_fail(fk_status s, const char *fmt, ...);
DevCsr internal_csr_view(fk_csr A);

}  // namespace fk
