/*
 * fk.h -- C ABI of the MI355X (gfx950) pipelined Krylov solver library libfk.so.
 *
 * The library solves sparse linear systems A x = b held in CSR form, in FP64,
 * with the pipelined conjugate gradient method (Algorithm 2 with the beta
 * recurrence of Eq. (3), Section 3.1) and the pipelined BiCGStab method
 * (Algorithm 4, Section 3.2) of Rupp, Weinbub, Juengel and Grasser,
 * "Pipelined Iterative Solvers with Kernel Fusion for GPUs" (arXiv:1410.4054).
 * The classical formulations (Algorithms 1 and 3) are provided as unfused
 * baselines built from one kernel per vector operation.  FK_CG_MIXED runs
 * the pipelined CG iteration in FP32 storage and arithmetic as the inner
 * solver of an FP64 iterative refinement (an extension: Section 3.1 cites a
 * mixed-precision pipelined CG on FPGAs as prior work, the paper itself
 * stays in FP64).
 *
 * Every step of an iteration runs in hand-written HIP kernels: the CSR
 * product fused with the first stage of the inner products that follow it
 * (Section 2.2), the vector updates fused with the next first-stage
 * reductions, and a second reduction stage done on the device by the last
 * workgroup to finish, which also evaluates alpha, beta, omega and the
 * convergence test, so no scalar crosses to the host inside an iteration.
 *
 * Conventions for every entry point:
 *   - Return value: an fk_status.  No exception crosses the ABI and nothing
 *     aborts.  On failure fk_last_error() gives a message (per thread).
 *   - Device pointers are HIP device memory of the current device (e.g. the
 *     data pointer of a torch.cuda tensor).  The library never frees
 *     caller memory.
 *   - `hip_stream` is a hipStream_t passed as void* (NULL = default stream).
 *   - Vectors are contiguous float64 arrays of length n.
 *   - CSR: int32 row_ptr[n+1] with row_ptr[0] = 0, nondecreasing,
 *     row_ptr[n] = nnz; int32 col_idx[nnz] in [0, n); float64 vals[nnz].
 *     Duplicate column indices in a row are allowed (they are summed).
 *   - Numbers: IEEE FP64 with round to nearest.  A CSR row is summed left to
 *     right in storage order (rows longer than FK_LONG_ROW are summed by a
 *     fixed tree instead).  Inner products accumulate error-free products
 *     in double-double and are rounded once, so they are independent of the
 *     launch shape and reproducible bit for bit from run to run.
 */
#ifndef FK_H
#define FK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fk_csr_s *fk_csr;
typedef struct fk_solver_s *fk_solver;
typedef struct fk_net_s *fk_net;
typedef struct fk_batch_s *fk_batch;

typedef enum {
    FK_OK = 0,              /* success; for fk_solve: converged             */
    FK_E_ARG = 1,           /* invalid argument (NULL, size, option)        */
    FK_E_CSR = 2,           /* malformed CSR arrays                         */
    FK_E_HIP = 3,           /* a HIP runtime call failed                    */
    FK_E_OOM = 4,           /* device or host allocation failed             */
    FK_NOT_CONVERGED = 5,   /* max_iter reached; x holds x_{max_iter}       */
    FK_BREAKDOWN = 6,       /* zero/non-finite denominator or residual      */
    FK_E_STATE = 7          /* call out of order (e.g. no solve yet)        */
} fk_status;

typedef enum {
    FK_CG_PIPELINED = 0,        /* Algorithm 2 + Eq. (3): 2 kernels/iteration   */
    FK_CG_CLASSICAL = 1,        /* Algorithm 1 as SpMV, dot, axpy, axpy, dot, xpay */
    FK_BICGSTAB_PIPELINED = 2,  /* Algorithm 4: 4 kernels/iteration             */
    FK_BICGSTAB_CLASSICAL = 3,  /* Algorithm 3, one kernel per operation         */
    FK_CG_MIXED = 4,            /* FP64 iterative refinement around FP32 Algorithm 2 */
    FK_GMRES_PIPELINED = 5,     /* Algorithm 6: restarted GMRES(m), 4 kernels/iteration */
    FK_GMRES_CLASSICAL = 6,     /* Algorithm 5: residual updated in the loop (+1 kernel) */
    FK_CG_MIXED_F32 = 7,        /* FK_CG_MIXED with FP32-accumulated inner products */
    FK_CG_PIPELINED_SPLIT = 8,  /* Algorithm 2 with the product's dots in their own
                                   kernel (Section 3.1's alternative): 3 kernels */
    FK_BICGSTAB_PIPELINED_SPLIT = 9, /* Algorithm 4 with both products' dots in their
                                   own kernels (Section 3.2's alternative): 6 kernels */
    FK_BICGSTAB_PIPELINED_2K = 10, /* Algorithm 4 in 2 kernels/iteration: each vector
                                   update of Section 3.2 folded into the product
                                   that follows it (the product recomputes the
                                   updated vector where it gathers it); the same
                                   iterates, bit for bit, as FK_BICGSTAB_PIPELINED */
    FK_CG_PIPELINED_1K = 11    /* Algorithm 2 + Eq. (3) in 1 kernel/iteration: the
                                   x, r, p update folded into the product the same
                                   way; the same iterates as FK_CG_PIPELINED */
} fk_method;

/* Rows with more nonzeros than this are summed by a fixed tree, not left to right. */
#define FK_LONG_ROW 2048

/* Solver options.  Zero-initialised fields take the defaults noted. */
typedef struct {
    int32_t method;          /* fk_method                                       */
    double rtol;             /* stop when ||r_k||_2 <= rtol * ||b||_2 (>= 0)   */
    int32_t max_iter;        /* >= 0; iterations allowed (0 = setup only);
                                FK_CG_MIXED: inner iterations over all sweeps  */
    int32_t record_history;  /* >= 0.  0: no history.  Otherwise keep
                                ||r_i||/||b|| for i = 0..min(k, cap-1) with
                                cap = min(max_iter + 1, FK_HISTORY_DEFAULT)
                                when 1, min(max_iter + 1, record_history) when
                                larger (FK_CG_MIXED: one entry per refinement
                                sweep, at most max_outer + 1)                 */
    int32_t unroll;          /* iterations enqueued between status polls (0 = 32) */
    int32_t flags;           /* FK_FLAG_* bits                                  */
    double inner_rtol;       /* FK_CG_MIXED: inner stop ||r_in|| <= inner_rtol *
                                ||r_j|| (>= 0; 0 = 1e-4)                       */
    int32_t max_outer;       /* FK_CG_MIXED: refinement sweeps allowed
                                (>= 0; 0 = 50)                                 */
    int32_t restart;         /* GMRES: restart length m (0 = 30; at most 64)    */
} fk_opts;

/* flags */
#define FK_FLAG_GRAPH 1      /* replay the enqueued iterations from a hipGraph */
#define FK_FLAG_PROFILE 2    /* time every kernel with HIP events              */
#define FK_FLAG_NO_SMALL 4   /* never use the single-workgroup solver           */
#define FK_FLAG_SCALARS 8    /* with record_history: also keep alpha, beta, omega
                                and the tested <r,r> per iteration (4 doubles
                                per history entry; fk_get_scalars)             */

/* History entries kept by default (record_history = 1): 512 KiB of device
 * memory, whatever max_iter is. */
#define FK_HISTORY_DEFAULT 65536

enum { FK_PTR_HOST = 0, FK_PTR_DEVICE = 1 };

/* Layouts the product kernels read (fk_csr_layout, fk_csr_set_layout). */
enum {
    FK_LAYOUT_AUTO = 0,        /* the creation rule below                      */
    FK_LAYOUT_ROW_BLOCKS = 1,  /* the CSR arrays, cut into row blocks          */
    FK_LAYOUT_SLICED = 2,      /* the nonzeros regrouped into 64-row slices    */
    FK_LAYOUT_SLICED16 = 3,    /* the same, columns as 16-bit row offsets      */
    FK_LAYOUT_SLOTS = 4        /* 64-row slices, one slot per column offset    */
};

/*
 * Create a device-resident CSR matrix (the CSR storage of Section 2.2).
 * The arrays are validated on the host (FK_E_CSR on any violation of the
 * conventions above, before any device work), then copied into library-owned
 * device memory; the caller keeps ownership of its arrays and may free them
 * as soon as this returns.  ptr_kind says where the three arrays live
 * (FK_PTR_HOST or FK_PTR_DEVICE; device arrays are copied back to the host
 * once for validation and row-block planning).  Requires 1 <= n,
 * 0 <= nnz <= INT32_MAX.  *out receives the handle.
 */
fk_status fk_csr_create(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                        const double *vals, int32_t ptr_kind, void *hip_stream, fk_csr *out);

/* Release a matrix.  Solvers created on it must be destroyed first. */
fk_status fk_csr_destroy(fk_csr A);

/* n and nnz of a matrix. */
fk_status fk_csr_shape(fk_csr A, int64_t *n, int64_t *nnz);

/* Row-block plan made at creation: number of row blocks (runs of at most 256
 * consecutive rows holding at most FK_LONG_ROW nonzeros, the unit of work of
 * the product kernels) and number of rows longer than FK_LONG_ROW. */
fk_status fk_csr_blocks(fk_csr A, int32_t *nblocks, int32_t *long_rows);

/*
 * Layout of the sparse products.  Both compute y_i as the sum of the row's
 * products a_ij v_j taken left to right in CSR order (the SpMV of Section
 * 2.2), so every result is bitwise the same in either layout; they differ
 * only in how the nonzeros sit in device memory (Section 4 compares solvers
 * across storage formats, ELLPACK among them):
 *  - FK_LAYOUT_ROW_BLOCKS: the CSR arrays; a workgroup stages the products
 *    of a run of rows in LDS and one thread sums each row.
 *  - FK_LAYOUT_SLICED: a copy of the nonzeros in slices of 64 consecutive
 *    rows; slice s stores w_s entries per row, w_s being its longest row,
 *    entry k of each row of the slice side by side (sliced ELLPACK without
 *    row sorting), shorter rows padded.  One lane sums one row; no LDS.
 *    Costs 12 bytes of device memory per stored entry next to the CSR
 *    arrays, which stay (other kernels read them).
 *  - FK_LAYOUT_SLICED16: the sliced layout with each column stored as a
 *    16-bit offset from its row, so a product reads about 10 bytes per
 *    entry instead of 12 (6 instead of 8 for FP32 values).  Possible when every
 *    column lies within 32767 of its row (banded and stencil matrices);
 *    2 more bytes of device memory per stored entry.
 *  - FK_LAYOUT_SLOTS: 64-row slices again, but slice s keeps one slot per
 *    distinct column offset (column - row) of its rows, in ascending
 *    order, 4 bytes each for the whole slice, and each row a 32-bit mask of
 *    the slots it has; slot k of a row holds the value of column row +
 *    offset_k (0 where absent).  A product reads about 8 bytes per stored
 *    entry plus 4 per row.  Possible when every row's columns strictly
 *    ascend (so slot order is CSR order), no slice has more than 32
 *    distinct offsets (stencils and other structured-grid matrices, at any
 *    bandwidth) and the slots pad the entries by at most 25 %.  12 more
 *    bytes of device memory per stored entry and 4 per row.
 * fk_csr_create picks SLOTS when possible, else a sliced layout when no row
 * has more than 64 nonzeros and the padding adds at most 25 % to the
 * entries read (SLICED16 when the offsets fit, else SLICED), else
 * ROW_BLOCKS.  fk_csr_layout reports the
 * layout in use, the entries its products read per call (nnz, or the slice
 * entries with padding) and, when matrix_bytes is not NULL, the bytes of
 * matrix data one FP64 product reads (values, column indices or offsets,
 * row or slice pointers, slot offsets and row masks; the 16-bit offsets are
 * read four at a time, so a row's last group counts whole).
 */
fk_status fk_csr_layout(fk_csr A, int32_t *layout, int64_t *stored_entries, int64_t *matrix_bytes);

/*
 * Force a layout: FK_LAYOUT_ROW_BLOCKS, FK_LAYOUT_SLICED (builds the slices
 * when absent, whatever their padding; FK_E_ARG if they would need more than
 * INT32_MAX entries), FK_LAYOUT_SLICED16 (the same; FK_E_ARG when a column
 * lies more than 32767 from its row), FK_LAYOUT_SLOTS (builds the slots when
 * absent; FK_E_ARG when the conditions above do not hold) or
 * FK_LAYOUT_AUTO (the creation rule).  Solvers read the
 * layout when they are created, so FK_E_STATE while any solver exists on A.
 * Runs on hip_stream and returns after it has drained.
 */
fk_status fk_csr_set_layout(fk_csr A, int32_t layout, void *hip_stream);

/*
 * Streaming mode of the sliced products (the fused SpMV + inner products of
 * Section 2.2 on the slice layouts; no effect on ROW_BLOCKS).  On, the
 * products load the matrix data non-temporally and each XCD's workgroups
 * sweep one contiguous eighth of the slices together, so that the vector
 * lines one slice gathers are still cached when the neighbouring planes'
 * slices gather them again.  Off, ordinary loads and a grid-stride order.
 * Results are bitwise the same either way; only the speed differs.
 * mode: -1 = by size (on when the matrix data one product reads plus four
 * FP64 vectors of length n exceed 256 MiB, the MI355X's Infinity Cache),
 * 0 = off, 1 = on.  The environment variables FK_STREAM (-1/0/1) and
 * FK_SELL_SWEEP (0/1, the order alone) set the default of a new matrix.
 * Solvers read the mode when they are created, so FK_E_STATE while any
 * solver exists on A; FK_E_ARG for another mode.
 * fk_csr_stream reports whether the mode is on and (when sweep is not NULL)
 * whether the products run in sweep order.
 */
fk_status fk_csr_set_stream(fk_csr A, int32_t mode);
fk_status fk_csr_stream(fk_csr A, int32_t *streaming, int32_t *sweep);

/*
 * Create a solver for A with options *o, bound to hip_stream.  Allocates the
 * library-owned workspace once, so fk_solve allocates nothing: the method's
 * work vectors (r, p, A p for Algorithm 2; r, r0*, p, A p, s, A s for
 * Algorithm 4: about 3n and 6n doubles; the one-kernel CG and the
 * two-kernel BiCGStab keep r, p and A p in two buffers each, the latter
 * without s), the buffer of per-workgroup
 * partial sums that the first reduction stage writes and the second reads
 * (Section 2.2, the two-stage reduction; Section 3.1, the partial results of
 * the three inner products of an iteration in one buffer), and the device
 * scalars alpha, beta, omega, <r,r> that the paper keeps on the host between
 * kernels (Section 3.1), plus the history buffers record_history asks for.
 * FK_E_ARG for an unknown method, negative sizes, non-finite or negative
 * tolerances or unknown flags; FK_E_OOM when an allocation fails (nothing is
 * left allocated).
 *
 * Pipelined solves of small systems (n <= 4096 for CG, 3072 for the
 * one-kernel CG, n <= 2048 for
 * BiCGStab, nnz <= 65536, no row longer than FK_LONG_ROW, vectors fitting
 * the device's LDS) run as one single-workgroup kernel per solve, whose
 * iterates equal those of the multi-kernel path; FK_FLAG_NO_SMALL disables
 * that.  fk_solver_uses_small() tells which path a solver takes.
 */
fk_status fk_solver_create(fk_csr A, const fk_opts *o, void *hip_stream, fk_solver *out);

/*
 * FK_CG_MIXED (iterative refinement with an FP32 inner solver): sweep
 * j = 0, 1, ... computes r_j = b - A x_j in FP64 (values summed row by row
 * in CSR order) and stops when ||r_j|| <= rtol ||b||; otherwise it solves
 * A d = r_j approximately by pipelined CG (Algorithm 2, Eq. (3)) with d_0 = 0,
 * FP32 vectors, FP32 matrix values (rounded once, when the solver is
 * created) and FP32 arithmetic, until its recursively updated residual
 * satisfies ||r_in|| <= inner_rtol ||(float) r_j||, and sets
 * x_{j+1} = x_j + d in FP64.  Inner products are exact products of the FP32
 * operands accumulated in double-double, so they are reproducible as on the
 * FP64 path.  The solve ends FK_NOT_CONVERGED when max_iter inner
 * iterations or max_outer sweeps are used up or an inner solve stops without
 * an iteration (its correction would be 0), and FK_BREAKDOWN (x = x_j) when
 * an inner solve breaks down or a residual is not finite.  k
 * (fk_get_iterations) counts inner iterations over all sweeps, the residual
 * and its history are those of the FP64 residuals r_j, and
 * fk_get_refinements gives the number of sweeps (corrections applied).
 * Workspace: 4n floats plus nnz FP32 matrix values.
 *
 * FK_CG_MIXED_F32: the same refinement, but the inner solver accumulates in
 * FP32 throughout: each inner product adds FP32-rounded products to FP32
 * sums (per thread, then fixed-order trees over lanes, waves and
 * workgroups), and alpha, beta (Eq. (3)), the inner norm and its test are
 * formed in FP32.  The sums are reproducible run to run for a given launch
 * shape but not equal to a sequential FP32 sum; each is within the FP32
 * bound gamma_n sum |a_i b_i| of the exact value.
 *
 * FK_GMRES_PIPELINED / FK_GMRES_CLASSICAL (restarted simpler GMRES(m) with
 * classical Gram-Schmidt, Section 3.3): a cycle starts from r0 = b - A x
 * (its true norm rho0 is the history entry at the restart and decides
 * convergence), v_0 = r0 / rho0, and for i = 1..m: w = A v_{i-1};
 * R[j][i] = <v_j, w> for j = 1..i-1 (all from the same w); w -= sum_j
 * R[j][i] v_j; R[i][i] = ||w||; v_i = w / R[i][i]; xi_i = <r, v_i> with
 * r = v_0 (pipelined: no residual update) or r updated as r -= xi_i v_i
 * (classical).  Per iteration the pipelined form runs four kernels: the CSR
 * product with <v_{i-1}, w>, the remaining inner products, the update with
 * ||w||^2, the normalisation with xi_i; every second reduction stage runs on
 * the device.  The device ends a cycle early when rho0 sqrt(1 - sum xi^2)
 * (floored at 0) meets the tolerance (that value is the history entry of the
 * iteration), after m steps, when max_iter products are used, or before a
 * step whose ||w|| is 0 or not finite.  Per cycle the host reads R and xi,
 * solves R eta = xi and the device sets x += rho0 (eta_1 v_0 +
 * sum_{j>=2} eta_j v_{j-1}).  k counts products A v over all cycles.  A cycle
 * with no step is a breakdown.  Workspace: (m+2) n doubles.
 *
 * Solve A x = b (the problem of Section 1, by the method the solver was
 * created with: Algorithms 1-6 of Section 3, the setup and iteration steps
 * in the paper's order).  b_dev, x_dev: caller-owned device float64[n]; x
 * holds x0 on entry and x_k on return.  Work is enqueued on the solver's stream and the
 * call returns once it has completed.  Returns FK_OK (converged),
 * FK_NOT_CONVERGED (x = x_{max_iter}), FK_BREAKDOWN (x = last finite iterate
 * before the failing step) or an error.  b = 0 gives x = 0, k = 0, FK_OK.
 */
fk_status fk_solve(fk_solver S, const double *b_dev, double *x_dev);

/* Iterations k of the last solve: the number of solution updates performed,
 * i.e. passes through the loop body of Algorithms 1-4 (index i of the loop
 * when it stops, plus one); GMRES: products A v over all cycles (Section 3.3).
 * FK_E_STATE before the first completed solve. */
fk_status fk_get_iterations(fk_solver S, int32_t *k);

/* ||r_k||_2 / ||b||_2 of the last solve, from the recursively updated residual
 * (pipelined BiCGStab: from the expansion of <r_{k}, r_{k}> in Section 3.2). */
fk_status fk_get_residual(fk_solver S, double *rel_res);

/* Residual history of the last solve: out[i] = ||r_i||/||b||, i = 0..k, the
 * norm of the recursively updated residual that the paper monitors once per
 * iteration through <r_i, r_i> (Section 3.1; Section 3.2: the expansion of
 * <r_{i+1}, r_{i+1}> for BiCGStab).  Sets *len to the number of entries kept,
 * min(k+1, the history capacity of record_history) and writes min(cap, *len)
 * of them.  FK_E_STATE without record_history or before a solve.
 * FK_CG_MIXED: out[j] = ||b - A x_j||/||b|| for sweeps j = 0..J. */
fk_status fk_get_residual_history(fk_solver S, double *out, int32_t cap, int32_t *len);

/* Per-iteration scalars of the last solve (for diagnostics): for iteration
 * i < *len = min(k, history capacity), out[4*i + 0..3] = alpha_i, beta_i,
 * omega_i (0 for CG), and the A-expanded (BiCGStab) or plain <r,r> used for
 * the test; min(cap, *len) iterations are written.  Needs record_history and
 * FK_FLAG_SCALARS; not recorded for FK_CG_MIXED or GMRES (FK_E_STATE). */
fk_status fk_get_scalars(fk_solver S, double *out, int32_t cap, int32_t *len);

/* Average device time per launch of each kernel kind during the last solve
 * made with FK_FLAG_PROFILE.  Kinds are the FK_KERNEL_* values below;
 * avg_us[kind] and count[kind] are written for kind < cap. */
enum {
    FK_KERNEL_SETUP = 0,       /* r0 = b - A x0 and its reductions            */
    FK_KERNEL_SPMV_DOT = 1,    /* fused CSR product + first-stage dots
                                  (FK_BICGSTAB_PIPELINED_2K: A s_i, with s_i
                                  formed but not stored;
                                  FK_CG_PIPELINED_1K: x, r, p and A p)       */
    FK_KERNEL_UPDATE_DOT = 2,  /* fused vector updates + first-stage dot(s)
                                  (FK_BICGSTAB_PIPELINED_2K: x, r, p, A p)    */
    FK_KERNEL_SPMV = 3,        /* plain CSR product (classical)               */
    FK_KERNEL_DOT = 4,         /* plain dot (classical)                        */
    FK_KERNEL_AXPY = 5,        /* plain vector update (classical)             */
    FK_KERNEL_SMALL = 6,       /* whole solve in one workgroup (small systems) */
    FK_KERNEL_RESIDUAL = 7,    /* FK_CG_MIXED: FP64 r_j = b - A x_j + its dots  */
    FK_KERNEL_KINDS = 8
};
fk_status fk_get_kernel_times(fk_solver S, double *avg_us, int32_t *count, int32_t cap);

fk_status fk_solver_destroy(fk_solver S);

/* *small = 1 if fk_solve runs the single-workgroup solver, else 0. */
fk_status fk_solver_uses_small(fk_solver S, int32_t *small);

/* FK_CG_MIXED: refinement sweeps (corrections x += d) of the last solve;
 * 0 for the other methods. */
fk_status fk_get_refinements(fk_solver S, int32_t *sweeps);

/*
 * q = A p with optional fused first-stage reductions (the fused kernel of
 * Section 2.2): if dots_host is not NULL it receives {<p,q>, <q,q>}.
 * Calls on the same matrix share its reduction scratch: do not overlap them.
 * p_dev, q_dev: device float64[n], must not alias.  Synchronous.
 */
fk_status fk_spmv(fk_csr A, const double *p_dev, double *q_dev, double *dots_host, void *hip_stream);

/*
 * The kernel time of q = A p (Section 2.2's product): `reps` launches back
 * to back, each carrying two HIP events that the device stamps when the
 * kernel itself starts and ends; *avg_us receives their average duration.
 * mode 0: the product alone; 1: fused with the first stage of <p,q>, <q,q>
 * and their second stage (as fk_spmv with dots); 2: the product, then a
 * separate kernel for the two inner products (Section 2.2's unfused pair;
 * the average is that of the pair, each kernel timed on its own).
 * FK_E_ARG for reps < 1 or another mode.  Synchronous.
 */
fk_status fk_spmv_time(fk_csr A, const double *p_dev, double *q_dev, int32_t mode, int32_t reps,
                       double *avg_us, void *hip_stream);

/*
 * q = A p in FP32, the inner product kernel of FK_CG_MIXED / FK_CG_MIXED_F32
 * (Section 2.2's fused kernel in single precision): the values of A rounded
 * to FP32 (once, at the first call after a layout change, kept with the
 * matrix), each row summed left to right in FP32.  If dots_host is not NULL
 * it receives {<p,q>, <q,q>}: exact sums of the FP32 operands rounded to
 * FP64 (f32acc = 0) or FP32 accumulations (f32acc = 1; the float returned
 * as a double).  p_dev, q_dev: device float32[n], must not alias.  Shares
 * the matrix's reduction scratch with fk_spmv.  Synchronous.
 */
fk_status fk_spmv32(fk_csr A, const float *p_dev, float *q_dev, int32_t f32acc, double *dots_host,
                    void *hip_stream);

/* <a, b> over n >= 0 device doubles, written to *out_host.  Synchronous. */
fk_status fk_dot(int64_t n, const double *a_dev, const double *b_dev, double *out_host, void *hip_stream);

/* out = alpha x + beta y over n >= 0 device doubles (out may alias x or y);
 * enqueued on hip_stream, not waited for. */
fk_status fk_axpby(int64_t n, double alpha, const double *x_dev, double beta, const double *y_dev,
                   double *out_dev, void *hip_stream);

/* Plain device copy of n_bytes (a streaming kernel, for bandwidth calibration). */
fk_status fk_copy(void *dst_dev, const void *src_dev, int64_t n_bytes, void *hip_stream);

/*
 * Learned initial guess for a sequence of solves on an nx-by-ny grid (an
 * extension for the many related small-to-medium systems of transient
 * problems that motivate the paper, Section 1; the network itself is not in
 * the paper).  Row i of the matrix is grid point (i % nx, i / nx), so
 * n = nx * ny.  The network N is a learned local approximate inverse: from
 * the residual r = b - A x of a guess x (FP64, rows summed in CSR order) it
 * predicts a correction, x <- x + N(r).  A step starts from the
 * extrapolation x = 2 u_m - u_{m-1} of the solutions of the two previous
 * steps (pass u_m twice at the first step) and applies N `passes` times.
 * N is a BF16 convolutional network run on the matrix cores: `layers` 3x3
 * cross-correlations with zero padding and no bias (1 -> 16 -> ... -> 16 ->
 * 1 channels, `channels` = 16), FP32 accumulation, with FK_NET_RELU or
 * FK_NET_LINEAR (identity: a deep linear network, a learned linear
 * approximate inverse) between layers.  N has no bias, so N(a r) = a N(r)
 * for a > 0 (every a when linear): each pass works at the scale of its own
 * residual and no normalisation is needed.
 *
 * Weights are FP32, layer after layer, each as W[co][ci][ky][kx] (kx along
 * x, tap (kx, ky) reads the point (x + kx - 1, y + ky - 1)); the count is
 * 16*9 + (layers-2)*16*16*9 + 16*9 (fk_net_num_weights).  The caller
 * supplies the initial weights (the library draws no random numbers).
 * Vectors are device float64[n]; calls on one network must not overlap.
 */
enum { FK_NET_RELU = 0, FK_NET_LINEAR = 1 };
fk_status fk_net_num_weights(int32_t layers, int32_t channels, int64_t *count);
fk_status fk_net_create(int32_t layers, int32_t channels, int32_t activation, const float *weights_host,
                        int64_t count, fk_net *out);
fk_status fk_net_destroy(fk_net N);
fk_status fk_net_get_weights(fk_net N, float *weights_host, int64_t count);
/* Replace the weights and reset the optimiser state. */
fk_status fk_net_set_weights(fk_net N, const float *weights_host, int64_t count);

/* Raw network output N(r) for r = b - A (2 u_m - u_{m-1}) into device
 * float32 y[n].  Synchronous. */
fk_status fk_net_forward(fk_net N, fk_csr A, int32_t nx, int32_t ny, const double *b_dev,
                         const double *um_dev, const double *um1_dev, float *y_dev, void *hip_stream);

/*
 * x0 = g + N(b - A g) with g = 2 u_m - u_{m-1}, then passes - 1 more times
 * x0 += N(b - A x0) (1 <= passes <= 16); then the fallback: if
 * ||b - A x0|| > ||b - A u_m|| (or is not finite), x0 = u_m, the previous
 * step's solution.  The guess only changes where the solver starts;
 * fk_solve decides convergence.  Enqueued on hip_stream; if fallback_host
 * is not NULL the call waits and writes 1 there when it fell back, else 0.
 * x0 must not alias the inputs.
 */
fk_status fk_net_guess(fk_net N, fk_csr A, int32_t nx, int32_t ny, const double *b_dev,
                       const double *um_dev, const double *um1_dev, int32_t passes, double *x0_dev,
                       int32_t *fallback_host, void *hip_stream);

/*
 * Training on one sample (b, u_m, u_{m-1}) with known solution u_next:
 * the plane r = b - A g and the target u_next - g are divided by s = max|r|
 * (exact, order-independent), and the loss is mean((N - target)^2) over
 * the grid.  (With u_m = u_{m-1} = 0 the sample is any pair r = b,
 * target u_next.)  fk_net_gradient writes dloss/dweights (canonical order) and the
 * loss to the host without changing the weights; fk_net_train_step takes
 * one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, step size lr) and, if
 * loss_host is not NULL, waits and writes the loss before the step.
 */
fk_status fk_net_gradient(fk_net N, fk_csr A, int32_t nx, int32_t ny, const double *b_dev,
                          const double *um_dev, const double *um1_dev, const double *unext_dev,
                          float *grad_host, double *loss_host, void *hip_stream);
fk_status fk_net_train_step(fk_net N, fk_csr A, int32_t nx, int32_t ny, const double *b_dev,
                            const double *um_dev, const double *um1_dev, const double *unext_dev,
                            float lr, double *loss_host, void *hip_stream);

/*
 * Batched solves: many independent SPD systems of uneven size, each by FP64
 * iterative refinement around FP32 pipelined CG (the arithmetic of
 * FK_CG_MIXED, Algorithm 2 with Eq. (3) inside), all in one persistent
 * launch (an extension for the many small-to-medium systems of Section 1).
 * The batch is one block-diagonal CSR matrix over n = sys_ptr[count] rows:
 * system s owns rows [sys_ptr[s], sys_ptr[s+1]) (at least one) and its rows
 * may reference only its own columns (FK_E_CSR otherwise, checked on the
 * host).  The arrays follow the CSR conventions above and are copied; the
 * caller keeps ownership.
 *
 * fk_batch_solve: b_dev, x_dev are device float64[n] (x holds x0 on entry).
 * Systems are claimed from a largest-first order.  A single workgroup
 * solves a system alone; systems with at most lds_rows rows keep their FP32
 * work vectors in LDS.  With team > 1, `teams` teams of `team` workgroups
 * (0 = as many as the resident workgroups hold; fewer if asked for more)
 * take systems from the large end, each system's rows split into one
 * contiguous chunk per member; the remaining resident workgroups take
 * systems alone from the small end.  A team whose next system fits the LDS
 * limit dissolves: from then on its members solve systems alone.  team = 0
 * chooses teams of 16 when some system has more rows than lds_rows, else no
 * teams.  Team members meet at barriers
 * and all-reduces in device memory; every wait is bounded by spin_limit
 * polls (0 = about 4 M, some seconds).  A wait that runs out aborts every
 * team: systems not solved keep status 3 and the call returns FK_E_HIP
 * (the kernel still ends).  Team and single results are the same, bit for
 * bit.  With
 * FK_FLAG_GRAPH (and a stream other than the default one) the launch is
 * captured once into a hipGraph and replayed while the arguments stay the
 * same.  The call waits for completion.  Per system: converged when
 * ||b_s - A_s x_s|| <= rtol ||b_s||; max_iter counts inner iterations over
 * all sweeps (0 = 10 n_s); b_s = 0 gives x_s = 0.
 */
typedef struct {
    double rtol;        /* >= 0                                              */
    double inner_rtol;  /* >= 0; 0 = 1e-4                                   */
    int32_t max_iter;   /* >= 0; 0 = 10 n_s per system                      */
    int32_t max_outer;  /* >= 0; 0 = 50                                      */
    int32_t workgroup;  /* threads per workgroup: 0 (= 1024), 256, 512, 1024 */
    int32_t lds_rows;   /* LDS-resident limit in rows: 0 = default (6144 or
                           what fits), < 0 = never                           */
    int32_t flags;      /* FK_FLAG_GRAPH                                      */
    int32_t team;       /* workgroups per team, 0..64: 0 = default, 1 = none  */
    int32_t teams;      /* >= 0: number of teams, 0 = default (above)         */
    int32_t spin_limit; /* >= 0: polls a team wait makes, 0 = default        */
} fk_batch_opts;

fk_status fk_batch_create(int32_t count, const int64_t *sys_ptr_host, int64_t nnz, const int32_t *row_ptr,
                          const int32_t *col_idx, const double *vals, int32_t ptr_kind, void *hip_stream,
                          fk_batch *out);
fk_status fk_batch_destroy(fk_batch B);
fk_status fk_batch_shape(fk_batch B, int32_t *count, int64_t *n, int64_t *nnz);
fk_status fk_batch_solve(fk_batch B, const fk_batch_opts *o, const double *b_dev, double *x_dev,
                         void *hip_stream);
/* Per-system results of the last solve into host arrays of `count` entries
 * (each may be NULL): status (0 converged, 1 not converged, 2 breakdown,
 * 3 not solved: a team gave up waiting),
 * inner iterations, refinement sweeps, ||b_s - A_s x_s|| / ||b_s|| of the
 * last residual evaluated. */
fk_status fk_batch_results(fk_batch B, int32_t *status, int32_t *iterations, int32_t *sweeps,
                           double *rel_res);

/*
 * For callers that cannot allocate device memory: code that runs while a HIP
 * graph is being captured, tight serving loops, harnesses that forbid
 * hipMalloc.  fk_solve_noalloc is fk_solve for the pipelined CG method
 * without a solver handle: the same kernels in the same order, hence the
 * same x, k and residual bit for bit as fk_solver_create + fk_solve with
 * the same options.  The call allocates nothing (no hipMalloc, hipFree,
 * pinned host memory, events or graphs): the work vectors r, p, A p, the
 * reduction partials and arrival counters and the device state live in one
 * static array of FK_NOALLOC_BYTES per device (24.4 MiB), which every device
 * that loads the library holds until the process ends.
 *
 * A: a matrix created on the current device with n <= FK_NOALLOC_MAX_N
 * (FK_E_ARG otherwise).  o: method FK_CG_PIPELINED, record_history 0,
 * flags 0 or FK_FLAG_NO_SMALL (FK_E_ARG otherwise); rtol, max_iter and
 * unroll as for fk_solve.  b_dev, x_dev: caller-owned device float64[n], x
 * holding x0 on entry and x_k on return.  iterations and rel_res (either may
 * be NULL) receive k and ||r_k||/||b|| as fk_get_iterations and
 * fk_get_residual would.  Returns FK_OK, FK_NOT_CONVERGED, FK_BREAKDOWN or
 * an error, as fk_solve.  Work runs on hip_stream; the call returns after it
 * has completed.
 *
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (the call clears what must start at zero).  Calls from
 * threads of one process on the same device are serialized by a lock held
 * for the whole call; anything else that overlapped with a call on the same
 * device's array would race with it.
 */
#define FK_NOALLOC_MAX_N 1048576
#define FK_NOALLOC_BYTES 25563392
fk_status fk_solve_noalloc(fk_csr A, const fk_opts *o, const double *b_dev, double *x_dev, void *hip_stream,
                           int32_t *iterations, double *rel_res);

const char *fk_status_str(fk_status s);
const char *fk_last_error(void);

/* Library build identifier (e.g. "fk 0.1 gfx950"). */
const char *fk_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FK_H */
