// Learned initial guess for sequences of related solves (transient problems):
// a small bias-free convolutional network in BF16 on the matrix cores, with
// hand-written inference and training kernels, and its C ABI (include/fk.h).
//
// The network N is a learned local approximate inverse of A on an nx-by-ny
// grid (row = ix + nx*iy): from the residual r = b - A x of a guess x it
// predicts the correction, x <- x + N(r).  A time step starts from the
// extrapolation g = 2 u_m - u_{m-1} of the two previous solutions and may
// apply N more than once (each pass takes the residual left by the previous
// pass).  N is L layers of 3x3 cross-correlation with zero padding and no
// bias, 1 -> C -> ... -> C -> 1 channels, C = 16, with ReLU or the identity
// between layers (the identity makes N a deep linear network, a learned
// linear approximate inverse).  With no bias N(a r) = a N(r) for a > 0 (for
// every a when linear), so inference needs no normalisation and a later
// pass works at the scale of its own (smaller) residual; training divides
// each sample by max|r| (order-independent, exact).
//
// Layout: activations are BF16, pixel-major with 4 (input plane and output,
// padded with zero channels) or 16 (hidden) channels per pixel, so a lane
// fetches 4 channels of one pixel in one 8-byte load.  A 3x3 convolution is an implicit GEMM per 16-pixel
// tile: D[co][px] = sum over (tap, ci) of W[co][ci][tap] * X[px+tap][ci],
// one v_mfma_f32_16x16x16_bf16 per K-slice of 16 (one tap of 16 channels,
// or four taps of 4 channels), FP32 accumulation.  The weight gradient is a
// GEMM over pixels, reduced in a fixed order (workgroup, then a second
// kernel), so training is reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fk.h"
#include "fk_internal.hpp"

namespace fk {
namespace net {

constexpr int NWG = 256;           // threads per workgroup (4 waves)
constexpr int CH = 16;             // hidden channels (one MFMA tile)
constexpr int MAX_LAYERS = 8;
constexpr int DW_GRID = 256;       // workgroups of a weight-gradient launch
constexpr int DW_ELEMS = 9 * CH * CH;  // packed gradient of one layer [tap][co][ci]
constexpr int RED_GRID = 512;      // workgroups of the loss / check reductions

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u)
        return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Pixel of tap t (ky = t / 3, kx = t % 3, offset (kx-1, ky-1)) from the
// pixel at (x, y), or -1 outside the grid (zero padding).
__device__ __forceinline__ int64_t tap_pixel_xy(int x, int y, int t, int nx, int ny)
{
    x += (t % 3) - 1;
    y += (t / 3) - 1;
    if (x < 0 || x >= nx || y < 0 || y >= ny)
        return -1;
    return (int64_t)y * nx + x;
}

__device__ __forceinline__ int64_t tap_pixel(int64_t p, int t, int nx, int ny, int64_t n)
{
    if (p >= n)
        return -1;
    return tap_pixel_xy((int)(p % nx), (int)(p / nx), t, nx, ny);
}

__device__ __forceinline__ bf16x4 load4(const uint16_t *a, int64_t idx)
{
    return *reinterpret_cast<const bf16x4 *>(a + idx);  // idx is a multiple of 4
}

// ------------------------------------------------------------- convolution

enum Epi : int {
    EPI_ACT = 0,    // out = bf16(act(acc)), 16 channels (act: ReLU or identity)
    EPI_MASK = 1,   // out = bf16(acc * act'(mask)), 16 channels (backward data)
    EPI_Y = 2,      // y = acc of channel 0 (FP32 plane)
    EPI_GUESS = 3,  // x0 = (ca xa + cb xb) + acc of channel 0 (FP64)
};

struct ConvArgs {
    int nx, ny;
    int64_t n;
    const uint16_t *in;    // [n][CINP]
    const bf16x4 *w;       // packed operands [J][64]
    uint16_t *out;         // EPI_RELU, EPI_MASK: [n][16]
    const uint16_t *mask;  // EPI_MASK: [n][16]
    float *y;              // EPI_Y
    double *x0;            // EPI_GUESS
    const double *xa, *xb;  // EPI_GUESS: base guess ca xa + cb xb
    double ca, cb;
    int relu;               // EPI_ACT, EPI_MASK: 1 = ReLU, 0 = identity
};

template <int CINP, int EPI>
__global__ __launch_bounds__(NWG) void k_conv(ConvArgs a)
{
    constexpr int J = (9 * CINP + 15) / 16;
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4;
    const int px = lane & 15;
    bf16x4 w[J];
#pragma unroll
    for (int j = 0; j < J; ++j)
        w[j] = a.w[j * 64 + lane];
    const int64_t ntiles = (a.n + 15) / 16;
    const int64_t wave = (int64_t)blockIdx.x * (NWG / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (NWG / 64);
    for (int64_t t = wave; t < ntiles; t += nwaves) {
        const int64_t p = t * 16 + px;
        const int x = (int)(p % a.nx), y = (int)(p / a.nx);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < J; ++j) {
            int tap, c0;
            if constexpr (CINP == 16) {
                tap = j;
                c0 = 4 * grp;
            } else {
                tap = 4 * j + grp;
                c0 = 0;
            }
            bf16x4 b = {0, 0, 0, 0};
            if (tap < 9 && p < a.n) {
                const int64_t q = tap_pixel_xy(x, y, tap, a.nx, a.ny);
                if (q >= 0)
                    b = load4(a.in, q * CINP + c0);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w[j], b, acc, 0, 0, 0);
        }
        if (p >= a.n)
            continue;
        // lane holds channels 4*grp .. 4*grp+3 of pixel p
        if constexpr (EPI == EPI_ACT || EPI == EPI_MASK) {
            bf16x4 o;
            if constexpr (EPI == EPI_MASK) {
                bf16x4 m = {1, 1, 1, 1};
                if (a.relu)
                    m = load4(a.mask, p * 16 + 4 * grp);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    o[i] = (short)((!a.relu || bf2f((uint16_t)m[i]) > 0.f) ? f2bf(acc[i]) : 0);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    o[i] = (short)f2bf((!a.relu || acc[i] > 0.f) ? acc[i] : 0.f);
            }
            *reinterpret_cast<bf16x4 *>(a.out + p * 16 + 4 * grp) = o;
        } else if constexpr (EPI == EPI_Y) {
            if (grp == 0)
                a.y[p] = acc[0];
        } else {
            if (grp == 0)
                a.x0[p] = (a.ca * a.xa[p] + a.cb * a.xb[p]) + (double)acc[0];
        }
    }
}


// ------------------------------------------------------ residual rows

// Nonzeros of a row requested together (with their gathers) before the
// first is added; the sum itself runs left to right in CSR order.
constexpr int RB = 8;

// sum_j a_ij (ca xa_c + cb xb_c) over row i, left to right.
__device__ __forceinline__ double row_base(const DevCsr &A, int64_t i, const double *xa, const double *xb,
                                           double ca, double cb)
{
    const int32_t j0 = A.row_ptr[i], j1 = A.row_ptr[i + 1];
    double q = 0.0;
    for (int32_t j = j0; j < j1; j += RB) {
        int32_t c[RB];
        double v[RB], g[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            c[k] = 0;
            v[k] = 0.0;
            if (j + k < j1) {
                c[k] = A.col_idx[j + k];
                v[k] = A.vals[j + k];
            }
        }
#pragma unroll
        for (int k = 0; k < RB; ++k)
            g[k] = j + k < j1 ? ca * xa[c[k]] + cb * xb[c[k]] : 0.0;
#pragma unroll
        for (int k = 0; k < RB; ++k)
            if (j + k < j1)
                q = q + v[k] * g[k];
    }
    return q;
}

// (sum_j a_ij x_c, sum_j a_ij y_c) over row i, each left to right.
__device__ __forceinline__ void row_dot2(const DevCsr &A, int64_t i, const double *x, const double *y,
                                         double &qx, double &qy)
{
    const int32_t j0 = A.row_ptr[i], j1 = A.row_ptr[i + 1];
    qx = 0.0;
    qy = 0.0;
    for (int32_t j = j0; j < j1; j += RB) {
        int32_t c[RB];
        double v[RB], gx[RB], gy[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            c[k] = 0;
            v[k] = 0.0;
            if (j + k < j1) {
                c[k] = A.col_idx[j + k];
                v[k] = A.vals[j + k];
            }
        }
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            gx[k] = j + k < j1 ? x[c[k]] : 0.0;
            gy[k] = j + k < j1 ? y[c[k]] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            if (j + k < j1) {
                qx = qx + v[k] * gx[k];
                qy = qy + v[k] * gy[k];
            }
        }
    }
}

// ------------------------------------------------ fused inference (one pass)

// One pass x_out = base + N(b - A base), base = ca xa + cb xb, in one launch.
// A workgroup owns a TX x TY tile of the grid.  It forms r = b - A base on
// the tile plus a halo of L points (rows summed left to right, base read
// from global memory, so any CSR works) into LDS, then runs the L layers in
// LDS, each on a region one point smaller than its input, and writes
// base + N on the tile.  Region points outside the grid hold zeros, which is
// the zero padding of the layered kernels; the MFMA slices and BF16 rounding
// points are those of k_conv, so the result equals the layered forward pass
// bit for bit.
constexpr int FTX = 32, FTY = 16;   // output tile
constexpr int FWAVES = 8;           // waves per workgroup

struct FusedArgs {
    DevCsr A;
    int nx, ny, layers, relu;
    const double *b, *xa, *xb;
    double ca, cb;
    double *xout;
    const bf16x4 *w;     // packed forward operands, layer after layer
    int pf[MAX_LAYERS];  // offset of layer l's operands
};

__host__ __device__ constexpr int fused_region(int h) { return (FTX + 2 * h) * (FTY + 2 * h); }
// LDS bytes: r plane (4 channels) on the halo-L region plus two 16-channel
// buffers on the largest hidden region (halo L-1).
inline size_t fused_lds_bytes(int L)
{
    return (size_t)fused_region(L) * 8 + 2 * (size_t)fused_region(L - 1) * 32;
}

// The workgroup's dynamic LDS.  Activations are addressed by offsets into
// it (not by pointers), so every access compiles to ds_read / ds_write.
extern __shared__ __align__(16) uint16_t fused_lds[];

// One layer in LDS: input region of halo h+1 (CINP channels) at element
// offset in_off, output region of halo h at out_off.  LAST: write base + acc
// to xout on the tile.
template <int CINP, bool LAST>
__device__ __forceinline__ void fused_layer(const FusedArgs &a, int in_off, int out_off, int h,
                                            const bf16x4 *w, int gx0, int gy0)
{
    constexpr int J = (9 * CINP + 15) / 16;
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4, px = lane & 15;
    const int wv = threadIdx.x >> 6;
    const int Wo = FTX + 2 * h, Ho = FTY + 2 * h;
    const int Wi = Wo + 2;
    bf16x4 wr[J];
#pragma unroll
    for (int j = 0; j < J; ++j)
        wr[j] = w[j * 64 + lane];
    const int nchunks = (Wo * Ho + 15) / 16;
    for (int c = wv; c < nchunks; c += FWAVES) {
        const int q = c * 16 + px;
        const bool valid = q < Wo * Ho;
        const int qx = valid ? q % Wo : 0, qy = valid ? q / Wo : 0;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < J; ++j) {
            int tap, c0;
            if constexpr (CINP == 16) {
                tap = j;
                c0 = 4 * grp;
            } else {
                tap = 4 * j + grp;
                c0 = 0;
            }
            bf16x4 bv = {0, 0, 0, 0};
            if (tap < 9 && valid) {
                const int ix = qx + (tap % 3), iy = qy + (tap / 3);
                bv = *reinterpret_cast<const bf16x4 *>(&fused_lds[in_off + (iy * Wi + ix) * CINP + c0]);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wr[j], bv, acc, 0, 0, 0);
        }
        if (!valid)
            continue;
        const int gx = gx0 - h + qx, gy = gy0 - h + qy;
        const bool inside = gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny;
        if constexpr (LAST) {
            if (grp == 0 && inside) {
                const int64_t p = (int64_t)gy * a.nx + gx;
                a.xout[p] = (a.ca * a.xa[p] + a.cb * a.xb[p]) + (double)acc[0];
            }
        } else {
            bf16x4 o = {0, 0, 0, 0};
            if (inside) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    o[i] = (short)f2bf((!a.relu || acc[i] > 0.f) ? acc[i] : 0.f);
            }
            *reinterpret_cast<bf16x4 *>(&fused_lds[out_off + q * 16 + 4 * grp]) = o;
        }
    }
}

__global__ __launch_bounds__(FWAVES * 64) void k_net_fused(FusedArgs a)
{
    const int L = a.layers;
    const int tiles_x = (a.nx + FTX - 1) / FTX;
    const int gx0 = (int)(blockIdx.x % tiles_x) * FTX;
    const int gy0 = (int)(blockIdx.x / tiles_x) * FTY;
    // r plane at element 0, then two 16-channel buffers
    const int buf[2] = {fused_region(L) * 4, fused_region(L) * 4 + fused_region(L - 1) * 16};
    // r = b - A base on the halo-L region (zeros outside the grid)
    const int Wr = FTX + 2 * L, Hr = FTY + 2 * L;
    for (int q = threadIdx.x; q < Wr * Hr; q += FWAVES * 64) {
        const int gx = gx0 - L + q % Wr, gy = gy0 - L + q / Wr;
        bf16x4 o = {0, 0, 0, 0};
        if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny) {
            const int64_t i = (int64_t)gy * a.nx + gx;
            const double acc = row_base(a.A, i, a.xa, a.xb, a.ca, a.cb);
            o[0] = (short)f2bf((float)(a.b[i] - acc));
        }
        *reinterpret_cast<bf16x4 *>(&fused_lds[q * 4]) = o;
    }
    __syncthreads();
    int in = 0;
    for (int l = 0; l < L; ++l) {
        const int h = L - 1 - l;
        const int out = buf[l & 1];
        const bf16x4 *w = a.w + a.pf[l];
        if (l == L - 1)
            fused_layer<16, true>(a, in, 0, h, w, gx0, gy0);
        else if (l == 0)
            fused_layer<4, false>(a, in, out, h, w, gx0, gy0);
        else
            fused_layer<16, false>(a, in, out, h, w, gx0, gy0);
        __syncthreads();
        in = out;
    }
}

// ------------------------------------------------------- weight gradient

// Partial dW[tap][co][ci] = sum over pixels p of G[p][co] * X[p + tap][ci]
// for this workgroup's tiles: one MFMA per tap and 16-pixel tile (K =
// pixels).  The four waves are summed in wave order in LDS.
template <int CINP, int GP>
__global__ __launch_bounds__(NWG) void k_dw(int nx, int ny, int64_t n, const uint16_t *act,
                                              const uint16_t *g, float *partials)
{
    __shared__ float red[DW_ELEMS];
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4;
    const int col = lane & 15;  // row co of A, column ci of B
    const int wv = threadIdx.x >> 6;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t)
        acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int64_t ntiles = (n + 15) / 16;
    const int64_t wave = (int64_t)blockIdx.x * (NWG / 64) + wv;
    const int64_t nwaves = (int64_t)gridDim.x * (NWG / 64);
    for (int64_t t = wave; t < ntiles; t += nwaves) {
        const int64_t p0 = t * 16 + 4 * grp;
        bf16x4 av = {0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (col < GP && p0 + q < n)
                av[q] = (short)g[(p0 + q) * GP + col];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            bf16x4 bv = {0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t s = tap_pixel(p0 + q, tap, nx, ny, n);
                if (col < CINP && s >= 0)
                    bv[q] = (short)act[s * CINP + col];
            }
            acc[tap] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[tap], 0, 0, 0);
        }
    }
    // acc[tap][i] = D[co = 4*grp + i][ci = col]
    for (int w = 0; w < NWG / 64; ++w) {
        if (wv == w) {
#pragma unroll
            for (int tap = 0; tap < 9; ++tap)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int e = tap * 256 + (4 * grp + i) * 16 + col;
                    red[e] = (w == 0) ? acc[tap][i] : red[e] + acc[tap][i];
                }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < DW_ELEMS; e += NWG)
        partials[(size_t)blockIdx.x * DW_ELEMS + e] = red[e];
}

struct LayerMeta {
    int cin, cout, cinp, coutp;
    int woff;    // offset of W[co][ci][ky][kx] in the canonical weight vector
    int jf, jt;  // MFMA slices of the forward / transposed operands
    int pf, pt;  // offsets (in bf16x4) of the packed forward / transposed operands
};
struct NetMeta {
    int layers;
    int relu;  // 1: ReLU between layers, 0: identity
    int nweights;
    LayerMeta l[MAX_LAYERS];
};

// Second stage: grad[canonical] = sum over workgroups, in workgroup order.
__global__ __launch_bounds__(NWG) void k_dw_reduce(const float *partials, int nparts, LayerMeta m,
                                                   float *grad)
{
    for (int e = blockIdx.x * NWG + threadIdx.x; e < DW_ELEMS; e += gridDim.x * NWG) {
        const int tap = e / 256, co = (e / 16) % 16, ci = e % 16;
        if (co >= m.cout || ci >= m.cin)
            continue;
        float s = 0.f;
        for (int w = 0; w < nparts; ++w)
            s += partials[(size_t)w * DW_ELEMS + e];
        grad[m.woff + (co * m.cin + ci) * 9 + tap] = s;
    }
}

// ------------------------------------------------- weights: Adam and packing

__global__ __launch_bounds__(NWG) void k_adam(int count, float *w, float *mo, float *ve,
                                              const float *g, float lr, float c1, float c2)
{
    constexpr float B1 = 0.9f, B2 = 0.999f, EPS = 1e-8f;
    for (int i = blockIdx.x * NWG + threadIdx.x; i < count; i += gridDim.x * NWG) {
        const float gi = g[i];
        const float m = B1 * mo[i] + (1.f - B1) * gi;
        const float v = B2 * ve[i] + (1.f - B2) * gi * gi;
        mo[i] = m;
        ve[i] = v;
        w[i] = w[i] - lr * (m / c1) / (sqrtf(v / c2) + EPS);
    }
}

// MFMA A operands in lane order.  Lane L, item q holds row i = L % 16 and
// K index k = 4 (L / 16) + q of slice j.  Forward: row = output channel,
// k = (tap, input channel).  Transposed (backward data of layer l): row =
// input channel of l, k = (tap', output channel of l), weight of the
// mirrored tap 8 - tap'.
__global__ __launch_bounds__(NWG) void k_pack(NetMeta nm, const float *wcan, bf16x4 *packed)
{
    for (int l = 0; l < nm.layers; ++l) {
        const LayerMeta m = nm.l[l];
        const int nf = m.jf * 64, nt = m.jt * 64;
        for (int e = blockIdx.x * NWG + threadIdx.x; e < nf + nt; e += gridDim.x * NWG) {
            const bool tr = e >= nf;
            const int idx = tr ? e - nf : e;
            const int j = idx / 64, L = idx % 64;
            const int row = L % 16;
            const int kp = tr ? m.coutp : m.cinp;  // channels per tap of this operand
            bf16x4 o;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 4 * (L / 16) + q;
                const int tap = kp == 16 ? j : 4 * j + k / 4;
                const int ch = kp == 16 ? k : k % 4;
                float v = 0.f;
                if (tap < 9) {
                    if (!tr && row < m.cout && ch < m.cin)
                        v = wcan[m.woff + (row * m.cin + ch) * 9 + tap];
                    if (tr && ch < m.cout && row < m.cin)
                        v = wcan[m.woff + (ch * m.cin + row) * 9 + (8 - tap)];
                }
                o[q] = (short)f2bf(v);
            }
            packed[(tr ? m.pt : m.pf) + idx] = o;
        }
    }
}

// ------------------------------------------------------------- features

enum FeatMode : int {
    FEAT_RAW = 0,   // inference: the plane r as it is
    FEAT_SCAN = 1,  // training, pass 1: r to rbuf, max |r| to *maxbits
    FEAT_NORM = 2,  // training, pass 2: plane and target divided by max |r|
};

// One thread per row.  The base guess x = ca xa + cb xb is formed at every
// column the row touches; r = b - A x with the row summed left to right.
// Input plane [n][4] = (r, 0, 0, 0).
template <int MODE>
__global__ __launch_bounds__(NWG) void k_features(DevCsr A, const double *b, const double *xa,
                                                  const double *xb, double ca, double cb,
                                                  const double *unext, double *rbuf,
                                                  unsigned long long *maxbits, uint16_t *feat,
                                                  float *target)
{
    const int64_t n = A.n;
    for (int64_t i = (int64_t)blockIdx.x * NWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * NWG) {
        double r;
        if constexpr (MODE == FEAT_NORM) {
            r = rbuf[i];
        } else {
            r = b[i] - row_base(A, i, xa, xb, ca, cb);
        }
        if constexpr (MODE == FEAT_SCAN) {
            rbuf[i] = r;
            atomicMax(maxbits, (unsigned long long)__double_as_longlong(fabs(r)));
            continue;
        }
        double s = 1.0;
        if constexpr (MODE == FEAT_NORM) {
            s = __longlong_as_double((long long)*maxbits);
            if (!(s > 0.0))
                s = 1.0;
            target[i] = (float)((unext[i] - (ca * xa[i] + cb * xb[i])) / s);
        }
        bf16x4 o = {0, 0, 0, 0};
        o[0] = (short)f2bf((float)(r / s));
        *reinterpret_cast<bf16x4 *>(feat + i * 4) = o;
    }
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

// ---------------------------------------------------------- loss, check

__device__ __forceinline__ double wg_sum(double v, double *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = NWG / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

// Mean squared error of y against target; dy = 2 (y - t) / n into channel 0
// of the output gradient plane ([n][4] BF16).
__global__ __launch_bounds__(NWG) void k_loss(int64_t n, const float *y, const float *t, uint16_t *gout,
                                              double *partials)
{
    __shared__ double lds[NWG];
    double acc = 0.0;
    const float inv = 2.0f / (float)n;
    for (int64_t i = (int64_t)blockIdx.x * NWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * NWG) {
        const float d = y[i] - t[i];
        acc += (double)d * (double)d;
        bf16x4 o = {0, 0, 0, 0};
        o[0] = (short)f2bf(d * inv);
        *reinterpret_cast<bf16x4 *>(gout + i * 4) = o;
    }
    const double s = wg_sum(acc, lds);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(NWG) void k_loss_final(int nparts, const double *partials, int64_t n,
                                                    double *loss)
{
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < nparts; ++w)
            s += partials[w];
        *loss = s / (double)n;
    }
}

// ||b - A x0||^2 and ||b - A u_m||^2, per workgroup.
__global__ __launch_bounds__(NWG) void k_check(DevCsr A, const double *b, const double *x0,
                                               const double *um, double *partials)
{
    __shared__ double lds[NWG];
    double a0 = 0.0, a1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NWG + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * NWG) {
        double q0, q1;
        row_dot2(A, i, x0, um, q0, q1);
        const double r0 = b[i] - q0, r1 = b[i] - q1;
        a0 += r0 * r0;
        a1 += r1 * r1;
    }
    const double s0 = wg_sum(a0, lds);
    const double s1 = wg_sum(a1, lds);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s0;
        partials[2 * blockIdx.x + 1] = s1;
    }
}

// Fallback decision: flag[0] = 1 when the residual of x0 is larger than
// that of u_m (or not finite).  One workgroup sums the partials of k_check,
// thread t taking partials t, t + NWG, ..., then a fixed tree.
__global__ __launch_bounds__(NWG) void k_select(int nparts, const double *partials, int32_t *flag)
{
    __shared__ double lds[NWG];
    double a0 = 0.0, a1 = 0.0;
    for (int w = threadIdx.x; w < nparts; w += NWG) {
        a0 += partials[2 * w];
        a1 += partials[2 * w + 1];
    }
    const double r0 = wg_sum(a0, lds);
    const double r1 = wg_sum(a1, lds);
    if (threadIdx.x == 0)
        *flag = (!(r0 <= r1)) ? 1 : 0;
}

// x0 = u_m where k_select fell back; returns at once otherwise.
__global__ __launch_bounds__(NWG) void k_fallback(int64_t n, const int32_t *flag, const double *um,
                                                  double *x0)
{
    if (*flag == 0)
        return;
    for (int64_t i = (int64_t)blockIdx.x * NWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * NWG)
        x0[i] = um[i];
}

}  // namespace net
}  // namespace fk

// =================================================================== host

using namespace fk;
using namespace fk::net;

struct fk_net_s {
    NetMeta meta{};
    int device = 0;
    float *w = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;  // canonical FP32
    bf16x4 *packed = nullptr;
    int npacked = 0;
    long adam_t = 0;
    // per-grid workspace
    int64_t cap = 0;
    uint16_t *feat = nullptr;             // [n][4]
    uint16_t *act[MAX_LAYERS] = {};       // act[l], l = 1..L-1: [n][16]
    uint16_t *g16[2] = {nullptr, nullptr};  // [n][16] gradient ping-pong
    uint16_t *g4 = nullptr;               // [n][4] output gradient
    float *y = nullptr, *target = nullptr;
    double *rbuf = nullptr;
    unsigned long long *maxbits = nullptr;
    float *dwpart = nullptr;
    double *redpart = nullptr, *loss = nullptr;
    int32_t *flag = nullptr;
    double *xtmp = nullptr;               // [n] ping-pong iterate of multi-pass guesses
};

namespace {

fk_status net_fail(fk_status s, const char *msg) { return internal_fail(s, "%s", msg); }

#define NET_HIP(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return internal_fail(FK_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

bool make_meta(int layers, int channels, int activation, NetMeta *nm)
{
    if (layers < 2 || layers > MAX_LAYERS || channels != CH ||
        (activation != FK_NET_RELU && activation != FK_NET_LINEAR))
        return false;
    nm->layers = layers;
    nm->relu = activation == FK_NET_RELU ? 1 : 0;
    int woff = 0, pk = 0;
    for (int l = 0; l < layers; ++l) {
        LayerMeta &m = nm->l[l];
        m.cin = l == 0 ? 1 : CH;
        m.cinp = l == 0 ? 4 : 16;
        m.cout = l == layers - 1 ? 1 : CH;
        m.coutp = l == layers - 1 ? 4 : 16;
        m.woff = woff;
        woff += m.cout * m.cin * 9;
        m.jf = (9 * m.cinp + 15) / 16;
        m.jt = (9 * m.coutp + 15) / 16;
        m.pf = pk;
        pk += m.jf * 64;
        m.pt = pk;
        pk += m.jt * 64;
    }
    nm->nweights = woff;
    return true;
}

template <typename T>
void dfree(T *&p)
{
    if (p)
        (void)hipFree(p);
    p = nullptr;
}

void release_workspace(fk_net N)
{
    dfree(N->feat);
    for (auto &a : N->act)
        dfree(a);
    dfree(N->g16[0]);
    dfree(N->g16[1]);
    dfree(N->g4);
    dfree(N->y);
    dfree(N->target);
    dfree(N->rbuf);
    dfree(N->maxbits);
    dfree(N->dwpart);
    dfree(N->redpart);
    dfree(N->loss);
    dfree(N->flag);
    dfree(N->xtmp);
    N->cap = 0;
}

template <typename T>
hipError_t dalloc(T **p, size_t count)
{
    return hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(count, 1) * sizeof(T));
}

fk_status ensure_workspace(fk_net N, int64_t n)
{
    if (N->cap >= n)
        return FK_OK;
    release_workspace(N);
    const size_t un = (size_t)n;
    hipError_t e = hipSuccess;
    e = e ? e : dalloc(&N->feat, un * 4);
    for (int l = 1; l < N->meta.layers && e == hipSuccess; ++l)
        e = dalloc(&N->act[l], un * 16);
    e = e ? e : dalloc(&N->g16[0], un * 16);
    e = e ? e : dalloc(&N->g16[1], un * 16);
    e = e ? e : dalloc(&N->g4, un * 4);
    e = e ? e : dalloc(&N->y, un);
    e = e ? e : dalloc(&N->target, un);
    e = e ? e : dalloc(&N->rbuf, un);
    e = e ? e : dalloc(&N->maxbits, 1);
    e = e ? e : dalloc(&N->dwpart, (size_t)DW_GRID * DW_ELEMS);
    e = e ? e : dalloc(&N->redpart, (size_t)2 * RED_GRID);
    e = e ? e : dalloc(&N->loss, 1);
    e = e ? e : dalloc(&N->flag, 1);
    e = e ? e : dalloc(&N->xtmp, un);
    if (e != hipSuccess) {
        release_workspace(N);
        return e == hipErrorOutOfMemory ? net_fail(FK_E_OOM, "network workspace: out of device memory")
                                        : internal_fail(FK_E_HIP, "network workspace: %s", hipGetErrorString(e));
    }
    N->cap = n;
    return FK_OK;
}

int grid_for(int64_t work, int per, int cap)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (work + per - 1) / per));
}

fk_status check_grid(fk_net N, fk_csr A, int32_t nx, int32_t ny, DevCsr *view)
{
    if (!N || !A)
        return net_fail(FK_E_ARG, "NULL network or matrix");
    if (nx < 1 || ny < 1)
        return net_fail(FK_E_ARG, "grid sides must be >= 1");
    *view = internal_csr_view(A);
    if ((int64_t)nx * ny != (int64_t)view->n)
        return internal_fail(FK_E_ARG, "grid %d x %d does not match n = %d", nx, ny, view->n);
    return ensure_workspace(N, view->n);
}

// Forward through all layers from N->feat; the last layer writes y
// (x0 == nullptr) or x0 = (ca xa + cb xb) + y.
hipError_t forward(fk_net N, int nx, int ny, int64_t n, double *x0, const double *xa, const double *xb,
                   double ca, double cb, hipStream_t s)
{
    const int L = N->meta.layers;
    const int grid = grid_for((n + 15) / 16, NWG / 64, 4096);
    const uint16_t *in = N->feat;
    for (int l = 0; l < L; ++l) {
        const LayerMeta &m = N->meta.l[l];
        ConvArgs a{nx, ny, n, in, N->packed + m.pf, nullptr, nullptr, nullptr, nullptr, xa, xb, ca, cb,
                   N->meta.relu};
        if (l < L - 1) {
            a.out = N->act[l + 1];
            if (l == 0)
                hipLaunchKernelGGL((k_conv<4, EPI_ACT>), dim3(grid), dim3(NWG), 0, s, a);
            else
                hipLaunchKernelGGL((k_conv<16, EPI_ACT>), dim3(grid), dim3(NWG), 0, s, a);
            in = N->act[l + 1];
        } else if (x0) {
            a.x0 = x0;
            hipLaunchKernelGGL((k_conv<16, EPI_GUESS>), dim3(grid), dim3(NWG), 0, s, a);
        } else {
            a.y = N->y;
            hipLaunchKernelGGL((k_conv<16, EPI_Y>), dim3(grid), dim3(NWG), 0, s, a);
        }
    }
    return hipGetLastError();
}

// Normalised features and target of one training sample, forward, loss and
// backward: the gradient lands in N->grad, the loss in N->loss.
hipError_t loss_and_gradient(fk_net N, const DevCsr &A, int nx, int ny, const double *b, const double *um,
                             const double *um1, const double *unext, hipStream_t s)
{
    const int64_t n = A.n;
    const int L = N->meta.layers;
    const int gv = grid_for(n, NWG, 2048);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, N->maxbits);
    hipLaunchKernelGGL((k_features<FEAT_SCAN>), dim3(gv), dim3(NWG), 0, s, A, b, um, um1, 2.0, -1.0, unext,
                       N->rbuf, N->maxbits, N->feat, N->target);
    hipLaunchKernelGGL((k_features<FEAT_NORM>), dim3(gv), dim3(NWG), 0, s, A, b, um, um1, 2.0, -1.0, unext,
                       N->rbuf, N->maxbits, N->feat, N->target);
    hipError_t e = forward(N, nx, ny, n, nullptr, um, um1, 2.0, -1.0, s);
    if (e != hipSuccess)
        return e;
    const int gl = grid_for(n, NWG, RED_GRID);
    hipLaunchKernelGGL(k_loss, dim3(gl), dim3(NWG), 0, s, n, N->y, N->target, N->g4, N->redpart);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(NWG), 0, s, gl, N->redpart, n, N->loss);
    const int gc = grid_for((n + 15) / 16, NWG / 64, 4096);
    const uint16_t *gcur = N->g4;  // gradient w.r.t. the output of layer l
    int pp = 0;
    for (int l = L - 1; l >= 0; --l) {
        const LayerMeta &m = N->meta.l[l];
        const uint16_t *act = l == 0 ? N->feat : N->act[l];
        if (l == 0)
            hipLaunchKernelGGL((k_dw<4, 16>), dim3(DW_GRID), dim3(NWG), 0, s, nx, ny, n, act, gcur, N->dwpart);
        else if (l == L - 1)
            hipLaunchKernelGGL((k_dw<16, 4>), dim3(DW_GRID), dim3(NWG), 0, s, nx, ny, n, act, gcur, N->dwpart);
        else
            hipLaunchKernelGGL((k_dw<16, 16>), dim3(DW_GRID), dim3(NWG), 0, s, nx, ny, n, act, gcur, N->dwpart);
        hipLaunchKernelGGL(k_dw_reduce, dim3(DW_ELEMS / NWG), dim3(NWG), 0, s, N->dwpart, DW_GRID, m, N->grad);
        if (l > 0) {
            ConvArgs a{nx, ny, n, gcur, N->packed + m.pt, N->g16[pp], N->act[l], nullptr, nullptr, nullptr, nullptr,
                       0.0, 0.0, N->meta.relu};
            if (l == L - 1)
                hipLaunchKernelGGL((k_conv<4, EPI_MASK>), dim3(gc), dim3(NWG), 0, s, a);
            else
                hipLaunchKernelGGL((k_conv<16, EPI_MASK>), dim3(gc), dim3(NWG), 0, s, a);
            gcur = N->g16[pp];
            pp ^= 1;
        }
    }
    return hipGetLastError();
}

hipError_t pack(fk_net N, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack, dim3(grid_for(N->npacked, NWG, 64)), dim3(NWG), 0, s, N->meta, N->w, N->packed);
    return hipGetLastError();
}

}  // namespace

extern "C" fk_status fk_net_num_weights(int32_t layers, int32_t channels, int64_t *count)
{
    NetMeta nm{};
    if (!count)
        return net_fail(FK_E_ARG, "NULL argument");
    if (!make_meta(layers, channels, FK_NET_RELU, &nm))
        return net_fail(FK_E_ARG, "layers must be in [2, 8] and channels 16");
    *count = nm.nweights;
    return FK_OK;
}

extern "C" fk_status fk_net_create(int32_t layers, int32_t channels, int32_t activation, const float *weights,
                                   int64_t count, fk_net *out)
{
    if (!out)
        return net_fail(FK_E_ARG, "out is NULL");
    *out = nullptr;
    NetMeta nm{};
    if (!make_meta(layers, channels, activation, &nm))
        return net_fail(FK_E_ARG, "layers must be in [2, 8], channels 16, activation FK_NET_RELU or FK_NET_LINEAR");
    if (!weights || count != nm.nweights)
        return internal_fail(FK_E_ARG, "expected %d initial weights", nm.nweights);
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(weights[i]))
            return net_fail(FK_E_ARG, "initial weights must be finite");
    fk_net N = new (std::nothrow) fk_net_s;
    if (!N)
        return net_fail(FK_E_OOM, "host allocation failed");
    N->meta = nm;
    N->npacked = nm.l[layers - 1].pt + nm.l[layers - 1].jt * 64;
    (void)hipGetDevice(&N->device);
    const size_t nw = (size_t)nm.nweights;
    hipError_t e = dalloc(&N->w, nw);
    e = e ? e : dalloc(&N->m, nw);
    e = e ? e : dalloc(&N->v, nw);
    e = e ? e : dalloc(&N->grad, nw);
    e = e ? e : dalloc(&N->packed, (size_t)N->npacked);
    e = e ? e : hipMemcpy(N->w, weights, nw * 4, hipMemcpyHostToDevice);
    e = e ? e : hipMemset(N->m, 0, nw * 4);
    e = e ? e : hipMemset(N->v, 0, nw * 4);
    e = e ? e : hipMemset(N->grad, 0, nw * 4);
    e = e ? e : pack(N, nullptr);
    e = e ? e : hipDeviceSynchronize();
    if (e != hipSuccess) {
        fk_net_destroy(N);
        return internal_fail(FK_E_HIP, "fk_net_create: %s", hipGetErrorString(e));
    }
    *out = N;
    return FK_OK;
}

extern "C" fk_status fk_net_destroy(fk_net N)
{
    if (!N)
        return net_fail(FK_E_ARG, "NULL network");
    (void)hipDeviceSynchronize();
    release_workspace(N);
    dfree(N->w);
    dfree(N->m);
    dfree(N->v);
    dfree(N->grad);
    dfree(N->packed);
    delete N;
    return FK_OK;
}

extern "C" fk_status fk_net_get_weights(fk_net N, float *out, int64_t count)
{
    if (!N || !out || count != N->meta.nweights)
        return net_fail(FK_E_ARG, "bad argument");
    NET_HIP(hipMemcpy(out, N->w, (size_t)count * 4, hipMemcpyDeviceToHost));
    return FK_OK;
}

extern "C" fk_status fk_net_set_weights(fk_net N, const float *w, int64_t count)
{
    if (!N || !w || count != N->meta.nweights)
        return net_fail(FK_E_ARG, "bad argument");
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(w[i]))
            return net_fail(FK_E_ARG, "weights must be finite");
    NET_HIP(hipDeviceSynchronize());
    NET_HIP(hipMemcpy(N->w, w, (size_t)count * 4, hipMemcpyHostToDevice));
    NET_HIP(hipMemset(N->m, 0, (size_t)count * 4));
    NET_HIP(hipMemset(N->v, 0, (size_t)count * 4));
    N->adam_t = 0;
    NET_HIP(pack(N, nullptr));
    NET_HIP(hipDeviceSynchronize());
    return FK_OK;
}

extern "C" fk_status fk_net_forward(fk_net N, fk_csr Ah, int32_t nx, int32_t ny, const double *b,
                                    const double *um, const double *um1, float *y, void *stream)
{
    DevCsr A;
    fk_status st = check_grid(N, Ah, nx, ny, &A);
    if (st != FK_OK)
        return st;
    if (!b || !um || !um1 || !y)
        return net_fail(FK_E_ARG, "NULL vector");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = A.n;
    hipLaunchKernelGGL((k_features<FEAT_RAW>), dim3(grid_for(n, NWG, 2048)), dim3(NWG), 0, s, A, b, um, um1,
                       2.0, -1.0, nullptr, nullptr, nullptr, N->feat, nullptr);
    NET_HIP(forward(N, nx, ny, n, nullptr, um, um1, 2.0, -1.0, s));
    NET_HIP(hipMemcpyAsync(y, N->y, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    NET_HIP(hipStreamSynchronize(s));
    return FK_OK;
}

extern "C" fk_status fk_net_guess(fk_net N, fk_csr Ah, int32_t nx, int32_t ny, const double *b,
                                  const double *um, const double *um1, int32_t passes, double *x0,
                                  int32_t *fallback, void *stream)
{
    DevCsr A;
    fk_status st = check_grid(N, Ah, nx, ny, &A);
    if (st != FK_OK)
        return st;
    if (!b || !um || !um1 || !x0)
        return net_fail(FK_E_ARG, "NULL vector");
    if (x0 == um || x0 == um1 || x0 == b)
        return net_fail(FK_E_ARG, "x0 must not alias b, u_m or u_m1");
    if (passes < 1 || passes > 16)
        return net_fail(FK_E_ARG, "passes must be in [1, 16]");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = A.n;
    // One fused launch per pass.  A pass reads its base around every point
    // of its tile while other tiles write their output, so consecutive
    // passes alternate between x0 and a workspace vector, the last one
    // writing x0.
    FusedArgs fa{};
    fa.A = A;
    fa.nx = nx;
    fa.ny = ny;
    fa.layers = N->meta.layers;
    fa.relu = N->meta.relu;
    fa.b = b;
    fa.w = N->packed;
    for (int l = 0; l < N->meta.layers; ++l)
        fa.pf[l] = N->meta.l[l].pf;
    const int tiles = ((nx + FTX - 1) / FTX) * ((ny + FTY - 1) / FTY);
    const size_t lds = fused_lds_bytes(N->meta.layers);
    double *bufs[2] = {x0, N->xtmp};
    for (int k = 0; k < passes; ++k) {
        const int dst = (passes - 1 - k) & 1;
        if (k == 0) {
            fa.xa = um;
            fa.xb = um1;
            fa.ca = 2.0;
            fa.cb = -1.0;
        } else {
            fa.xa = fa.xb = bufs[dst ^ 1];
            fa.ca = 1.0;
            fa.cb = 0.0;
        }
        fa.xout = bufs[dst];
        hipLaunchKernelGGL(k_net_fused, dim3(tiles), dim3(FWAVES * 64), lds, s, fa);
    }
    NET_HIP(hipGetLastError());
    const int gr = grid_for(n, NWG, RED_GRID);
    hipLaunchKernelGGL(k_check, dim3(gr), dim3(NWG), 0, s, A, b, x0, um, N->redpart);
    hipLaunchKernelGGL(k_select, dim3(1), dim3(NWG), 0, s, gr, N->redpart, N->flag);
    hipLaunchKernelGGL(k_fallback, dim3(gr), dim3(NWG), 0, s, n, N->flag, um, x0);
    NET_HIP(hipGetLastError());
    if (fallback) {
        NET_HIP(hipMemcpyAsync(fallback, N->flag, 4, hipMemcpyDeviceToHost, s));
        NET_HIP(hipStreamSynchronize(s));
    }
    return FK_OK;
}

extern "C" fk_status fk_net_gradient(fk_net N, fk_csr Ah, int32_t nx, int32_t ny, const double *b,
                                     const double *um, const double *um1, const double *unext, float *grad,
                                     double *loss, void *stream)
{
    DevCsr A;
    fk_status st = check_grid(N, Ah, nx, ny, &A);
    if (st != FK_OK)
        return st;
    if (!b || !um || !um1 || !unext || !grad || !loss)
        return net_fail(FK_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    NET_HIP(loss_and_gradient(N, A, nx, ny, b, um, um1, unext, s));
    NET_HIP(hipMemcpyAsync(grad, N->grad, (size_t)N->meta.nweights * 4, hipMemcpyDeviceToHost, s));
    NET_HIP(hipMemcpyAsync(loss, N->loss, 8, hipMemcpyDeviceToHost, s));
    NET_HIP(hipStreamSynchronize(s));
    return FK_OK;
}

extern "C" fk_status fk_net_train_step(fk_net N, fk_csr Ah, int32_t nx, int32_t ny, const double *b,
                                       const double *um, const double *um1, const double *unext, float lr,
                                       double *loss, void *stream)
{
    DevCsr A;
    fk_status st = check_grid(N, Ah, nx, ny, &A);
    if (st != FK_OK)
        return st;
    if (!b || !um || !um1 || !unext)
        return net_fail(FK_E_ARG, "NULL vector");
    if (!(lr > 0.f) || !std::isfinite(lr))
        return net_fail(FK_E_ARG, "learning rate must be finite and > 0");
    hipStream_t s = (hipStream_t)stream;
    NET_HIP(loss_and_gradient(N, A, nx, ny, b, um, um1, unext, s));
    N->adam_t++;
    const float c1 = 1.f - std::pow(0.9f, (float)N->adam_t);
    const float c2 = 1.f - std::pow(0.999f, (float)N->adam_t);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(N->meta.nweights, NWG, 64)), dim3(NWG), 0, s, N->meta.nweights,
                       N->w, N->m, N->v, N->grad, lr, c1, c2);
    NET_HIP(pack(N, s));
    if (loss) {
        NET_HIP(hipMemcpyAsync(loss, N->loss, 8, hipMemcpyDeviceToHost, s));
        NET_HIP(hipStreamSynchronize(s));
    }
    return FK_OK;
}
