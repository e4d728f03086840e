// C ABI of libfk.so (declared in include/fk.h): CSR validation and row-block
// planning on the host, device workspace, and the host drivers that enqueue
// the per-iteration kernel sequences of Algorithms 1-4 (Sections 3.1, 3.2).
//
// The drivers never wait for a scalar inside an iteration: every scalar
// (alpha, beta, omega, the convergence test) is evaluated on the device by
// the last workgroup of each reduction point.  The host enqueues `unroll`
// iterations at a time, keeps one batch in flight ahead of the one it is
// waiting for, and reads back a single status word per batch; kernels
// enqueued after convergence return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fk.h"
#include "fk_internal.hpp"

using namespace fk;

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

static fk_status fail(fk_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

fk_status fk::internal_fail(fk_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(FK_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

static fk_status oom_or_hip(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(FK_E_OOM, "%s: out of device memory", what);
    return fail(FK_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

template <typename T>
static fk_status dev_alloc(T **p, size_t count, const char *what)
{
    *p = nullptr;
    if (count == 0)
        count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return oom_or_hip(e, what);
    }
    return FK_OK;
}

template <typename T>
static void dev_free(T *&p)
{
    if (p)
        (void)hipFree(p);
    p = nullptr;
}

// ------------------------------------------------------------- launch shape

static int env_int(const char *name, int dflt, int lo, int hi)
{
    const char *s = getenv(name);
    if (!s || !*s)
        return dflt;
    long v = strtol(s, nullptr, 10);
    return (int)std::min<long>(hi, std::max<long>(lo, v));
}

// Workgroups of a product launch, a multiple of 8 so that every XCD owns
// the same number of them, at most FK_SPMV_GRID when that is set.
//  - Row blocks: one block per workgroup up to 2048 (eight 256-thread
//    workgroups per CU of the 256-CU part), each taking a contiguous chunk.
//  - Sliced: two slices per wave.  Measured on MI355X, that beats one and
//    four on the 128^3 Poisson matrix (32768 slices) and on the 1024^2
//    convection-diffusion matrix (16384 slices) alike.
static int spmv_grid(bool sliced, int64_t units)
{
    static const int gcap = env_int("FK_SPMV_GRID", GMAX, 8, GMAX);
    int64_t g = sliced ? (units + 2 * WAVES - 1) / (2 * WAVES) : std::min<int64_t>(units, 2048);
    g = std::min<int64_t>(g, gcap);
    if (g >= 8)
        g &= ~7;
    return (int)std::max<int64_t>(g, 1);
}

static int vec_grid(int64_t n)
{
    static const int gmax = env_int("FK_VEC_GRID", 1024, 1, GMAX);
    int64_t g = (n + WG - 1) / WG;
    g = std::min<int64_t>(g, gmax);
    return (int)std::max<int64_t>(g, 1);
}

// ------------------------------------------------------------------ matrix

struct fk_csr_s {
    int64_t n = 0, nnz = 0;
    int32_t *row_ptr = nullptr, *col_idx = nullptr, *blocks = nullptr, *block_j0 = nullptr;
    double *vals = nullptr;
    int32_t nblocks = 0;
    int32_t long_rows = 0;
    int device = 0;
    // sliced layout (built when it pays, or on request); sell_off4 exists
    // when every column is within 32767 of its row
    int32_t *sell_ptr = nullptr, *sell_col = nullptr, *sell_ptr4 = nullptr;
    short4 *sell_off4 = nullptr;
    double *sell_vals = nullptr;
    int32_t nslices = 0;      // > 0 once the sliced arrays exist
    int64_t sell_entries = 0;
    // slot layout (built when every slice has few distinct column offsets)
    int32_t *dg_ptr = nullptr, *dg_off = nullptr;
    uint32_t *dg_mask = nullptr;
    double *dg_vals = nullptr;
    int32_t dg_nslices = 0;   // > 0 once the slot arrays exist
    int32_t dg_max_width = 0;    // most slots of any slice
    int32_t sell_max_width = 0;  // most entries per row of any slice (sliced layouts)
    int64_t dg_entries = 0;
    int32_t layout = FK_LAYOUT_ROW_BLOCKS;  // layout the products read
    // scratch reduction state for fk_spmv / fk_spmv32
    DevState *st = nullptr;
    double *partials = nullptr;
    int solvers = 0;
    // FP32 values for fk_spmv32, in the order of the layout they were made for
    float *vals32 = nullptr;
    int32_t vals32_layout = -1;

    bool slots() const { return layout == FK_LAYOUT_SLOTS; }
    bool sliced() const { return layout == FK_LAYOUT_SLICED || layout == FK_LAYOUT_SLICED16 || slots(); }
    DevCsr view() const
    {
        const int32_t sw = sweep_grid() > 0 ? 1 : 0;
        const int32_t nt = streaming() ? 1 : 0;
        if (slots())
            return DevCsr{(int32_t)n, (int32_t)nnz, nblocks, row_ptr, col_idx, vals, blocks, block_j0,
                          dg_nslices, dg_ptr, nullptr, dg_vals, nullptr, nullptr, dg_off, dg_mask, sw, nt,
                          dg_max_width};
        return DevCsr{(int32_t)n,  (int32_t)nnz, nblocks,  row_ptr,
                      col_idx,     vals,         blocks,   block_j0,
                      sliced() ? nslices : 0,    sell_ptr, sell_col,
                      sell_vals,   sell_ptr4,
                      layout == FK_LAYOUT_SLICED16 ? sell_off4 : nullptr,
                      nullptr,     nullptr,      sliced() ? sw : 0, sliced() ? nt : 0,
                      sliced() ? sell_max_width : 0};
    }
    // Entries the products read: nnz, or the slice entries with padding.
    int64_t stored_entries() const { return slots() ? dg_entries : sliced() ? sell_entries : nnz; }
    int64_t sell_words4 = 0;  // 8-byte words of the 16-bit column offsets
    // Bytes of matrix data one FP64 product reads: values, column indices
    // (or offsets), row pointers (or slice pointers).
    int64_t matrix_bytes() const
    {
        if (slots())
            return 8 * dg_entries + 4 * (dg_entries / SLICE) + 4 * (int64_t)dg_nslices * SLICE +
                   4 * ((int64_t)dg_nslices + 1);
        if (layout == FK_LAYOUT_SLICED16)
            return 8 * sell_entries + 8 * sell_words4 + 8 * ((int64_t)nslices + 1);
        if (layout == FK_LAYOUT_SLICED)
            return 12 * sell_entries + 4 * ((int64_t)nslices + 1);
        return 12 * nnz + 4 * (n + 1);
    }
    int32_t cus = 0;    // compute units of the device (resident workgroups = 8 per CU)
    // Streaming mode of the sliced products (non-temporal matrix loads and
    // sweep order): -1 = by size (below), 0 = off, 1 = on (FK_STREAM);
    // FK_SELL_SWEEP = 0 / 1 overrides the order alone.
    int32_t stream_req = -1;
    int32_t sweep_req = -1;
    int64_t slices() const { return slots() ? dg_nslices : sliced() ? nslices : 0; }
    // By size: the matrix data one product reads plus four FP64 vectors (those
    // of a pipelined CG iteration) exceed the 256 MiB Infinity Cache of the
    // MI355X.  Below that the cache keeps the matrix from one product to the
    // next (128^3 Poisson: 126 MB + 67 MB), and non-temporal loads, which do
    // not leave lines in it, cost a quarter of the product's speed; above it
    // (160^3, 192^3) they keep the gathered vector lines in L2 and the cache.
    bool streaming() const
    {
        if (!sliced())
            return false;
        if (stream_req >= 0)
            return stream_req != 0;
        return matrix_bytes() + 32 * n > ((int64_t)256 << 20);
    }
    bool sweep_on() const { return sweep_req >= 0 ? sweep_req != 0 : streaming(); }
    // Workgroups of a sweep-order product: as many as are resident at once
    // (8 per CU at the product kernels' register cap), fewer for small
    // matrices (at least one slice per wave); 0 when not in sweep order.
    int sweep_grid() const
    {
        if (!sweep_on() || !sliced() || cus <= 0)
            return 0;
        int64_t g = std::min<int64_t>((int64_t)8 * cus, (slices() + WAVES - 1) / WAVES);
        g &= ~(int64_t)7;
        return (int)g;
    }
    int spmv_grid() const
    {
        const int sg = sweep_grid();
        if (sg > 0)
            return sg;
        return ::spmv_grid(sliced(), slots() ? dg_nslices : sliced() ? nslices : nblocks);
    }
};

DevCsr fk::internal_csr_view(fk_csr A) { return A->view(); }

static fk_status validate_csr(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci)
{
    if (rp[0] != 0)
        return fail(FK_E_CSR, "row_ptr[0] = %d, expected 0", rp[0]);
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i])
            return fail(FK_E_CSR, "row_ptr decreases at row %lld", (long long)i);
    if ((int64_t)rp[n] != nnz)
        return fail(FK_E_CSR, "row_ptr[n] = %d, expected nnz = %lld", rp[n], (long long)nnz);
    for (int64_t j = 0; j < nnz; ++j)
        if (ci[j] < 0 || (int64_t)ci[j] >= n)
            return fail(FK_E_CSR, "col_idx[%lld] = %d outside [0, %lld)", (long long)j, ci[j],
                        (long long)n);
    return FK_OK;
}

// Row blocks: consecutive rows, at most WG rows and NNZ_MAX nonzeros per
// block; a row with more than NNZ_MAX nonzeros forms a block of its own.
static std::vector<int32_t> plan_blocks(const int32_t *rp, int64_t n, int32_t *long_rows)
{
    std::vector<int32_t> b;
    b.reserve((size_t)(n / WG + 2));
    b.push_back(0);
    *long_rows = 0;
    int64_t r = 0;
    while (r < n) {
        const int64_t start = r;
        if ((int64_t)rp[r + 1] - rp[r] > NNZ_MAX) {
            ++*long_rows;
            b.push_back((int32_t)(r + 1));
            ++r;
            continue;
        }
        int64_t nz = 0;
        while (r < n && r - start < WG) {
            const int64_t len = (int64_t)rp[r + 1] - rp[r];
            if (len > NNZ_MAX || nz + len > NNZ_MAX)
                break;
            nz += len;
            ++r;
        }
        b.push_back((int32_t)r);
    }
    return b;
}

// Sliced layout: slice s covers rows [s*SLICE, (s+1)*SLICE) and stores
// width_s = longest row of the slice entries per row.  Returns the entry
// offsets of the slices (entries[nslices] = total, padding included) and
// the longest row.
static std::vector<int64_t> plan_slices(const int32_t *rp, int64_t n, int64_t *max_len)
{
    const int64_t ns = (n + SLICE - 1) / SLICE;
    std::vector<int64_t> off((size_t)ns + 1, 0);
    *max_len = 0;
    for (int64_t sl = 0; sl < ns; ++sl) {
        int64_t w = 0;
        for (int64_t r = sl * SLICE; r < std::min<int64_t>(n, (sl + 1) * SLICE); ++r)
            w = std::max<int64_t>(w, (int64_t)rp[r + 1] - rp[r]);
        *max_len = std::max(*max_len, w);
        off[(size_t)sl + 1] = off[(size_t)sl] + w * SLICE;
    }
    return off;
}

// Rows longer than this are left to the row-block layout: one lane would
// walk them alone while its wave waits.
constexpr int64_t SLICED_MAX_ROW = 64;

// The creation rule: slices when no row is long and padding adds at most a
// quarter to the entries read.
static bool sliced_pays(const std::vector<int64_t> &off, int64_t nnz, int64_t max_len)
{
    const int64_t entries = off.back();
    return nnz > 0 && max_len <= SLICED_MAX_ROW && 4 * entries <= 5 * nnz && entries <= INT32_MAX;
}

// Uploads the sliced arrays of A from host copies of its row pointers and
// column indices; values are gathered on the device from A->vals.
static fk_status build_slices(fk_csr A, const int32_t *rp, const int32_t *ci,
                              const std::vector<int64_t> &off, hipStream_t s)
{
    const int64_t n = A->n;
    const int64_t ns = (int64_t)off.size() - 1;
    const int64_t entries = off.back();
    if (entries > INT32_MAX)
        return fail(FK_E_ARG, "sliced layout needs %lld entries, more than int32 offsets hold",
                    (long long)entries);
    // 16-bit offsets: four entries of a row per 8-byte word; slice s has
    // ceil(width_s / 4) * SLICE words from ptr4[s].
    std::vector<int32_t> ptr, col, map, ptr4;
    std::vector<short4> rel;
    try {
        ptr.resize((size_t)ns + 1);
        ptr4.resize((size_t)ns + 1);
        col.assign((size_t)std::max<int64_t>(entries, 1), -1);
        map.assign((size_t)std::max<int64_t>(entries, 1), -1);
        ptr4[0] = 0;
        for (int64_t sl = 0; sl < ns; ++sl) {
            const int64_t w = (off[(size_t)sl + 1] - off[(size_t)sl]) / SLICE;
            ptr4[(size_t)sl + 1] = ptr4[(size_t)sl] + (int32_t)((w + 3) / 4 * SLICE);
        }
        rel.assign((size_t)std::max<int32_t>(ptr4[(size_t)ns], 1),
                   make_short4(SELL_PAD, SELL_PAD, SELL_PAD, SELL_PAD));
    } catch (const std::bad_alloc &) {
        return fail(FK_E_OOM, "host allocation failed");
    }
    for (int64_t sl = 0; sl <= ns; ++sl)
        ptr[(size_t)sl] = (int32_t)off[(size_t)sl];
    bool narrow = true;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t sl = r / SLICE, lane = r % SLICE;
        for (int32_t j = rp[r]; j < rp[r + 1]; ++j) {
            const int64_t k = j - rp[r];
            const size_t e = (size_t)(off[(size_t)sl] + k * SLICE + lane);
            col[e] = ci[j];
            map[e] = j;
            const int64_t d = (int64_t)ci[j] - r;
            if (d < -32767 || d > 32767) {
                narrow = false;
                continue;
            }
            short4 &wd = rel[(size_t)(ptr4[(size_t)sl] + (k / 4) * SLICE + lane)];
            const int16_t v16 = (int16_t)d;
            switch (k % 4) {
            case 0: wd.x = v16; break;
            case 1: wd.y = v16; break;
            case 2: wd.z = v16; break;
            default: wd.w = v16; break;
            }
        }
    }
    int32_t *d_ptr = nullptr, *d_col = nullptr, *d_map = nullptr, *d_ptr4 = nullptr;
    short4 *d_rel = nullptr;
    double *d_vals = nullptr;
    fk_status st = dev_alloc(&d_ptr, (size_t)ns + 1, "slice offsets");
    if (st == FK_OK)
        st = dev_alloc(&d_col, col.size(), "slice columns");
    if (st == FK_OK && narrow)
        st = dev_alloc(&d_ptr4, ptr4.size(), "slice offsets (16-bit columns)");
    if (st == FK_OK && narrow)
        st = dev_alloc(&d_rel, rel.size(), "slice column offsets");
    if (st == FK_OK)
        st = dev_alloc(&d_vals, col.size(), "slice values");
    if (st == FK_OK)
        st = dev_alloc(&d_map, map.size(), "slice map");
    hipError_t e = hipSuccess;
    if (st == FK_OK) {
        e = hipMemcpyAsync(d_ptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_col, col.data(), col.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && narrow)
            e = hipMemcpyAsync(d_ptr4, ptr4.data(), ptr4.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && narrow)
            e = hipMemcpyAsync(d_rel, rel.data(), rel.size() * sizeof(short4), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_map, map.data(), map.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = launch_gather_vals((int64_t)col.size(), d_vals, A->vals, d_map, vec_grid((int64_t)col.size()), s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            st = fail(FK_E_HIP, "building the sliced layout: %s", hipGetErrorString(e));
    }
    dev_free(d_map);
    if (st != FK_OK) {
        dev_free(d_ptr);
        dev_free(d_col);
        dev_free(d_ptr4);
        dev_free(d_rel);
        dev_free(d_vals);
        return st;
    }
    dev_free(A->sell_ptr);
    dev_free(A->sell_col);
    dev_free(A->sell_ptr4);
    dev_free(A->sell_off4);
    dev_free(A->sell_vals);
    A->sell_ptr = d_ptr;
    A->sell_col = d_col;
    A->sell_ptr4 = d_ptr4;
    A->sell_off4 = d_rel;
    A->sell_words4 = narrow ? ptr4[(size_t)ns] : 0;
    A->sell_vals = d_vals;
    A->nslices = (int32_t)ns;
    A->sell_entries = entries;
    int64_t mw = 0;
    for (int64_t sl = 0; sl < ns; ++sl)
        mw = std::max<int64_t>(mw, (off[(size_t)sl + 1] - off[(size_t)sl]) / SLICE);
    A->sell_max_width = (int32_t)mw;
    return FK_OK;
}

// Slot layout: slice s keeps one slot per distinct column offset
// (column - row) of its rows, in ascending order, and each row a mask of
// the slots it has.  Slot order is column order, so a row is still summed
// left to right in CSR order, provided its columns ascend.  Applies when
// every row's columns strictly ascend, no slice has more than DG_MAX_SLOTS
// distinct offsets, and the slots add at most a quarter to the entries.
// Returns the slot offsets of every slice (offs[ptr[s] .. ptr[s+1])) or
// false.
static bool plan_slots(const int32_t *rp, const int32_t *ci, int64_t n, int64_t nnz,
                       std::vector<int32_t> &ptr, std::vector<int32_t> &offs)
{
    if (nnz <= 0)
        return false;
    const int64_t ns = (n + SLICE - 1) / SLICE;
    ptr.assign((size_t)ns + 1, 0);
    offs.clear();
    std::vector<int32_t> d;
    for (int64_t sl = 0; sl < ns; ++sl) {
        d.clear();
        for (int64_t r = sl * SLICE; r < std::min<int64_t>(n, (sl + 1) * SLICE); ++r) {
            for (int32_t j = rp[r]; j < rp[r + 1]; ++j) {
                if (j > rp[r] && ci[j] <= ci[j - 1])
                    return false;  // columns must strictly ascend
                d.push_back((int32_t)((int64_t)ci[j] - r));
            }
        }
        std::sort(d.begin(), d.end());
        d.erase(std::unique(d.begin(), d.end()), d.end());
        if ((int64_t)d.size() > DG_MAX_SLOTS)
            return false;
        offs.insert(offs.end(), d.begin(), d.end());
        ptr[(size_t)sl + 1] = (int32_t)offs.size();
        if ((int64_t)offs.size() * SLICE * 4 > 5 * nnz + 4 * DG_MAX_SLOTS * SLICE)
            return false;  // early out: padding beyond the quarter
    }
    const int64_t entries = (int64_t)offs.size() * SLICE;
    return 4 * entries <= 5 * nnz && entries <= INT32_MAX;
}

// Uploads the slot arrays of A from host copies of its row pointers and
// column indices and the plan of plan_slots; values are gathered on the
// device from A->vals.
static fk_status build_slots(fk_csr A, const int32_t *rp, const int32_t *ci, const std::vector<int32_t> &sptr,
                             const std::vector<int32_t> &offs, hipStream_t s)
{
    const int64_t n = A->n;
    const int64_t ns = (int64_t)sptr.size() - 1;
    const int64_t entries = (int64_t)offs.size() * SLICE;
    std::vector<int32_t> eptr, map;
    std::vector<uint32_t> mask;
    try {
        eptr.resize((size_t)ns + 1);
        map.assign((size_t)std::max<int64_t>(entries, 1), -1);
        mask.assign((size_t)ns * SLICE, 0u);
    } catch (const std::bad_alloc &) {
        return fail(FK_E_OOM, "host allocation failed");
    }
    for (int64_t sl = 0; sl <= ns; ++sl)
        eptr[(size_t)sl] = sptr[(size_t)sl] * SLICE;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t sl = r / SLICE, lane = r % SLICE;
        const int32_t *o0 = offs.data() + sptr[(size_t)sl], *o1 = offs.data() + sptr[(size_t)sl + 1];
        for (int32_t j = rp[r]; j < rp[r + 1]; ++j) {
            const int32_t d = (int32_t)((int64_t)ci[j] - r);
            const int64_t k = std::lower_bound(o0, o1, d) - o0;  // present by construction
            map[(size_t)(eptr[(size_t)sl] + k * SLICE + lane)] = j;
            mask[(size_t)r] |= 1u << k;
        }
    }
    int32_t *d_ptr = nullptr, *d_off = nullptr, *d_map = nullptr;
    uint32_t *d_mask = nullptr;
    double *d_vals = nullptr;
    fk_status st = dev_alloc(&d_ptr, eptr.size(), "slot slice offsets");
    if (st == FK_OK)
        st = dev_alloc(&d_off, std::max<size_t>(offs.size(), 1), "slot column offsets");
    if (st == FK_OK)
        st = dev_alloc(&d_mask, mask.size(), "slot row masks");
    if (st == FK_OK)
        st = dev_alloc(&d_vals, map.size(), "slot values");
    if (st == FK_OK)
        st = dev_alloc(&d_map, map.size(), "slot map");
    hipError_t e = hipSuccess;
    if (st == FK_OK) {
        e = hipMemcpyAsync(d_ptr, eptr.data(), eptr.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_off, offs.data(), offs.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_mask, mask.data(), mask.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_map, map.data(), map.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = launch_gather_vals((int64_t)map.size(), d_vals, A->vals, d_map, vec_grid((int64_t)map.size()), s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            st = fail(FK_E_HIP, "building the slot layout: %s", hipGetErrorString(e));
    }
    dev_free(d_map);
    if (st != FK_OK) {
        dev_free(d_ptr);
        dev_free(d_off);
        dev_free(d_mask);
        dev_free(d_vals);
        return st;
    }
    dev_free(A->dg_ptr);
    dev_free(A->dg_off);
    dev_free(A->dg_mask);
    dev_free(A->dg_vals);
    A->dg_ptr = d_ptr;
    A->dg_off = d_off;
    A->dg_mask = d_mask;
    A->dg_vals = d_vals;
    A->dg_nslices = (int32_t)ns;
    A->dg_entries = entries;
    int32_t mw = 0;
    for (int64_t sl = 0; sl < ns; ++sl)
        mw = std::max(mw, sptr[(size_t)sl + 1] - sptr[(size_t)sl]);
    A->dg_max_width = mw;
    return FK_OK;
}

static void csr_release(fk_csr A)
{
    dev_free(A->dg_ptr);
    dev_free(A->dg_off);
    dev_free(A->dg_mask);
    dev_free(A->dg_vals);
    dev_free(A->sell_ptr);
    dev_free(A->sell_col);
    dev_free(A->sell_ptr4);
    dev_free(A->sell_off4);
    dev_free(A->sell_vals);
    dev_free(A->row_ptr);
    dev_free(A->col_idx);
    dev_free(A->vals);
    dev_free(A->blocks);
    dev_free(A->block_j0);
    dev_free(A->st);
    dev_free(A->partials);
    dev_free(A->vals32);
}

extern "C" fk_status fk_csr_create(int64_t n, int64_t nnz, const int32_t *row_ptr,
                                   const int32_t *col_idx, const double *vals, int32_t ptr_kind,
                                   void *hip_stream, fk_csr *out)
{
    if (!out)
        return fail(FK_E_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || n >= INT32_MAX)
        return fail(FK_E_ARG, "n = %lld outside [1, 2^31-1)", (long long)n);
    if (nnz < 0 || nnz > INT32_MAX)
        return fail(FK_E_ARG, "nnz = %lld outside [0, 2^31-1]", (long long)nnz);
    if (!row_ptr || (nnz > 0 && (!col_idx || !vals)))
        return fail(FK_E_ARG, "NULL CSR array");
    if (ptr_kind != FK_PTR_HOST && ptr_kind != FK_PTR_DEVICE)
        return fail(FK_E_ARG, "ptr_kind = %d", ptr_kind);
    hipStream_t s = (hipStream_t)hip_stream;

    // Host copies of the index arrays for validation and planning.
    std::vector<int32_t> h_rp, h_ci;
    const int32_t *rp = row_ptr, *ci = col_idx;
    try {
        if (ptr_kind == FK_PTR_DEVICE) {
            h_rp.resize((size_t)n + 1);
            h_ci.resize((size_t)std::max<int64_t>(nnz, 1));
            HIP_TRY(hipMemcpyAsync(h_rp.data(), row_ptr, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost, s));
            if (nnz > 0)
                HIP_TRY(hipMemcpyAsync(h_ci.data(), col_idx, (size_t)nnz * 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            rp = h_rp.data();
            ci = h_ci.data();
        }
    } catch (const std::bad_alloc &) {
        return fail(FK_E_OOM, "host allocation failed");
    }
    fk_status st = validate_csr(n, nnz, rp, ci);
    if (st != FK_OK)
        return st;

    fk_csr A = new (std::nothrow) fk_csr_s;
    if (!A)
        return fail(FK_E_OOM, "host allocation failed");
    A->n = n;
    A->nnz = nnz;
    (void)hipGetDevice(&A->device);
    if (hipDeviceGetAttribute(&A->cus, hipDeviceAttributeMultiprocessorCount, A->device) != hipSuccess)
        A->cus = 0;
    A->stream_req = env_int("FK_STREAM", -1, -1, 1);
    A->sweep_req = env_int("FK_SELL_SWEEP", -1, -1, 1);
    std::vector<int32_t> blocks, block_j0;
    try {
        blocks = plan_blocks(rp, n, &A->long_rows);
        block_j0.resize(blocks.size());
        for (size_t b = 0; b < blocks.size(); ++b)
            block_j0[b] = rp[blocks[b]];
    } catch (const std::bad_alloc &) {
        delete A;
        return fail(FK_E_OOM, "host allocation failed");
    }
    A->nblocks = (int32_t)blocks.size() - 1;
    const hipMemcpyKind kind = ptr_kind == FK_PTR_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
#define CSR_TRY(expr)                                                                      \
    do {                                                                                   \
        fk_status s_ = (expr);                                                             \
        if (s_ != FK_OK) {                                                                 \
            csr_release(A);                                                                \
            delete A;                                                                      \
            return s_;                                                                     \
        }                                                                                  \
    } while (0)
#define CSR_HIP(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            csr_release(A);                                                                \
            delete A;                                                                      \
            return fail(FK_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
        }                                                                                  \
    } while (0)
    CSR_TRY(dev_alloc(&A->row_ptr, (size_t)n + 1, "row_ptr"));
    CSR_TRY(dev_alloc(&A->col_idx, (size_t)nnz, "col_idx"));
    CSR_TRY(dev_alloc(&A->vals, (size_t)nnz, "vals"));
    CSR_TRY(dev_alloc(&A->blocks, blocks.size(), "row blocks"));
    CSR_TRY(dev_alloc(&A->block_j0, blocks.size(), "row blocks"));
    CSR_TRY(dev_alloc(&A->st, 1, "state"));
    CSR_TRY(dev_alloc(&A->partials, RED_SCRATCH_DOUBLES, "partials"));
    CSR_HIP(hipMemcpyAsync(A->row_ptr, row_ptr, (size_t)(n + 1) * 4, kind, s));
    if (nnz > 0) {
        CSR_HIP(hipMemcpyAsync(A->col_idx, col_idx, (size_t)nnz * 4, kind, s));
        CSR_HIP(hipMemcpyAsync(A->vals, vals, (size_t)nnz * 8, kind, s));
    }
    CSR_HIP(hipMemcpyAsync(A->blocks, blocks.data(), blocks.size() * 4, hipMemcpyHostToDevice, s));
    CSR_HIP(hipMemcpyAsync(A->block_j0, block_j0.data(), block_j0.size() * 4, hipMemcpyHostToDevice, s));
    CSR_HIP(hipMemsetAsync(A->st, 0, sizeof(DevState), s));
    CSR_HIP(launch_red_init(A->partials, s));
    CSR_HIP(hipStreamSynchronize(s));
    {
        int64_t max_len = 0;
        std::vector<int64_t> off;
        try {
            off = plan_slices(rp, n, &max_len);
        } catch (const std::bad_alloc &) {
            CSR_TRY(fail(FK_E_OOM, "host allocation failed"));
        }
        std::vector<int32_t> sptr, offs;
        bool slots = false;
        try {
            slots = plan_slots(rp, ci, n, nnz, sptr, offs);
        } catch (const std::bad_alloc &) {
            CSR_TRY(fail(FK_E_OOM, "host allocation failed"));
        }
        if (slots) {
            CSR_TRY(build_slots(A, rp, ci, sptr, offs, s));
            A->layout = FK_LAYOUT_SLOTS;
        } else if (sliced_pays(off, nnz, max_len)) {
            CSR_TRY(build_slices(A, rp, ci, off, s));
            A->layout = A->sell_off4 ? FK_LAYOUT_SLICED16 : FK_LAYOUT_SLICED;
        }
    }
#undef CSR_TRY
#undef CSR_HIP
    *out = A;
    return FK_OK;
}

extern "C" fk_status fk_csr_destroy(fk_csr A)
{
    if (!A)
        return fail(FK_E_ARG, "NULL matrix");
    if (A->solvers > 0)
        return fail(FK_E_STATE, "%d solver(s) still use this matrix", A->solvers);
    csr_release(A);
    delete A;
    return FK_OK;
}

extern "C" fk_status fk_csr_shape(fk_csr A, int64_t *n, int64_t *nnz)
{
    if (!A || !n || !nnz)
        return fail(FK_E_ARG, "NULL argument");
    *n = A->n;
    *nnz = A->nnz;
    return FK_OK;
}

extern "C" fk_status fk_csr_layout(fk_csr A, int32_t *layout, int64_t *stored_entries, int64_t *matrix_bytes)
{
    if (!A || !layout || !stored_entries)
        return fail(FK_E_ARG, "NULL argument");
    *layout = A->layout;
    *stored_entries = A->stored_entries();
    if (matrix_bytes)
        *matrix_bytes = A->matrix_bytes();
    return FK_OK;
}

extern "C" fk_status fk_csr_set_stream(fk_csr A, int32_t mode)
{
    if (!A)
        return fail(FK_E_ARG, "NULL matrix");
    if (mode < -1 || mode > 1)
        return fail(FK_E_ARG, "stream mode must be -1, 0 or 1 (got %d)", mode);
    if (A->solvers > 0)
        return fail(FK_E_STATE, "%d solver(s) use this matrix; destroy them first", A->solvers);
    A->stream_req = mode;
    A->sweep_req = -1;
    return FK_OK;
}

extern "C" fk_status fk_csr_stream(fk_csr A, int32_t *streaming, int32_t *sweep)
{
    if (!A || !streaming)
        return fail(FK_E_ARG, "NULL argument");
    *streaming = A->streaming() ? 1 : 0;
    if (sweep)
        *sweep = A->sweep_grid() > 0 ? 1 : 0;
    return FK_OK;
}

extern "C" fk_status fk_csr_set_layout(fk_csr A, int32_t layout, void *hip_stream)
{
    if (!A)
        return fail(FK_E_ARG, "NULL matrix");
    if (layout != FK_LAYOUT_AUTO && layout != FK_LAYOUT_ROW_BLOCKS && layout != FK_LAYOUT_SLICED &&
        layout != FK_LAYOUT_SLICED16 && layout != FK_LAYOUT_SLOTS)
        return fail(FK_E_ARG, "unknown layout %d", layout);
    if (A->solvers > 0)
        return fail(FK_E_STATE, "%d solver(s) use this matrix; destroy them first", A->solvers);
    if (layout == FK_LAYOUT_ROW_BLOCKS) {
        A->layout = FK_LAYOUT_ROW_BLOCKS;
        return FK_OK;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    std::vector<int32_t> rp, ci;
    bool have_csr = false;
    // Host copies of the CSR arrays, read back once when a layout is built.
    auto read_back = [&]() -> fk_status {
        if (have_csr)
            return FK_OK;
        try {
            rp.resize((size_t)A->n + 1);
            ci.resize((size_t)std::max<int64_t>(A->nnz, 1));
        } catch (const std::bad_alloc &) {
            return fail(FK_E_OOM, "host allocation failed");
        }
        hipError_t e = hipMemcpyAsync(rp.data(), A->row_ptr, rp.size() * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && A->nnz > 0)
            e = hipMemcpyAsync(ci.data(), A->col_idx, (size_t)A->nnz * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return fail(FK_E_HIP, "reading the CSR arrays back: %s", hipGetErrorString(e));
        have_csr = true;
        return FK_OK;
    };
    // The slot layout first (requested, or the creation rule's first choice).
    if (layout == FK_LAYOUT_SLOTS || layout == FK_LAYOUT_AUTO) {
        if (A->dg_nslices == 0) {
            fk_status st = read_back();
            if (st != FK_OK)
                return st;
            std::vector<int32_t> sptr, offs;
            bool ok = false;
            try {
                ok = plan_slots(rp.data(), ci.data(), A->n, A->nnz, sptr, offs);
            } catch (const std::bad_alloc &) {
                return fail(FK_E_OOM, "host allocation failed");
            }
            if (ok) {
                st = build_slots(A, rp.data(), ci.data(), sptr, offs, s);
                if (st != FK_OK)
                    return st;
            } else if (layout == FK_LAYOUT_SLOTS) {
                return fail(FK_E_ARG, "no slot layout: a row's columns do not ascend, a slice has more than %d "
                            "distinct column offsets, or the slots pad the entries by more than a quarter",
                            DG_MAX_SLOTS);
            }
        }
        if (A->dg_nslices > 0) {
            A->layout = FK_LAYOUT_SLOTS;
            return FK_OK;
        }
    }
    if (A->nslices == 0 || layout == FK_LAYOUT_AUTO) {
        fk_status st = read_back();
        if (st != FK_OK)
            return st;
        std::vector<int64_t> off;
        int64_t max_len = 0;
        try {
            off = plan_slices(rp.data(), A->n, &max_len);
        } catch (const std::bad_alloc &) {
            return fail(FK_E_OOM, "host allocation failed");
        }
        if (layout == FK_LAYOUT_AUTO && !sliced_pays(off, A->nnz, max_len)) {
            A->layout = FK_LAYOUT_ROW_BLOCKS;
            return FK_OK;
        }
        if (A->nslices == 0) {
            st = build_slices(A, rp.data(), ci.data(), off, s);
            if (st != FK_OK)
                return st;
        }
    }
    if (layout == FK_LAYOUT_SLICED16 && !A->sell_off4)
        return fail(FK_E_ARG, "a column lies more than 32767 away from its row: no 16-bit offsets");
    if (layout == FK_LAYOUT_AUTO)
        layout = A->sell_off4 ? FK_LAYOUT_SLICED16 : FK_LAYOUT_SLICED;
    A->layout = layout;
    return FK_OK;
}

extern "C" fk_status fk_csr_blocks(fk_csr A, int32_t *nblocks, int32_t *long_rows)
{
    if (!A || !nblocks || !long_rows)
        return fail(FK_E_ARG, "NULL argument");
    *nblocks = A->nblocks;
    *long_rows = A->long_rows;
    return FK_OK;
}

// ------------------------------------------------------------------ solver

struct TimedLaunch {
    int kind;
    int slot;  // index of the start event; end event is slot + 1
};

struct fk_solver_s {
    fk_csr A = nullptr;
    fk_opts o{};
    hipStream_t stream = nullptr;
    int64_t n = 0;
    double *r = nullptr, *p = nullptr, *ap = nullptr, *s = nullptr, *as = nullptr, *rs = nullptr;
    // FK_BICGSTAB_PIPELINED_2K and FK_CG_PIPELINED_1K: the second buffers
    // of r, p and A p
    double *p2 = nullptr, *ap2 = nullptr, *r2 = nullptr;
    double *partials = nullptr, *hist = nullptr, *scal = nullptr;
    DevState *st = nullptr;
    int32_t hist_cap = 0;
    // pinned: [0] state written before a (inner) solve, [1] before the
    // refinement's first residual, [2] state read back
    DevState *h_init = nullptr;
    int32_t *h_status = nullptr;    // pinned, two poll slots
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
    DevState last{};
    bool solved = false;
    bool red_dirty = false;  // a reduction gave up: rewrite the scratch's markers first
    fk_status last_status = FK_E_STATE;
    int grid_spmv = 1, grid_vec = 1;
    // FK_BICGSTAB_PIPELINED_2K: workgroups of its two fused steps;
    // FK_CG_PIPELINED_1K: of its one (grid_xap)
    int grid_sas = 1, grid_xap = 1;
    // profiling
    std::vector<hipEvent_t> prof_ev[2];  // one event pool per batch slot
    std::vector<TimedLaunch> prof_batch[2];
    int prof_next[2] = {0, 0};
    double prof_us[FK_KERNEL_KINDS] = {};
    int32_t prof_n[FK_KERNEL_KINDS] = {};
    // graph replay of one batch of `unroll` iterations
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    double *graph_x = nullptr;
    int graph_iters = 0;
    bool small = false;        // whole solve in one single-workgroup launch
    bool small_stage = false;  // ... with the matrix staged in LDS
    // FK_CG_MIXED: FP32 inner vectors and matrix values; the refinement's
    // own state (st is the inner solver's); sweeps of the last solve.
    bool mixed = false;
    bool f32acc = false;  // FK_CG_MIXED_F32: inner dots and scalars in FP32
    float *r32 = nullptr, *p32 = nullptr, *ap32 = nullptr, *d32 = nullptr, *vals32 = nullptr;
    DevState *st_outer = nullptr;
    int32_t sweeps = 0;
    // GMRES(m): basis V ((m+1) x n), triangular factor R ((m+1)^2, row 0 =
    // xi), eta (m+1), multi-dot scratch, host copies of R and eta.
    bool gmres = false;
    int32_t gm = 0;
    double *V = nullptr, *gR = nullptr, *geta = nullptr, *gpart = nullptr;
    std::vector<double> hR, heta;

    // The mixed method records the refinement's residuals only.
    RedArgs red(int fin, uint32_t mask) const
    {
        return RedArgs{st, partials, mixed ? nullptr : hist, mixed ? nullptr : scal, fin, mask};
    }
    RedArgs red_outer() const { return RedArgs{st_outer, partials, hist, nullptr, FIN_MIX_OUTER, RUN_ACTIVE}; }
    // A reduction point that also folds in the `kpub` dots published by the
    // `npub` workgroups of an earlier FIN_PUBLISH launch.
    RedArgs red_fold(int fin, uint32_t mask, int npub, int kpub) const
    {
        RedArgs a = red(fin, mask);
        a.npub = npub;
        a.kpub = kpub;
        return a;
    }
};

static void solver_release(fk_solver S)
{
    dev_free(S->r);
    dev_free(S->p);
    dev_free(S->ap);
    dev_free(S->p2);
    dev_free(S->ap2);
    dev_free(S->r2);
    dev_free(S->s);
    dev_free(S->as);
    dev_free(S->rs);
    dev_free(S->partials);
    dev_free(S->hist);
    dev_free(S->scal);
    dev_free(S->st);
    dev_free(S->r32);
    dev_free(S->p32);
    dev_free(S->ap32);
    dev_free(S->d32);
    dev_free(S->vals32);
    dev_free(S->st_outer);
    dev_free(S->V);
    dev_free(S->gR);
    dev_free(S->geta);
    dev_free(S->gpart);
    if (S->h_init)
        (void)hipHostFree(S->h_init);
    if (S->h_status)
        (void)hipHostFree(S->h_status);
    S->h_init = nullptr;
    S->h_status = nullptr;
    for (auto &e : S->poll_ev)
        if (e)
            (void)hipEventDestroy(e);
    for (auto &pool : S->prof_ev) {
        for (auto e : pool)
            (void)hipEventDestroy(e);
        pool.clear();
    }
    if (S->graph_exec)
        (void)hipGraphExecDestroy(S->graph_exec);
    if (S->graph)
        (void)hipGraphDestroy(S->graph);
    S->graph_exec = nullptr;
    S->graph = nullptr;
}

static bool is_bicg(int m)
{
    return m == FK_BICGSTAB_PIPELINED || m == FK_BICGSTAB_CLASSICAL || m == FK_BICGSTAB_PIPELINED_SPLIT ||
           m == FK_BICGSTAB_PIPELINED_2K;
}
// Algorithm 4 with the four-kernel or the two-kernel schedule (same iterates).
static bool is_bicg_pipelined(int m) { return m == FK_BICGSTAB_PIPELINED || m == FK_BICGSTAB_PIPELINED_2K; }
static bool is_gmres(int m) { return m == FK_GMRES_PIPELINED || m == FK_GMRES_CLASSICAL; }

static size_t max_lds_per_workgroup(int device)
{
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess)
        return 0;
    return (size_t)lds;
}

// Static LDS of the single-workgroup kernels (state, reduction scratch) plus margin.
constexpr size_t SMALL_STATIC_LDS = 4096;

// The single-workgroup solver takes pipelined solves of systems whose
// vectors fit one workgroup's registers and LDS and whose matrix is small
// enough to be re-read from the caches every iteration.
static bool small_path_ok(fk_csr A, const fk_opts &o)
{
    if (o.flags & FK_FLAG_NO_SMALL)
        return false;
    if (o.method != FK_CG_PIPELINED && o.method != FK_CG_PIPELINED_1K && !is_bicg_pipelined(o.method))
        return false;
    const bool bicg = is_bicg_pipelined(o.method);
    const int rpt = small_rows_per_thread(A->n);
    if (rpt == 0 || (bicg && rpt > 2) || A->nnz > 65536 || A->long_rows > 0)
        return false;
    // Where the grid kernels overtake one workgroup (2D Poisson, 30 fixed
    // iterations, us per iteration, one workgroup / grid): two-kernel CG
    // 12.2 / 15.0 at n = 3,969, 16.2 / 16.6 at 6,400, 18.8 / 14.8 at 8,100;
    // one-kernel CG 9.8 / 11.4 at 2,500, 12.3 / 11.7 at 3,969.
    if (o.method == FK_CG_PIPELINED && A->n > 4096)
        return false;
    if (o.method == FK_CG_PIPELINED_1K && A->n > 3072)
        return false;
    return small_lds_bytes(bicg, A->n) + SMALL_STATIC_LDS <= max_lds_per_workgroup(A->device);
}

// Workgroups of a fused product-and-update step (the two-kernel BiCGStab,
// the one-kernel CG): one round of resident workgroups, at most 4 per CU
// and never more than the product grid; on the sliced layouts sized so that
// every wave takes the same number of slices (a wave with one slice more
// than the others sets the launch's end).  Measured on 1024^2
// convection-diffusion (16384 slices): the BiCGStab x, r, p, A p step holds
// 4 workgroups per CU, and 1024 of them (4 slices per wave) beat 2048 (two
// rounds) by 6 %; for its s, A s step (7 per CU resident) 1024 beat 1368
// (3 slices per wave) and 2048 by 4-6 %.
static int fused_grid(fk_csr A, int step, int grid_spmv)
{
    // at most 4 per CU (FK_FUSED_PER_CU): more waves per SIMD, each with
    // fewer entries in flight, measured slower
    static const int cap = env_int("FK_FUSED_PER_CU", 4, 1, 8);
    const int per_cu = std::min(fused_per_cu(A->view(), step), cap);
    int64_t g = grid_spmv;
    if (per_cu > 0 && A->cus > 0 && g > (int64_t)per_cu * A->cus) {
        g = (int64_t)per_cu * A->cus;
        const int64_t sl = A->slices();
        if (sl > 0) {
            const int64_t spw = (sl + (int64_t)WAVES * g - 1) / ((int64_t)WAVES * g);
            g = (sl + (int64_t)WAVES * spw - 1) / ((int64_t)WAVES * spw);
        }
    }
    if (g >= 8)
        g = (g + 7) & ~(int64_t)7;
    return (int)std::max<int64_t>(g, 1);
}

extern "C" fk_status fk_solver_create(fk_csr A, const fk_opts *o, void *hip_stream, fk_solver *out)
{
    if (!out)
        return fail(FK_E_ARG, "out is NULL");
    *out = nullptr;
    if (!A || !o)
        return fail(FK_E_ARG, "NULL argument");
    if (o->method < FK_CG_PIPELINED || o->method > FK_CG_PIPELINED_1K)
        return fail(FK_E_ARG, "unknown method %d", o->method);
    if (o->restart < 0 || o->restart > GM_MAX)
        return fail(FK_E_ARG, "restart outside [0, %d]", GM_MAX);
    if (!(o->inner_rtol >= 0.0) || !std::isfinite(o->inner_rtol))
        return fail(FK_E_ARG, "inner_rtol must be finite and >= 0");
    if (o->max_outer < 0)
        return fail(FK_E_ARG, "max_outer < 0");
    if (!(o->rtol >= 0.0) || !std::isfinite(o->rtol))
        return fail(FK_E_ARG, "rtol must be finite and >= 0");
    if (o->max_iter < 0)
        return fail(FK_E_ARG, "max_iter < 0");
    if (o->unroll < 0 || o->unroll > 4096)
        return fail(FK_E_ARG, "unroll outside [0, 4096]");
    if (o->flags & ~(FK_FLAG_GRAPH | FK_FLAG_PROFILE | FK_FLAG_NO_SMALL | FK_FLAG_SCALARS))
        return fail(FK_E_ARG, "unknown flags 0x%x", o->flags);
    if (o->record_history < 0)
        return fail(FK_E_ARG, "record_history < 0");

    fk_solver S = new (std::nothrow) fk_solver_s;
    if (!S)
        return fail(FK_E_OOM, "host allocation failed");
    S->A = A;
    S->o = *o;
    if (S->o.unroll == 0)
        S->o.unroll = 32;
    S->mixed = o->method == FK_CG_MIXED || o->method == FK_CG_MIXED_F32;
    S->f32acc = o->method == FK_CG_MIXED_F32;
    S->gmres = is_gmres(o->method);
    S->gm = o->restart == 0 ? 30 : o->restart;
    if (S->o.inner_rtol == 0.0)
        S->o.inner_rtol = 1e-4;
    if (S->o.max_outer == 0)
        S->o.max_outer = 50;
    S->stream = (hipStream_t)hip_stream;
    S->n = A->n;
    S->grid_spmv = A->spmv_grid();
    S->grid_vec = vec_grid(A->n);
    if (o->method == FK_BICGSTAB_PIPELINED_2K) {
        S->grid_sas = fused_grid(A, FUSED_BICG_SAS, S->grid_spmv);
        S->grid_xap = fused_grid(A, FUSED_BICG_XAP, S->grid_spmv);
    }
    if (o->method == FK_CG_PIPELINED_1K)
        S->grid_xap = fused_grid(A, FUSED_CG_XAP, S->grid_spmv);
    const size_t n = (size_t)A->n;
#define S_TRY(expr)                                                                        \
    do {                                                                                   \
        fk_status s_ = (expr);                                                             \
        if (s_ != FK_OK) {                                                                 \
            solver_release(S);                                                             \
            delete S;                                                                      \
            return s_;                                                                     \
        }                                                                                  \
    } while (0)
#define S_HIP(expr)                                                                        \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            solver_release(S);                                                             \
            delete S;                                                                      \
            return fail(FK_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
        }                                                                                  \
    } while (0)
    if (S->gmres) {
        const size_t m1 = (size_t)S->gm + 1;
        S_TRY(dev_alloc(&S->r, n, "r"));
        S_TRY(dev_alloc(&S->V, m1 * n, "Krylov basis"));
        S_TRY(dev_alloc(&S->gR, m1 * m1, "R"));
        S_TRY(dev_alloc(&S->geta, m1, "eta"));
        S_TRY(dev_alloc(&S->gpart, GM_PART_DOUBLES, "multi-dot partials"));
        try {
            S->hR.assign(m1 * m1, 0.0);
            S->heta.assign(m1, 0.0);
        } catch (const std::bad_alloc &) {
            solver_release(S);
            delete S;
            return fail(FK_E_OOM, "host allocation failed");
        }
    } else if (S->mixed) {
        S_TRY(dev_alloc(&S->r32, n, "r32"));
        S_TRY(dev_alloc(&S->p32, n, "p32"));
        S_TRY(dev_alloc(&S->ap32, n, "Ap32"));
        S_TRY(dev_alloc(&S->d32, n, "d32"));
        S_TRY(dev_alloc(&S->vals32, (size_t)A->stored_entries(), "FP32 values"));
        S_TRY(dev_alloc(&S->st_outer, 1, "refinement state"));
    } else {
        S_TRY(dev_alloc(&S->r, n, "r"));
        S_TRY(dev_alloc(&S->p, n, "p"));
        S_TRY(dev_alloc(&S->ap, n, "Ap"));
    }
    if (is_bicg(o->method)) {
        if (o->method != FK_BICGSTAB_PIPELINED_2K)  // (which never stores s)
            S_TRY(dev_alloc(&S->s, n, "s"));
        S_TRY(dev_alloc(&S->as, n, "As"));
        S_TRY(dev_alloc(&S->rs, n, "r0*"));
    }
    if (o->method == FK_BICGSTAB_PIPELINED_2K || o->method == FK_CG_PIPELINED_1K) {
        S_TRY(dev_alloc(&S->p2, n, "p (second buffer)"));
        S_TRY(dev_alloc(&S->r2, n, "r (second buffer)"));
        S_TRY(dev_alloc(&S->ap2, n, "Ap (second buffer)"));
    }
    S_TRY(dev_alloc(&S->partials, RED_SCRATCH_DOUBLES, "partials"));
    S_TRY(dev_alloc(&S->st, 1, "state"));
    // History: entries 0 .. cap-1 are kept (the device drops later ones), cap
    // = min(iterations + 1, FK_HISTORY_DEFAULT or the count asked for), so a
    // large max_iter does not size the buffers.
    const int64_t hist_want = o->record_history == 1 ? FK_HISTORY_DEFAULT : o->record_history;
    if (o->record_history && S->mixed) {
        S->hist_cap = (int32_t)std::min<int64_t>((int64_t)S->o.max_outer + 1, hist_want);
        S_TRY(dev_alloc(&S->hist, (size_t)S->hist_cap, "history"));
    } else if (o->record_history) {
        S->hist_cap = (int32_t)std::min<int64_t>((int64_t)o->max_iter + 1, hist_want);
        S_TRY(dev_alloc(&S->hist, (size_t)S->hist_cap, "history"));
        if ((o->flags & FK_FLAG_SCALARS) && !S->mixed && !S->gmres)
            S_TRY(dev_alloc(&S->scal, (size_t)S->hist_cap * 4, "scalars"));
    }
    S_HIP(hipHostMalloc(reinterpret_cast<void **>(&S->h_init), 3 * sizeof(DevState), hipHostMallocDefault));
    S_HIP(hipHostMalloc(reinterpret_cast<void **>(&S->h_status), 2 * sizeof(int32_t), hipHostMallocDefault));
    for (auto &e : S->poll_ev)
        S_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    S_HIP(hipMemsetAsync(S->st, 0, sizeof(DevState), S->stream));
    S_HIP(launch_red_init(S->partials, S->stream));
    if (S->gmres) {
        S_HIP(hipMemsetAsync(S->gR, 0, ((size_t)S->gm + 1) * ((size_t)S->gm + 1) * sizeof(double), S->stream));
        S_HIP(hipMemsetAsync(S->gpart, 0, GM_PART_DOUBLES * sizeof(double), S->stream));
    }
    if (S->mixed) {
        S_HIP(hipMemsetAsync(S->st_outer, 0, sizeof(DevState), S->stream));
        if (A->nnz > 0) {
            // the values of the layout the products read, stored_entries() of them
            const double *src = A->slots() ? A->dg_vals : A->sliced() ? A->sell_vals : A->vals;
            const int64_t m = A->stored_entries();
            S_HIP(launch_to_f32(m, S->vals32, src, vec_grid(m), S->stream));
        }
    }
    S->small = small_path_ok(A, S->o);
    S->small_stage = S->small &&
                     small_staged_lds_bytes(is_bicg_pipelined(o->method), A->n, A->nnz) +
                             SMALL_STATIC_LDS <= max_lds_per_workgroup(A->device);
    S_HIP(hipStreamSynchronize(S->stream));
#undef S_TRY
#undef S_HIP
    A->solvers++;
    *out = S;
    return FK_OK;
}

extern "C" fk_status fk_solver_destroy(fk_solver S)
{
    if (!S)
        return fail(FK_E_ARG, "NULL solver");
    (void)hipStreamSynchronize(S->stream);
    solver_release(S);
    if (S->A)
        S->A->solvers--;
    delete S;
    return FK_OK;
}

// ------------------------------------------------------------------ driver

namespace {

struct Enq {
    fk_solver S;
    bool profile;
    int batch;

    template <typename F>
    hipError_t run(int kind, F &&launch)
    {
        if (!profile)
            return launch();
        std::vector<hipEvent_t> &pool = S->prof_ev[batch];
        const int slot = S->prof_next[batch];
        while ((size_t)slot + 2 > pool.size()) {
            hipEvent_t e;
            hipError_t er = hipEventCreate(&e);
            if (er != hipSuccess)
                return er;
            pool.push_back(e);
        }
        // The events are stamped by the device at the start and end of the
        // kernel itself (not around its dispatch).
        set_launch_timing(pool[slot], pool[slot + 1]);
        hipError_t e = launch();
        set_launch_timing(nullptr, nullptr);
        if (e != hipSuccess)
            return e;
        S->prof_batch[batch].push_back(TimedLaunch{kind, slot});
        S->prof_next[batch] = slot + 2;
        return hipSuccess;
    }
};

#define ENQ(kind, call)                                                                    \
    do {                                                                                   \
        hipError_t e_ = q.run(kind, [&]() { return (call); });                              \
        if (e_ != hipSuccess)                                                              \
            return e_;                                                                     \
    } while (0)

hipError_t enqueue_setup(fk_solver S, Enq &q, const double *b, double *x)
{
    const DevCsr A = S->A->view();
    const int64_t n = S->n;
    const int gs = S->grid_spmv, gv = S->grid_vec;
    hipStream_t st = S->stream;
    if (S->mixed) {
        // Inner solve of A d = r32 from d_0 = 0: p_0 = r_0 = r32.
        const bool f = S->f32acc;
        ENQ(FK_KERNEL_SETUP, launch_inner_setup32(n, S->r32, S->p32, S->d32,
                                                  S->red(f ? FIN_SETUP32 : FIN_SETUP, RUN_ACTIVE), gv, st, f));
        ENQ(FK_KERNEL_SPMV_DOT, launch_spmv32(A, S->vals32, S->p32, S->ap32,
                                              S->red(f ? FIN_CG_ALPHA32 : FIN_CG_ALPHA, RUN_ACTIVE), gs, st, f));
        return hipSuccess;
    }
    double *rs = is_bicg(S->o.method) ? S->rs : nullptr;
    ENQ(FK_KERNEL_SETUP, launch_residual0(A, b, x, S->r, S->p, rs, S->red(FIN_SETUP, RUN_ACTIVE), gs, st));
    // b = 0: x = 0 (runs only in that state; not timed).
    hipError_t ez = launch_zero(x, n, S->st, 1u << ST_ZERO_RHS, gv, st);
    if (ez != hipSuccess)
        return ez;
    if (S->o.method == FK_CG_PIPELINED || S->o.method == FK_CG_PIPELINED_1K)
        ENQ(FK_KERNEL_SPMV_DOT, launch_spmv_dots(A, S->p, S->ap, nullptr, D_YV | D_YY,
                                                 S->red(FIN_CG_ALPHA, RUN_ACTIVE), gs, st));
    if (S->o.method == FK_CG_PIPELINED_SPLIT) {
        ENQ(FK_KERNEL_SPMV, launch_spmv_dots(A, S->p, S->ap, nullptr, 0, S->red(FIN_NONE, RUN_ACTIVE), gs, st));
        ENQ(FK_KERNEL_DOT, launch_dot(n, S->ap, S->p, S->ap, 2, S->red(FIN_CG_ALPHA, RUN_ACTIVE), gv, st));
    }
    if (S->o.method == FK_BICGSTAB_PIPELINED_2K)
        // A p_0 + <Ap_0, r0*>: rho_0 comes from the setup, then alpha_0; p_0
        // and A p_0 sit in the first buffers (iteration count 0).
        ENQ(FK_KERNEL_SPMV_DOT, launch_spmv_dots(A, S->p, S->ap, S->rs, D_YW,
                                                 S->red(FIN_B_RHO_ALPHA, RUN_ACTIVE), gs, st));
    return hipSuccess;
}

// `last`: this is iteration max_iter, after which nothing can run; launches
// that would only return at once are left out.
hipError_t enqueue_iteration(fk_solver S, Enq &q, double *x, bool last)
{
    const DevCsr A = S->A->view();
    const int64_t n = S->n;
    const int gs = S->grid_spmv, gv = S->grid_vec;
    hipStream_t st = S->stream;
    DevState *ds = S->st;
    switch (S->o.method) {
    case FK_CG_PIPELINED:
        // Fused x, r, p update + first stage of <r_i, r_i> (published); then
        // Ap_i + <p_i,Ap_i>, <Ap_i,Ap_i>, whose second stage also completes
        // <r_i, r_i>: one reduction round trip per iteration.  The product
        // runs in the last iteration too: it carries the convergence test.
        ENQ(FK_KERNEL_UPDATE_DOT, launch_cg_update(n, x, S->r, S->p, S->ap, S->red(FIN_PUBLISH, RUN_ACTIVE), gv, st));
        ENQ(FK_KERNEL_SPMV_DOT, launch_spmv_dots(A, S->p, S->ap, nullptr, D_YV | D_YY,
                                                 S->red_fold(FIN_CG_RR_ALPHA, RUN_ACTIVE, gv, 1), gs, st));
        break;
    case FK_CG_PIPELINED_1K: {
        // x, r, p of iteration i and A p_i + <p_i,Ap_i>, <Ap_i,Ap_i>, <r_i,r_i>
        // in one launch: convergence on r_i, then alpha_i, beta_i.
        const Cg1Io io{x, {S->r, S->r2}, {S->p, S->p2}, {S->ap, S->ap2}};
        ENQ(FK_KERNEL_SPMV_DOT, launch_cg1_xap(A, io, S->red(FIN_CG_RR_ALPHA, RUN_ACTIVE), S->grid_xap, st));
        break;
    }
    case FK_CG_PIPELINED_SPLIT:
        // Section 3.1's alternative: the product and its two dots in separate
        // kernels (3 launches, one more pass over p and A p).
        ENQ(FK_KERNEL_UPDATE_DOT, launch_cg_update(n, x, S->r, S->p, S->ap, S->red(FIN_PUBLISH, RUN_ACTIVE), gv, st));
        ENQ(FK_KERNEL_SPMV, launch_spmv_dots(A, S->p, S->ap, nullptr, 0, S->red(FIN_NONE, RUN_ACTIVE), gs, st));
        ENQ(FK_KERNEL_DOT, launch_dot(n, S->ap, S->p, S->ap, 2, S->red_fold(FIN_CG_RR_ALPHA, RUN_ACTIVE, gv, 1),
                                      gv, st));
        break;
    case FK_BICGSTAB_PIPELINED_SPLIT:
        // Section 3.2's alternative: both products without dots, each
        // followed by a dot kernel (6 launches per iteration).
        ENQ(FK_KERNEL_SPMV, launch_spmv_dots(A, S->p, S->ap, nullptr, 0, S->red(FIN_NONE, RUN_ACTIVE), gs, st));
        ENQ(FK_KERNEL_DOT, launch_dot(n, S->ap, S->rs, nullptr, 1, S->red_fold(FIN_B_RHO_ALPHA, RUN_ACTIVE, gv, 2),
                                      gv, st));
        ENQ(FK_KERNEL_UPDATE_DOT, launch_bicg_s(n, S->r, S->ap, S->s, S->red(FIN_PUBLISH, RUN_ACTIVE), gv, st));
        ENQ(FK_KERNEL_SPMV, launch_spmv_dots(A, S->s, S->as, nullptr, 0, S->red(FIN_NONE, RUN_ACTIVE), gs, st));
        ENQ(FK_KERNEL_DOT, launch_dot(n, S->as, S->s, S->as, 3, S->red_fold(FIN_B_SS_OMEGA, RUN_ACTIVE, gv, 1), gv,
                                      st, S->rs));
        ENQ(FK_KERNEL_UPDATE_DOT, launch_bicg_xrp(n, x, S->r, S->p, S->s, S->as, S->ap, S->rs,
                                                  S->red(FIN_B_XRP_PUB, RUN_BICG_UPDATE), gv, st));
        break;
    case FK_CG_CLASSICAL:
        ENQ(FK_KERNEL_SPMV, launch_spmv_dots(A, S->p, S->ap, nullptr, 0, S->red(FIN_NONE, RUN_ACTIVE), gs, st));
        ENQ(FK_KERNEL_DOT, launch_dot(n, S->p, S->ap, nullptr, 1, S->red(FIN_C_CG_ALPHA, RUN_ACTIVE), gv, st));
        ENQ(FK_KERNEL_AXPY, launch_axpy(n, x, x, S->p, 0, 0, ds, RUN_ACTIVE, gv, st));
        ENQ(FK_KERNEL_AXPY, launch_axpy(n, S->r, S->r, S->ap, 0, 1, ds, RUN_ACTIVE, gv, st));
        ENQ(FK_KERNEL_DOT, launch_dot(n, S->r, S->r, nullptr, 1, S->red(FIN_C_CG_BETA, RUN_ACTIVE), gv, st));
        if (!last)
            ENQ(FK_KERNEL_AXPY, launch_xpay(n, S->p, S->r, nullptr, ds, RUN_ACTIVE, gv, st));
        break;
    case FK_BICGSTAB_PIPELINED:
        // The product A p also completes the previous update's <r,r0*>,
        // <r,r> (rho_i), then alpha_i.
        ENQ(FK_KERNEL_SPMV_DOT, launch_spmv_dots(A, S->p, S->ap, S->rs, D_YW,
                                                 S->red_fold(FIN_B_RHO_ALPHA, RUN_ACTIVE, gv, 2), gs, st));
        // s update publishes <s,s>; the product A s completes it with its
        // own three dots (half-step test, then omega and beta).
        ENQ(FK_KERNEL_UPDATE_DOT, launch_bicg_s(n, S->r, S->ap, S->s, S->red(FIN_PUBLISH, RUN_ACTIVE), gv, st));
        ENQ(FK_KERNEL_SPMV_DOT, launch_spmv_dots(A, S->s, S->as, S->rs, D_YV | D_YY | D_YW,
                                                 S->red_fold(FIN_B_SS_OMEGA, RUN_ACTIVE, gv, 1), gs, st));
        ENQ(FK_KERNEL_UPDATE_DOT, launch_bicg_xrp(n, x, S->r, S->p, S->s, S->as, S->ap, S->rs,
                                                  S->red(FIN_B_XRP_PUB, RUN_BICG_UPDATE), gv, st));
        break;
    case FK_BICGSTAB_PIPELINED_2K: {
        // s_i and A s_i (+ <As,s>, <As,As>, <As,r0*>, <s,s>: half-step test,
        // omega_i, beta_i, decision on i+1); then x, r, p of iteration i+1
        // and A p_{i+1} (+ <Ap,r0*>, <r,r0*>, <r,r>: rho, alpha), or, after
        // a decision, the last x, r and the final reduction.
        const Bicg2Io io{x, {S->r, S->r2}, S->as, S->rs, {S->p, S->p2}, {S->ap, S->ap2}};
        ENQ(FK_KERNEL_SPMV_DOT, launch_bicg2_sas(A, io, S->red(FIN_B_SS_OMEGA, RUN_ACTIVE), S->grid_sas, st));
        ENQ(FK_KERNEL_UPDATE_DOT,
            launch_bicg2_xap(A, io, S->red(FIN_B_XRP_ALPHA, RUN_BICG_UPDATE), S->grid_xap, st));
        break;
    }
    case FK_BICGSTAB_CLASSICAL:
        ENQ(FK_KERNEL_SPMV, launch_spmv_dots(A, S->p, S->ap, nullptr, 0, S->red(FIN_NONE, RUN_ACTIVE), gs, st));
        ENQ(FK_KERNEL_DOT, launch_dot(n, S->ap, S->rs, nullptr, 1, S->red(FIN_B_ALPHA, RUN_ACTIVE), gv, st));
        ENQ(FK_KERNEL_AXPY, launch_axpy(n, S->s, S->r, S->ap, 0, 1, ds, RUN_ACTIVE, gv, st));
        ENQ(FK_KERNEL_DOT, launch_dot(n, S->s, S->s, nullptr, 1, S->red(FIN_B_SS, RUN_ACTIVE), gv, st));
        ENQ(FK_KERNEL_SPMV, launch_spmv_dots(A, S->s, S->as, nullptr, 0, S->red(FIN_NONE, RUN_ACTIVE), gs, st));
        ENQ(FK_KERNEL_DOT, launch_dot(n, S->as, S->s, S->as, 2, S->red(FIN_C_B_OMEGA, RUN_ACTIVE), gv, st));
        ENQ(FK_KERNEL_AXPY, launch_axpy(n, x, x, S->p, 0, 0, ds, RUN_ACTIVE_OR_HALF, gv, st));
        ENQ(FK_KERNEL_AXPY, launch_copy_fin(n, S->r, S->s, S->red(FIN_HALF_DONE, RUN_HALF), st));
        ENQ(FK_KERNEL_AXPY, launch_axpy(n, x, x, S->s, 1, 0, ds, RUN_ACTIVE, gv, st));
        ENQ(FK_KERNEL_AXPY, launch_axpy(n, S->r, S->s, S->as, 1, 1, ds, RUN_ACTIVE, gv, st));
        ENQ(FK_KERNEL_DOT, launch_dot(n, S->r, S->r, nullptr, 1, S->red(FIN_C_B_RR, RUN_ACTIVE), gv, st));
        ENQ(FK_KERNEL_DOT, launch_dot(n, S->r, S->rs, nullptr, 1, S->red(FIN_C_B_RHO, RUN_ACTIVE), gv, st));
        if (!last)
            ENQ(FK_KERNEL_AXPY, launch_xpay(n, S->p, S->r, S->ap, ds, RUN_ACTIVE, gv, st));
        break;
    case FK_CG_MIXED:
    case FK_CG_MIXED_F32: {
        // Algorithm 2 in FP32 on the correction d (x is not touched).
        const bool f = S->f32acc;
        ENQ(FK_KERNEL_UPDATE_DOT, launch_cg_update32(n, S->d32, S->r32, S->p32, S->ap32,
                                                     S->red(FIN_PUBLISH, RUN_ACTIVE), gv, st, f));
        ENQ(FK_KERNEL_SPMV_DOT, launch_spmv32(A, S->vals32, S->p32, S->ap32,
                                              S->red_fold(f ? FIN_CG_RR_ALPHA32 : FIN_CG_RR_ALPHA, RUN_ACTIVE,
                                                          gv, 1),
                                              gs, st, f));
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipSuccess;
}

void harvest_profile(fk_solver S, int batch)
{
    const std::vector<hipEvent_t> &pool = S->prof_ev[batch];
    for (const TimedLaunch &t : S->prof_batch[batch]) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pool[t.slot], pool[t.slot + 1]) == hipSuccess) {
            S->prof_us[t.kind] += 1000.0 * (double)ms;
            S->prof_n[t.kind] += 1;
        }
    }
}

// Refinement step on the FP64 side: x += d (when `add`), then
// r32 = (float)(b - A x) with its FP64 norm test; waits and leaves the
// refinement state in h_init[2].
hipError_t mixed_outer(fk_solver S, const double *b, double *x, bool add, bool profile)
{
    const DevCsr A = S->A->view();
    hipStream_t st = S->stream;
    S->prof_batch[0].clear();
    S->prof_next[0] = 0;
    Enq q{S, profile, 0};
    if (add)
        ENQ(FK_KERNEL_AXPY, launch_add32(S->n, x, S->d32, S->grid_vec, st));
    ENQ(FK_KERNEL_RESIDUAL, launch_residual32(A, b, x, S->r32, S->red_outer(), S->grid_spmv, st));
    hipError_t e = hipMemcpyAsync(&S->h_init[2], S->st_outer, sizeof(DevState), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess)
        return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return e;
    if (profile)
        harvest_profile(S, 0);
    return hipSuccess;
}

#undef ENQ

// A reduction point that gave up waiting (DevState::red_fault) voids the
// solve: report it, and rewrite the scratch's empty markers before the next.
static fk_status reduction_fault(fk_solver S)
{
    S->red_dirty = true;
    return fail(FK_E_HIP, "a cross-workgroup reduction did not complete; the solve is void");
}

hipError_t enqueue_poll(fk_solver S, int slot)
{
    const char *status_addr = reinterpret_cast<const char *>(S->st) + offsetof(DevState, status);
    hipError_t e = hipMemcpyAsync(&S->h_status[slot], status_addr, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, S->stream);
    if (e != hipSuccess)
        return e;
    return hipEventRecord(S->poll_ev[slot], S->stream);
}

// Capture `iters` iterations into a graph (reused while x stays the same).
hipError_t ensure_graph(fk_solver S, double *x, int iters)
{
    if (S->graph_exec && S->graph_x == x && S->graph_iters == iters)
        return hipSuccess;
    if (S->graph_exec)
        (void)hipGraphExecDestroy(S->graph_exec);
    if (S->graph)
        (void)hipGraphDestroy(S->graph);
    S->graph_exec = nullptr;
    S->graph = nullptr;
    hipError_t e = hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return e;
    Enq q{S, false, 0};
    hipError_t e2 = hipSuccess;
    for (int i = 0; i < iters && e2 == hipSuccess; ++i)
        e2 = enqueue_iteration(S, q, x, false);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(S->stream, &g);
    if (e2 != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        return e2;
    }
    if (e != hipSuccess)
        return e;
    e = hipGraphInstantiate(&S->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return e;
    }
    S->graph = g;
    S->graph_x = x;
    S->graph_iters = iters;
    return hipSuccess;
}

}  // namespace

static fk_status finish_solve(fk_solver S);

// Multi-kernel solve: writes the initial state (rtol, max_iter, hist_cap),
// enqueues the setup and batches of `unroll` iterations with one batch in
// flight ahead of the one waited for, and leaves the final state in S->last.
static fk_status run_batches(fk_solver S, const double *b, double *x, double rtol, int64_t max_iter,
                             int32_t hist_cap, bool profile, bool graph)
{
    DevState init{};
    init.status = ST_RUNNING;
    init.rtol = rtol;
    init.max_iter = (int32_t)max_iter;
    init.hist_cap = hist_cap;
    S->h_init[0] = init;
    HIP_TRY(hipMemcpyAsync(S->st, &S->h_init[0], sizeof(DevState), hipMemcpyHostToDevice, S->stream));

    const int U = S->o.unroll;
    int64_t launched = 0;
    int cur = 0;

    auto enqueue_batch = [&](int slot, bool with_setup) -> hipError_t {
        S->prof_batch[slot].clear();
        S->prof_next[slot] = 0;
        Enq q{S, profile, slot};
        hipError_t e = hipSuccess;
        if (with_setup)
            e = enqueue_setup(S, q, b, x);
        if (e != hipSuccess)
            return e;
        const int64_t todo = std::min<int64_t>(U, max_iter - launched);
        const bool reaches_end = launched + todo == max_iter;
        if (graph && todo == U && !reaches_end) {
            e = ensure_graph(S, x, U);
            if (e != hipSuccess)
                return e;
            e = hipGraphLaunch(S->graph_exec, S->stream);
        } else {
            for (int64_t i = 0; i < todo && e == hipSuccess; ++i)
                e = enqueue_iteration(S, q, x, reaches_end && i == todo - 1);
        }
        if (e != hipSuccess)
            return e;
        launched += todo;
        return enqueue_poll(S, slot);
    };

    // A batch slot is reused only after its poll has been waited for (and its
    // profile events harvested).
    hipError_t e = enqueue_batch(0, true);
    if (e != hipSuccess)
        return fail(FK_E_HIP, "enqueue: %s", hipGetErrorString(e));
    for (;;) {
        const bool more = launched < max_iter;
        if (more) {
            e = enqueue_batch(cur ^ 1, false);
            if (e != hipSuccess)
                return fail(FK_E_HIP, "enqueue: %s", hipGetErrorString(e));
        }
        HIP_TRY(hipEventSynchronize(S->poll_ev[cur]));
        const int32_t status = S->h_status[cur];
        // Every launch of a batch ran if the solve was still going (or had
        // just used up its iteration budget) when the batch ended.
        if (profile && (status == ST_RUNNING || status == ST_NOT_CONVERGED))
            harvest_profile(S, cur);
        if (status != ST_RUNNING || !more)
            break;
        cur ^= 1;
    }
    HIP_TRY(hipMemcpyAsync(&S->h_init[2], S->st, sizeof(DevState), hipMemcpyDeviceToHost, S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
    S->last = S->h_init[2];
    if (S->last.red_fault)
        return reduction_fault(S);
    return FK_OK;
}

// Restarted GMRES(m), Algorithm 6 (pipelined) or Algorithm 5 (classical
// residual update): a cycle is enqueued at once (its kernels return at once
// after the device ends the cycle), then R and xi are read back, R eta = xi
// is solved on the host and x is updated on the device.
#define ENQ(kind, call)                                                                    \
    do {                                                                                   \
        hipError_t e_ = q.run(kind, [&]() { return (call); });                              \
        if (e_ != hipSuccess)                                                              \
            return e_;                                                                     \
    } while (0)

static fk_status solve_gmres(fk_solver S, const double *b, double *x, bool profile)
{
    const DevCsr A = S->A->view();
    const int64_t n = S->n;
    const int m = S->gm, m1 = m + 1;
    const int gs = S->grid_spmv, gv = S->grid_vec;
    hipStream_t st = S->stream;
    const bool classical = S->o.method == FK_GMRES_CLASSICAL;
    DevState init{};
    init.status = ST_RUNNING;
    init.rtol = S->o.rtol;
    init.max_iter = S->o.max_iter;
    init.hist_cap = S->hist_cap;
    init.gm = m;
    S->h_init[0] = init;
    HIP_TRY(hipMemcpyAsync(S->st, &S->h_init[0], sizeof(DevState), hipMemcpyHostToDevice, st));
    auto vec = [&](int j) { return S->V + (size_t)j * n; };
    auto red = [&](int fin) { return RedArgs{S->st, S->partials, S->hist, S->gR, fin, RUN_ACTIVE}; };
    for (;;) {
        S->prof_batch[0].clear();
        S->prof_next[0] = 0;
        Enq q{S, profile, 0};
        hipError_t e = [&]() -> hipError_t {
            // r0 = b - A x, ||r0||, ||b|| (first cycle); v_0 = r0 / rho0
            ENQ(FK_KERNEL_SETUP, launch_residual0(A, b, x, S->r, vec(0), nullptr, red(FIN_GM_SETUP), gs, st));
            ENQ(FK_KERNEL_SETUP, launch_gm_scale(n, vec(0), S->r, S->st, RUN_ACTIVE, gv, st));
            if (classical)
                ENQ(FK_KERNEL_AXPY, launch_gm_scale(n, S->r, S->r, S->st, RUN_ACTIVE, gv, st));
            const double *rxi = classical ? S->r : vec(0);
            for (int i = 1; i <= m; ++i) {
                // w = A v_{i-1} (into slot i), with <v_{i-1}, w> when i >= 2
                ENQ(FK_KERNEL_SPMV_DOT, launch_spmv_dots(A, vec(i - 1), vec(i), nullptr, i >= 2 ? D_YV : 0,
                                                         red(i >= 2 ? FIN_GM_R1 : FIN_NONE), gs, st));
                if (i >= 3) {
                    ENQ(FK_KERNEL_DOT, launch_gm_multidot(n, S->V, vec(i), 1, i - 1, S->gpart, S->st, RUN_ACTIVE, st));
                    ENQ(FK_KERNEL_DOT, launch_gm_multidot_fin(1, i - 1, i, S->gR, m1, S->gpart, S->st, RUN_ACTIVE, st));
                }
                ENQ(FK_KERNEL_UPDATE_DOT, launch_gm_update(n, vec(i), S->V, i, m1, red(FIN_GM_NORM), gv, st));
                ENQ(FK_KERNEL_UPDATE_DOT, launch_gm_normalize(n, vec(i), rxi, i, m1, red(FIN_GM_XI), gv, st));
                if (classical)
                    ENQ(FK_KERNEL_AXPY, launch_gm_rupdate(n, S->r, vec(i), i, S->gR, S->st, RUN_ACTIVE, gv, st));
            }
            return hipSuccess;
        }();
        if (e != hipSuccess)
            return fail(FK_E_HIP, "GMRES enqueue: %s", hipGetErrorString(e));
        HIP_TRY(hipMemcpyAsync(&S->h_init[2], S->st, sizeof(DevState), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(S->hR.data(), S->gR, S->hR.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (profile)
            harvest_profile(S, 0);
        DevState cur = S->h_init[2];
        if (cur.red_fault)
            return reduction_fault(S);
        if (cur.status == ST_ZERO_RHS) {
            HIP_TRY(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        if (cur.status != ST_CYCLE_DONE) {  // decided at the cycle start
            S->last = cur;
            return finish_solve(S);
        }
        const int used = cur.gi - 1;
        if (used == 0) {
            cur.status = ST_BREAKDOWN;
            S->last = cur;
            return finish_solve(S);
        }
        const double *R = S->hR.data();
        for (int i = used; i >= 1; --i) {  // R eta = xi by back substitution
            double sacc = R[i];
            for (int j = i + 1; j <= used; ++j)
                sacc = sacc - R[(size_t)i * m1 + j] * S->heta[j];
            S->heta[i] = sacc / R[(size_t)i * m1 + i];
        }
        HIP_TRY(hipMemcpyAsync(S->geta, S->heta.data(), (size_t)m1 * sizeof(double), hipMemcpyHostToDevice, st));
        HIP_TRY(launch_gm_xupdate(n, x, S->V, S->geta, used, S->st, gv, st));
        // next cycle: status back to running (the pinned word is free again)
        S->h_status[0] = ST_RUNNING;
        HIP_TRY(hipMemcpyAsync(reinterpret_cast<char *>(S->st) + offsetof(DevState, status), &S->h_status[0],
                               sizeof(int32_t), hipMemcpyHostToDevice, st));
    }
}

#undef ENQ

// Iterative refinement around the FP32 inner solver (FK_CG_MIXED).
static fk_status solve_mixed(fk_solver S, const double *b, double *x, bool profile, bool graph)
{
    DevState init{};
    init.status = ST_RUNNING;
    init.rtol = S->o.rtol;
    init.max_iter = S->o.max_outer;
    init.hist_cap = S->hist_cap;
    S->h_init[1] = init;
    HIP_TRY(hipMemcpyAsync(S->st_outer, &S->h_init[1], sizeof(DevState), hipMemcpyHostToDevice, S->stream));
    hipError_t e = mixed_outer(S, b, x, false, profile);  // r_0
    if (e != hipSuccess)
        return fail(FK_E_HIP, "refinement residual: %s", hipGetErrorString(e));
    DevState outer = S->h_init[2];
    if (outer.red_fault)
        return reduction_fault(S);
    int64_t used = 0;
    while (outer.status == ST_RUNNING) {
        if (S->sweeps >= S->o.max_outer || used >= S->o.max_iter) {
            outer.status = ST_NOT_CONVERGED;
            break;
        }
        fk_status fs = run_batches(S, nullptr, x, S->o.inner_rtol, S->o.max_iter - used, 0, profile, graph);
        if (fs != FK_OK)
            return fs;
        used += S->last.it;
        if (S->last.status == ST_BREAKDOWN) {
            outer.status = ST_BREAKDOWN;
            break;
        }
        if (S->last.it == 0) {  // no inner iteration: the correction would be 0
            outer.status = ST_NOT_CONVERGED;
            break;
        }
        e = mixed_outer(S, b, x, true, profile);  // x_{j+1} = x_j + d; r_{j+1}
        if (e != hipSuccess)
            return fail(FK_E_HIP, "refinement step: %s", hipGetErrorString(e));
        S->sweeps++;
        outer = S->h_init[2];
        if (outer.red_fault)
            return reduction_fault(S);
    }
    if (outer.status == ST_ZERO_RHS) {
        HIP_TRY(hipMemsetAsync(x, 0, (size_t)S->n * sizeof(double), S->stream));
        HIP_TRY(hipStreamSynchronize(S->stream));
    }
    outer.it = (int32_t)used;
    S->last = outer;
    return finish_solve(S);
}

extern "C" fk_status fk_solve(fk_solver S, const double *b, double *x)
{
    if (!S || !b || !x)
        return fail(FK_E_ARG, "NULL argument");
    S->solved = false;
    S->sweeps = 0;
    if (S->red_dirty) {
        HIP_TRY(launch_red_init(S->partials, S->stream));
        S->red_dirty = false;
    }
    const bool profile = (S->o.flags & FK_FLAG_PROFILE) != 0;
    const bool graph = !profile && (S->o.flags & FK_FLAG_GRAPH) != 0 && S->stream != nullptr;
    if (profile) {
        for (int k = 0; k < FK_KERNEL_KINDS; ++k) {
            S->prof_us[k] = 0.0;
            S->prof_n[k] = 0;
        }
    }
    if (S->mixed)
        return solve_mixed(S, b, x, profile, graph);
    if (S->gmres)
        return solve_gmres(S, b, x, profile);

    if (S->small) {
        DevState init{};
        init.status = ST_RUNNING;
        init.rtol = S->o.rtol;
        init.max_iter = S->o.max_iter;
        init.hist_cap = S->hist_cap;
        S->h_init[0] = init;
        HIP_TRY(hipMemcpyAsync(S->st, &S->h_init[0], sizeof(DevState), hipMemcpyHostToDevice, S->stream));
        const bool bicg = is_bicg_pipelined(S->o.method);
        std::vector<hipEvent_t> &pool = S->prof_ev[0];
        if (profile) {
            while (pool.size() < 2) {
                hipEvent_t ev;
                HIP_TRY(hipEventCreate(&ev));
                pool.push_back(ev);
            }
            set_launch_timing(pool[0], pool[1]);
        }
        hipError_t es = launch_small(bicg, S->A->view(), b, x, S->st, S->hist, S->scal,
                                     S->small_stage, S->stream);
        set_launch_timing(nullptr, nullptr);
        if (es != hipSuccess)
            return fail(FK_E_HIP, "single-workgroup solve: %s", hipGetErrorString(es));
        HIP_TRY(hipMemcpyAsync(&S->h_init[2], S->st, sizeof(DevState), hipMemcpyDeviceToHost, S->stream));
        HIP_TRY(hipStreamSynchronize(S->stream));
        S->last = S->h_init[2];
        if (profile) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pool[0], pool[1]) == hipSuccess) {
                S->prof_us[FK_KERNEL_SMALL] = 1000.0 * (double)ms;
                S->prof_n[FK_KERNEL_SMALL] = 1;
            }
        }
        if (S->last.status == ST_ZERO_RHS) {
            HIP_TRY(hipMemsetAsync(x, 0, (size_t)S->n * sizeof(double), S->stream));
            HIP_TRY(hipStreamSynchronize(S->stream));
        }
        return finish_solve(S);
    }

    fk_status fs = run_batches(S, b, x, S->o.rtol, S->o.max_iter, S->hist_cap, profile, graph);
    if (fs != FK_OK)
        return fs;
    return finish_solve(S);
}

// Map the final device state to the returned status.
static fk_status finish_solve(fk_solver S)
{
    S->solved = true;
    switch (S->last.status) {
    case ST_CONVERGED:
    case ST_ZERO_RHS:
        S->last_status = FK_OK;
        break;
    case ST_BREAKDOWN:
        S->last_status = FK_BREAKDOWN;
        break;
    default:
        S->last_status = FK_NOT_CONVERGED;
        break;
    }
    if (S->last_status == FK_BREAKDOWN)
        fail(FK_BREAKDOWN, "breakdown at iteration %d", S->last.it);
    else if (S->last_status == FK_NOT_CONVERGED)
        fail(FK_NOT_CONVERGED, "not converged after %d iterations (rel. residual %.3e)", S->last.it,
             S->last.last_rel);
    return S->last_status;
}

// ------------------------------------------------ solve without allocation

// The work memory of fk_solve_noalloc: one array per device, part of this
// file's code object, so it exists from the library's first use on a device
// until the process ends.  Regions, each 256-byte aligned: the device state,
// the reduction scratch (partials, arrival counters, published partials),
// then r, p and A p of FK_NOALLOC_MAX_N doubles each.  In host code the name
// `scratch` is only a host-side stand-in: host code passes kernels the
// device address that hipGetSymbolAddress returns for the current device.
namespace {
constexpr size_t NA_ALIGN = 256 / sizeof(double);
constexpr size_t na_round(size_t d) { return (d + NA_ALIGN - 1) / NA_ALIGN * NA_ALIGN; }
constexpr size_t NA_STATE = 0;
constexpr size_t NA_RED = NA_STATE + na_round(sizeof(DevState) / sizeof(double));
constexpr size_t NA_VEC = NA_RED + na_round(RED_SCRATCH_DOUBLES);
constexpr size_t NA_VEC_STRIDE = na_round(FK_NOALLOC_MAX_N);
constexpr size_t NA_DOUBLES = NA_VEC + 3 * NA_VEC_STRIDE;
static_assert(sizeof(DevState) % sizeof(double) == 0, "the state occupies whole doubles");
static_assert(NA_DOUBLES * sizeof(double) == FK_NOALLOC_BYTES, "fk.h states the array's size");

constexpr int NA_MAX_DEVICES = 64;
std::mutex g_na_mu[NA_MAX_DEVICES];   // one solve at a time per device
double *g_na_ptr[NA_MAX_DEVICES] = {};  // device address of `scratch`, per device
}  // namespace

static __device__ __align__(256) double scratch[NA_DOUBLES];

// The device address of `scratch` on `device` (the current device), looked
// up once per device.  Called with g_na_mu[device] held.
static fk_status noalloc_base(int device, double **base)
{
    if (!g_na_ptr[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(FK_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_na_ptr[device] = static_cast<double *>(ptr);
    }
    *base = g_na_ptr[device];
    return FK_OK;
}

extern "C" fk_status fk_solve_noalloc(fk_csr A, const fk_opts *o, const double *b, double *x, void *hip_stream,
                                      int32_t *iterations, double *rel_res)
{
    if (!A || !o || !b || !x)
        return fail(FK_E_ARG, "NULL argument");
    if (o->method != FK_CG_PIPELINED)
        return fail(FK_E_ARG, "fk_solve_noalloc solves with FK_CG_PIPELINED only");
    if (!(o->rtol >= 0.0) || !std::isfinite(o->rtol))
        return fail(FK_E_ARG, "rtol must be finite and >= 0");
    if (o->max_iter < 0)
        return fail(FK_E_ARG, "max_iter < 0");
    if (o->unroll < 0 || o->unroll > 4096)
        return fail(FK_E_ARG, "unroll outside [0, 4096]");
    if (o->record_history != 0)
        return fail(FK_E_ARG, "fk_solve_noalloc keeps no history (record_history must be 0)");
    if (o->flags & ~FK_FLAG_NO_SMALL)
        return fail(FK_E_ARG, "fk_solve_noalloc takes only FK_FLAG_NO_SMALL (flags 0x%x)", o->flags);
    if (A->n > FK_NOALLOC_MAX_N)
        return fail(FK_E_ARG, "n = %lld exceeds FK_NOALLOC_MAX_N = %d", (long long)A->n, FK_NOALLOC_MAX_N);
    int device = -1;
    HIP_TRY(hipGetDevice(&device));
    if (device != A->device)
        return fail(FK_E_ARG, "the matrix lives on device %d, the current device is %d", A->device, device);
    if (device < 0 || device >= NA_MAX_DEVICES)
        return fail(FK_E_ARG, "device %d outside [0, %d)", device, NA_MAX_DEVICES);

    std::lock_guard<std::mutex> lock(g_na_mu[device]);
    double *base = nullptr;
    fk_status fs = noalloc_base(device, &base);
    if (fs != FK_OK)
        return fs;
    hipStream_t st = (hipStream_t)hip_stream;

    // A solver view over the static array (no events, no pinned memory, no
    // history): the same enqueue functions as fk_solve, so the same kernels
    // in the same order.
    fk_solver_s S;
    S.A = A;
    S.o = *o;
    if (S.o.unroll == 0)
        S.o.unroll = 32;
    S.stream = st;
    S.n = A->n;
    S.grid_spmv = A->spmv_grid();
    S.grid_vec = vec_grid(A->n);
    S.st = reinterpret_cast<DevState *>(base + NA_STATE);
    S.partials = base + NA_RED;
    S.r = base + NA_VEC;
    S.p = S.r + NA_VEC_STRIDE;
    S.ap = S.p + NA_VEC_STRIDE;
    S.small = small_path_ok(A, S.o);
    S.small_stage = S.small && small_staged_lds_bytes(0, A->n, A->nnz) + SMALL_STATIC_LDS <=
                                   max_lds_per_workgroup(A->device);

    // The array keeps the last call's contents: the partial slots start
    // empty and the state from its initial values (fill kernels, no memset
    // nodes).
    HIP_TRY(launch_red_init(S.partials, st));
    HIP_TRY(launch_state_init(S.st, S.o.rtol, S.o.max_iter, 0, st));
    DevState last{};
    if (S.small) {
        HIP_TRY(launch_small(0, A->view(), b, x, S.st, nullptr, nullptr, S.small_stage, st));
    } else {
        Enq q{&S, false, 0};
        hipError_t e = enqueue_setup(&S, q, b, x);
        int64_t launched = 0;
        while (e == hipSuccess) {
            const int64_t todo = std::min<int64_t>(S.o.unroll, (int64_t)S.o.max_iter - launched);
            for (int64_t i = 0; i < todo && e == hipSuccess; ++i)
                e = enqueue_iteration(&S, q, x, launched + i + 1 == S.o.max_iter);
            if (e != hipSuccess)
                break;
            launched += todo;
            int32_t status = ST_RUNNING;
            e = hipMemcpyAsync(&status, reinterpret_cast<const char *>(S.st) + offsetof(DevState, status),
                               sizeof status, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess)
                e = hipStreamSynchronize(st);
            if (e != hipSuccess || status != ST_RUNNING || launched >= S.o.max_iter)
                break;
        }
        if (e != hipSuccess)
            return fail(FK_E_HIP, "fk_solve_noalloc: %s", hipGetErrorString(e));
    }
    HIP_TRY(hipMemcpyAsync(&last, S.st, sizeof(DevState), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (S.small && last.status == ST_ZERO_RHS) {
        HIP_TRY(launch_clear(x, A->n, vec_grid(A->n), st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    if (iterations)
        *iterations = last.it;
    if (rel_res)
        *rel_res = last.last_rel;
    if (last.red_fault)
        return fail(FK_E_HIP, "a cross-workgroup reduction did not complete; the solve is void");
    switch (last.status) {
    case ST_CONVERGED:
    case ST_ZERO_RHS:
        return FK_OK;
    case ST_BREAKDOWN:
        return fail(FK_BREAKDOWN, "breakdown at iteration %d", last.it);
    default:
        return fail(FK_NOT_CONVERGED, "not converged after %d iterations (rel. residual %.3e)", last.it,
                    last.last_rel);
    }
}

extern "C" fk_status fk_solver_uses_small(fk_solver S, int32_t *small)
{
    if (!S || !small)
        return fail(FK_E_ARG, "NULL argument");
    *small = S->small ? 1 : 0;
    return FK_OK;
}

extern "C" fk_status fk_get_refinements(fk_solver S, int32_t *sweeps)
{
    if (!S || !sweeps)
        return fail(FK_E_ARG, "NULL argument");
    if (!S->solved)
        return fail(FK_E_STATE, "no completed solve");
    *sweeps = S->sweeps;
    return FK_OK;
}

extern "C" fk_status fk_get_iterations(fk_solver S, int32_t *k)
{
    if (!S || !k)
        return fail(FK_E_ARG, "NULL argument");
    if (!S->solved)
        return fail(FK_E_STATE, "no completed solve");
    *k = S->last.it;
    return FK_OK;
}

extern "C" fk_status fk_get_residual(fk_solver S, double *rel)
{
    if (!S || !rel)
        return fail(FK_E_ARG, "NULL argument");
    if (!S->solved)
        return fail(FK_E_STATE, "no completed solve");
    *rel = S->last.last_rel;
    return FK_OK;
}

extern "C" fk_status fk_get_residual_history(fk_solver S, double *out, int32_t cap, int32_t *len)
{
    if (!S || !len || (cap > 0 && !out) || cap < 0)
        return fail(FK_E_ARG, "bad argument");
    if (!S->solved)
        return fail(FK_E_STATE, "no completed solve");
    if (!S->hist)
        return fail(FK_E_STATE, "solver created without record_history");
    *len = std::min(S->mixed ? S->sweeps + 1 : S->last.it + 1, S->hist_cap);
    const int32_t m = std::min(cap, *len);
    if (m > 0)
        HIP_TRY(hipMemcpyAsync(out, S->hist, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
    return FK_OK;
}

extern "C" fk_status fk_get_scalars(fk_solver S, double *out, int32_t cap, int32_t *len)
{
    if (!S || !len || (cap > 0 && !out) || cap < 0)
        return fail(FK_E_ARG, "bad argument");
    if (!S->solved)
        return fail(FK_E_STATE, "no completed solve");
    if (S->mixed || S->gmres)
        return fail(FK_E_STATE, "no per-iteration scalars for this method");
    if (!S->scal)
        return fail(FK_E_STATE, "solver created without record_history and FK_FLAG_SCALARS");
    *len = std::min(S->last.it, S->hist_cap);
    const int32_t m = std::min(cap, *len);
    if (m > 0)
        HIP_TRY(hipMemcpyAsync(out, S->scal, (size_t)m * 4 * sizeof(double), hipMemcpyDeviceToHost, S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
    return FK_OK;
}

extern "C" fk_status fk_get_kernel_times(fk_solver S, double *avg_us, int32_t *count, int32_t cap)
{
    if (!S || cap < 0 || (cap > 0 && (!avg_us || !count)))
        return fail(FK_E_ARG, "bad argument");
    for (int k = 0; k < cap && k < FK_KERNEL_KINDS; ++k) {
        count[k] = S->prof_n[k];
        avg_us[k] = S->prof_n[k] ? S->prof_us[k] / S->prof_n[k] : 0.0;
    }
    return FK_OK;
}

// ------------------------------------------------------- kernel entry points

// A reduction of one of the kernel entry points gave up waiting: clear the
// fault, rewrite the scratch's empty markers and report the call void.
static fk_status scratch_fault(DevState *st, double *partials, hipStream_t s)
{
    (void)hipMemsetAsync(reinterpret_cast<char *>(st) + offsetof(DevState, red_fault), 0, sizeof(int32_t), s);
    (void)launch_red_init(partials, s);
    (void)hipStreamSynchronize(s);
    return fail(FK_E_HIP, "a cross-workgroup reduction did not complete; the result is void");
}

extern "C" fk_status fk_spmv(fk_csr A, const double *p, double *q, double *dots_host, void *hip_stream)
{
    if (!A || !p || !q)
        return fail(FK_E_ARG, "NULL argument");
    if ((const void *)p == (const void *)q)
        return fail(FK_E_ARG, "p and q must not alias");
    hipStream_t s = (hipStream_t)hip_stream;
    const int dots = dots_host ? (D_YV | D_YY) : 0;
    RedArgs red{A->st, A->partials, nullptr, nullptr, FIN_NONE, RUN_ALWAYS};
    HIP_TRY(launch_spmv_dots(A->view(), p, q, nullptr, dots, red, A->spmv_grid(), s));
    if (dots_host) {
        DevState d;
        HIP_TRY(hipMemcpyAsync(&d, A->st, sizeof d, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (d.red_fault)
            return scratch_fault(A->st, A->partials, s);
        dots_host[0] = d.dots[0];
        dots_host[1] = d.dots[1];
    } else {
        HIP_TRY(hipStreamSynchronize(s));
    }
    return FK_OK;
}

extern "C" fk_status fk_spmv_time(fk_csr A, const double *p, double *q, int32_t mode, int32_t reps,
                                  double *avg_us, void *hip_stream)
{
    if (!A || !p || !q || !avg_us)
        return fail(FK_E_ARG, "NULL argument");
    if ((const void *)p == (const void *)q)
        return fail(FK_E_ARG, "p and q must not alias");
    if (reps < 1 || mode < 0 || mode > 2)
        return fail(FK_E_ARG, "reps must be >= 1 and mode 0, 1 or 2");
    hipStream_t s = (hipStream_t)hip_stream;
    const int kernels = mode == 2 ? 2 : 1;
    std::vector<hipEvent_t> ev((size_t)2 * kernels * reps, nullptr);
    auto release = [&]() {
        for (auto e : ev)
            if (e)
                (void)hipEventDestroy(e);
    };
    for (auto &e : ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            release();
            return fail(FK_E_HIP, "hipEventCreate failed");
        }
    }
    hipError_t e = hipSuccess;
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        hipEvent_t *pe = &ev[(size_t)2 * kernels * r];
        RedArgs red{A->st, A->partials, nullptr, nullptr, FIN_NONE, RUN_ALWAYS};
        set_launch_timing(pe[0], pe[1]);
        e = launch_spmv_dots(A->view(), p, q, nullptr, mode == 1 ? (D_YV | D_YY) : 0, red, A->spmv_grid(), s);
        if (e == hipSuccess && mode == 2) {
            set_launch_timing(pe[2], pe[3]);
            e = launch_dot(A->n, q, p, q, 2, red, vec_grid(A->n), s);
        }
    }
    set_launch_timing(nullptr, nullptr);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    double total = 0.0;
    for (size_t i = 0; e == hipSuccess && i < ev.size(); i += 2) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
        total += ms;
    }
    release();
    if (e != hipSuccess)
        return fail(FK_E_HIP, "fk_spmv_time: %s", hipGetErrorString(e));
    DevState d;
    HIP_TRY(hipMemcpyAsync(&d, A->st, sizeof d, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (d.red_fault)
        return scratch_fault(A->st, A->partials, s);
    *avg_us = 1000.0 * total / reps;
    return FK_OK;
}

extern "C" fk_status fk_spmv32(fk_csr A, const float *p, float *q, int32_t f32acc, double *dots_host,
                               void *hip_stream)
{
    if (!A || !p || !q)
        return fail(FK_E_ARG, "NULL argument");
    if ((const void *)p == (const void *)q)
        return fail(FK_E_ARG, "p and q must not alias");
    if (f32acc != 0 && f32acc != 1)
        return fail(FK_E_ARG, "f32acc must be 0 or 1");
    hipStream_t s = (hipStream_t)hip_stream;
    if (A->nnz > 0 && A->vals32_layout != A->layout) {
        // the FP32 values in the order the current layout's products read them
        dev_free(A->vals32);
        A->vals32_layout = -1;
        const int64_t m = A->stored_entries();
        fk_status fs = dev_alloc(&A->vals32, (size_t)m, "FP32 values");
        if (fs != FK_OK)
            return fs;
        const double *src = A->slots() ? A->dg_vals : A->sliced() ? A->sell_vals : A->vals;
        HIP_TRY(launch_to_f32(m, A->vals32, src, vec_grid(m), s));
        A->vals32_layout = A->layout;
    }
    RedArgs red{A->st, A->partials, nullptr, nullptr, FIN_NONE, RUN_ALWAYS};
    HIP_TRY(launch_spmv32(A->view(), A->vals32, p, q, red, A->spmv_grid(), s, f32acc != 0));
    DevState d;
    HIP_TRY(hipMemcpyAsync(&d, A->st, sizeof d, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (d.red_fault)
        return scratch_fault(A->st, A->partials, s);
    if (dots_host) {
        dots_host[0] = d.dots[0];
        dots_host[1] = d.dots[1];
    }
    return FK_OK;
}

namespace {
std::mutex g_dot_mu;
DevState *g_dot_st = nullptr;
double *g_dot_partials = nullptr;
}  // namespace

extern "C" fk_status fk_dot(int64_t n, const double *a, const double *b, double *out, void *hip_stream)
{
    if (!out || n < 0 || (n > 0 && (!a || !b)))
        return fail(FK_E_ARG, "bad argument");
    if (n == 0) {
        *out = 0.0;
        return FK_OK;
    }
    std::lock_guard<std::mutex> lock(g_dot_mu);
    hipStream_t s = (hipStream_t)hip_stream;
    if (!g_dot_st) {
        fk_status st = dev_alloc(&g_dot_st, 1, "dot state");
        if (st != FK_OK)
            return st;
        st = dev_alloc(&g_dot_partials, RED_SCRATCH_DOUBLES, "dot partials");
        if (st != FK_OK) {
            dev_free(g_dot_st);
            return st;
        }
        HIP_TRY(hipMemsetAsync(g_dot_st, 0, sizeof(DevState), s));
        HIP_TRY(launch_red_init(g_dot_partials, s));
    }
    RedArgs red{g_dot_st, g_dot_partials, nullptr, nullptr, FIN_NONE, RUN_ALWAYS};
    HIP_TRY(launch_dot(n, a, b, nullptr, 1, red, vec_grid(n), s));
    DevState d;
    HIP_TRY(hipMemcpyAsync(&d, g_dot_st, sizeof d, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (d.red_fault)
        return scratch_fault(g_dot_st, g_dot_partials, s);
    *out = d.dots[0];
    return FK_OK;
}

extern "C" fk_status fk_copy(void *dst, const void *src, int64_t n_bytes, void *hip_stream)
{
    if (n_bytes < 0 || (n_bytes > 0 && (!dst || !src)))
        return fail(FK_E_ARG, "bad argument");
    if (n_bytes == 0)
        return FK_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    static const int gmax = env_int("FK_COPY_GRID", 2048, 1, 65535);
    const int64_t n16 = n_bytes / 16;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(gmax, (n16 + WG - 1) / WG));
    HIP_TRY(launch_copy(dst, src, n_bytes, grid, s));
    return FK_OK;
}

extern "C" fk_status fk_axpby(int64_t n, double alpha, const double *x, double beta, const double *y,
                              double *out, void *hip_stream)
{
    if (n < 0 || (n > 0 && (!x || !y || !out)))
        return fail(FK_E_ARG, "bad argument");
    if (n == 0)
        return FK_OK;
    HIP_TRY(launch_axpby(n, alpha, x, beta, y, out, vec_grid(n), (hipStream_t)hip_stream));
    return FK_OK;
}

extern "C" const char *fk_status_str(fk_status s)
{
    switch (s) {
    case FK_OK: return "FK_OK";
    case FK_E_ARG: return "FK_E_ARG";
    case FK_E_CSR: return "FK_E_CSR";
    case FK_E_HIP: return "FK_E_HIP";
    case FK_E_OOM: return "FK_E_OOM";
    case FK_NOT_CONVERGED: return "FK_NOT_CONVERGED";
    case FK_BREAKDOWN: return "FK_BREAKDOWN";
    case FK_E_STATE: return "FK_E_STATE";
    }
    return "FK_UNKNOWN";
}

extern "C" const char *fk_last_error(void) { return g_err.c_str(); }

extern "C" const char *fk_version(void) { return "fk 0.1 gfx950"; }
