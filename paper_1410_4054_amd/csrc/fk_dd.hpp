// Double-double accumulation shared by the device kernels: sums of exact
// FP64 products kept as an unevaluated pair (hi, lo) and rounded once.
#pragma once

#include <hip/hip_runtime.h>

namespace fk {

struct dd {
    double hi, lo;
};

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    double z = s - a;
    e = (a - (s - z)) + (b - z);
}

// (a.hi + a.lo) + (b.hi + b.lo), renormalised.  Commutative bit for bit.
__device__ __forceinline__ dd dd_add(dd a, dd b)
{
    double s, e;
    two_sum(a.hi, b.hi, s, e);
    e = e + (a.lo + b.lo);
    double h = s + e;
    return dd{h, e - (h - s)};
}

// acc += a * b, keeping the rounding errors of the product and the sum.
__device__ __forceinline__ void dd_fma(dd &acc, double a, double b)
{
    double p = a * b;
    double pe = __builtin_fma(a, b, -p);
    double s, e;
    two_sum(acc.hi, p, s, e);
    acc.hi = s;
    acc.lo = acc.lo + (e + pe);
}

// A double moved across lanes by the DPP unit (an operand modifier of a
// vector move: no LDS round trip).  Lanes whose source lies outside their
// row, and lanes of rows that ROW_MASK leaves out, read zero.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_double(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ dd dd_add_dpp(dd v)
{
    return dd_add(v, dd{dpp_double<CTRL, ROW_MASK>(v.hi), dpp_double<CTRL, ROW_MASK>(v.lo)});
}

__device__ __forceinline__ double lane_value(double x, int lane)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum of a double-double over the 64 lanes in a fixed tree on the DPP
// unit: within each row of 16 lanes shifts by 1, 2, 4 and 8 leave the
// row's sum in its lane 15; a broadcast of lane 15 into the next row adds
// row 0 into lane 31 and row 2 into lane 63, one of lane 31 into rows 2
// and 3 adds rows 0-1 into lane 63.  Returned to every lane.  The same
// additions in the same order as any other fixed tree, six deep, without
// the LDS round trip a lane shuffle costs at each level.
__device__ __forceinline__ dd wave_sum(dd v)
{
    v = dd_add_dpp<0x111, 0xf>(v);  // row_shr:1
    v = dd_add_dpp<0x112, 0xf>(v);  // row_shr:2
    v = dd_add_dpp<0x114, 0xf>(v);  // row_shr:4
    v = dd_add_dpp<0x118, 0xf>(v);  // row_shr:8
    v = dd_add_dpp<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = dd_add_dpp<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return dd{lane_value(v.hi, 63), lane_value(v.lo, 63)};
}

__device__ __forceinline__ dd wave_reduce(dd v) { return wave_sum(v); }

// The same tree for a float.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_float(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, true));
}

__device__ __forceinline__ float wave_sum(float v)
{
    v = v + dpp_float<0x111, 0xf>(v);
    v = v + dpp_float<0x112, 0xf>(v);
    v = v + dpp_float<0x114, 0xf>(v);
    v = v + dpp_float<0x118, 0xf>(v);
    v = v + dpp_float<0x142, 0xa>(v);
    v = v + dpp_float<0x143, 0xc>(v);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Sum of a double-double over lanes 0 .. width-1 (width a power of two, at
// most 64; the other lanes' values are ignored): an xor butterfly, so every
// lane of a group of `width` ends with the same sum after log2(width)
// dependent additions.
__device__ __forceinline__ dd lanes_sum(dd v, int width)
{
    for (int off = width >> 1; off >= 1; off >>= 1) {
        dd o;
        o.hi = __shfl_xor(v.hi, off, 64);
        o.lo = __shfl_xor(v.lo, off, 64);
        v = dd_add(v, o);
    }
    return v;
}

}  // namespace fk
