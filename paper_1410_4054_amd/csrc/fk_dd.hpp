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

__device__ __forceinline__ dd wave_reduce(dd v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        dd o;
        o.hi = __shfl_xor(v.hi, off, 64);
        o.lo = __shfl_xor(v.lo, off, 64);
        v = dd_add(v, o);
    }
    return v;
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
