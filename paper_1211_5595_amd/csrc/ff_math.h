// ff_math.h -- float-float ("double-single") arithmetic for the per-ray
// set-up on the device.  Error-free transformations after Knuth (TwoSum),
// Dekker (FastTwoSum) and the FMA form of TwoProduct; division and square
// root by one or two Newton corrections of the binary32 result.  Relative
// error of each operation is a small multiple of 2^-44.  The library is
// built with -ffp-contract=off so the compiler keeps every rounding step.
#pragma once

#include "rt_internal.h"

namespace rtv {

__device__ __forceinline__ ff ff_make(float a) { return ff{a, 0.0f}; }

__device__ __forceinline__ ff two_sum(float a, float b) {
    float s = a + b;
    float bb = s - a;
    float e = (a - (s - bb)) + (b - bb);
    return ff{s, e};
}

// Requires |a| >= |b| (or a == 0).
__device__ __forceinline__ ff fast_two_sum(float a, float b) {
    float s = a + b;
    float e = b - (s - a);
    return ff{s, e};
}

__device__ __forceinline__ ff two_prod(float a, float b) {
    float p = a * b;
    return ff{p, fmaf(a, b, -p)};
}

__device__ __forceinline__ ff ff_add(ff a, ff b) {
    ff s = two_sum(a.hi, b.hi);
    ff t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ ff ff_neg(ff a) { return ff{-a.hi, -a.lo}; }
__device__ __forceinline__ ff ff_sub(ff a, ff b) { return ff_add(a, ff_neg(b)); }

__device__ __forceinline__ ff ff_mul(ff a, ff b) {
    ff p = two_prod(a.hi, b.hi);
    p.lo = fmaf(a.hi, b.lo, p.lo);
    p.lo = fmaf(a.lo, b.hi, p.lo);
    return fast_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ ff ff_mul_f(ff a, float b) {
    ff p = two_prod(a.hi, b);
    p.lo = fmaf(a.lo, b, p.lo);
    return fast_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ ff ff_div(ff a, ff b) {
    float q1 = a.hi / b.hi;
    ff r = ff_sub(a, ff_mul_f(b, q1));
    float q2 = r.hi / b.hi;
    r = ff_sub(r, ff_mul_f(b, q2));
    float q3 = r.hi / b.hi;
    ff q = fast_two_sum(q1, q2);
    return ff_add(q, ff_make(q3));
}

// a > 0.
__device__ __forceinline__ ff ff_sqrt(ff a) {
    float x = sqrtf(a.hi);
    ff r = ff_sub(a, two_prod(x, x));
    float c = r.hi / (2.0f * x);
    return fast_two_sum(x, c);
}

__device__ __forceinline__ bool ff_lt(ff a, ff b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
__device__ __forceinline__ bool ff_le(ff a, ff b) { return a.hi < b.hi || (a.hi == b.hi && a.lo <= b.lo); }
__device__ __forceinline__ ff ff_max(ff a, ff b) { return ff_lt(a, b) ? b : a; }
__device__ __forceinline__ ff ff_min(ff a, ff b) { return ff_lt(b, a) ? b : a; }

// floor of a float-float value as an integer (|a| < 2^30).
__device__ __forceinline__ int ff_floor_int(ff a) {
    float fh = floorf(a.hi);
    int m = (int)fh;
    if (fh == a.hi) m += (int)floorf(a.lo);
    return m;
}

// Signed 32.32 fixed point of a float-float value (|a| < 2^30): returns
// round(a * 2^32) within one unit.  hi * 2^32 and lo * 2^32 are exact
// power-of-two scalings; each is an integer-valued binary32 number (or is
// rounded to one) and converts to int64 exactly.  Subtracting floor(hi)
// from hi instead would drop a bit whenever -1 < hi < 0.
__device__ __forceinline__ long long ff_to_fixed32(ff a) {
    const long long H = (long long)rintf(a.hi * 4294967296.0f);
    const long long L = (long long)rintf(a.lo * 4294967296.0f);
    return H + L;
}

}  // namespace rtv
