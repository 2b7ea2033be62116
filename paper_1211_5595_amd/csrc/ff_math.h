// ff_math.h -- float-float ("double-single") arithmetic for the per-ray
// set-up on the device.  Error-free transformations after Knuth (TwoSum),
// Dekker (FastTwoSum) and the FMA form of TwoProduct; quotient, reciprocal
// and reciprocal square root from the hardware's binary32 estimates with
// Newton corrections against float-float residuals.  Relative
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

// a / b: quotient digits from the hardware reciprocal estimate of b.hi
// (within one unit in the last place), each corrected against the exact
// float-float residual, so the estimate's error does not reach the result.
__device__ __forceinline__ ff ff_div(ff a, ff b) {
    const float rb = __builtin_amdgcn_rcpf(b.hi);
    const float q1 = a.hi * rb;
    ff r = ff_sub(a, ff_mul_f(b, q1));
    const float q2 = r.hi * rb;
    r = ff_sub(r, ff_mul_f(b, q2));
    const float q3 = r.hi * rb;
    ff q = fast_two_sum(q1, q2);
    return ff_add(q, ff_make(q3));
}

// 1 / b, b != 0: the hardware estimate x (within one unit in the last place)
// with one Newton correction x + x (1 - b x), the residual in float-float.
__device__ __forceinline__ ff ff_rcp(ff b) {
    const float x = __builtin_amdgcn_rcpf(b.hi);
    const ff e = ff_sub(ff_make(1.0f), ff_mul_f(b, x));
    return fast_two_sum(x, x * e.hi);
}

// 1 / sqrt(a), a > 0: the hardware estimate y (within one unit in the last
// place) with one Newton correction y + y (1 - a y^2) / 2, the residual
// 1 - a y^2 formed in float-float.
__device__ __forceinline__ ff ff_rsqrt(ff a) {
    const float y = __builtin_amdgcn_rsqf(a.hi);
    const ff e = ff_sub(ff_make(1.0f), ff_mul(a, two_prod(y, y)));
    return fast_two_sum(y, y * (0.5f * e.hi));
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

// Signed 32.32 fixed point of a float-float value (|a| < 2^22): returns
// round(a * 2^32) within one unit.  hi * 2^32 and lo * 2^32 are exact
// power-of-two scalings; each is an integer-valued binary32 number (or is
// rounded to one) and converts exactly, hi's to a 64-bit integer and lo's,
// below 2^31 in magnitude, to a 32-bit one.  Subtracting floor(hi) from hi
// instead would drop a bit whenever -1 < hi < 0 (and so would splitting
// hi * 2^32 at 2^32 with a floor).
__device__ __forceinline__ long long ff_to_fixed32(ff a) {
    const long long H = (long long)rintf(a.hi * 4294967296.0f);
    const int L = (int)rintf(a.lo * 4294967296.0f);
    return H + (long long)L;
}

}  // namespace rtv
