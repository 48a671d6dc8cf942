// gb_wide_u128.h -- unsigned 128-bit arithmetic of the verification past 2^64
// as two 64-bit words: comparisons, sums and differences, residues modulo an
// odd q, the product of a residue by a constant below 2^40 with a
// double-precision quotient estimate, and 2^(28 N) mod q (the Montgomery form
// of 1 for gb_wide_limbs.h).
//
// Plain integer and double code: device functions in the kernels, and host
// functions in the tests (GB_WIDE_FN and __umul64hi defined before inclusion).
#pragma once

#include <stdint.h>

#ifndef GB_WIDE_FN
#define GB_WIDE_FN __device__ __forceinline__
#endif

// An unsigned 128-bit integer as two 64-bit words.
struct u128w {
    uint64_t lo, hi;
};

GB_WIDE_FN bool w_lt(u128w a, u128w b)
{
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}
GB_WIDE_FN bool w_eq(u128w a, u128w b) { return a.hi == b.hi && a.lo == b.lo; }
GB_WIDE_FN bool w_zero(u128w a) { return (a.hi | a.lo) == 0; }

GB_WIDE_FN u128w w_add64(u128w a, uint64_t b)
{
    u128w r;
    r.lo = a.lo + b;
    r.hi = a.hi + (r.lo < b ? 1u : 0u);
    return r;
}

GB_WIDE_FN u128w w_sub64(u128w a, uint64_t b)
{
    u128w r;
    r.lo = a.lo - b;
    r.hi = a.hi - (a.lo < b ? 1u : 0u);
    return r;
}

GB_WIDE_FN u128w w_sub(u128w a, u128w b)
{
    u128w r;
    r.lo = a.lo - b.lo;
    r.hi = a.hi - b.hi - (a.lo < b.lo ? 1u : 0u);
    return r;
}

// (a + b) mod q and (a - b) mod q for a, b < q.
GB_WIDE_FN u128w w_addmod(u128w a, u128w b, u128w q)
{
    // a + b >= q  <=>  a >= q - b
    const u128w qb = w_sub(q, b);
    if (!w_lt(a, qb))
        return w_sub(a, qb);
    u128w r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (r.lo < b.lo ? 1u : 0u);
    return r;
}

GB_WIDE_FN u128w w_submod(u128w a, u128w b, u128w q)
{
    const u128w d = w_sub(a, b);
    if (!w_lt(a, b))
        return d;
    u128w r;
    r.lo = d.lo + q.lo;
    r.hi = d.hi + q.hi + (r.lo < q.lo ? 1u : 0u);
    return r;
}

// x * c mod q for x < q and 1 <= c < 2^40, q odd with qinv_d = 1 / q in double
// precision.  The quotient k = floor(x c / q) < 2^40 is estimated in double
// precision: with at most seven roundings the estimate's relative error is
// below 2^-50, so its absolute error is below 2^-10 and its floor is k - 1, k
// or k + 1.  R = x c - k' q is formed over three 64-bit words (its top word is
// -1, 0 or 1, as R lies in [-q, 2q)) and corrected once either way.
GB_WIDE_FN u128w w_mul_small(u128w x, uint64_t c, u128w q, double qinv_d)
{
    const double xd = (double)x.hi * 18446744073709551616.0 + (double)x.lo;
    const double kd = __builtin_floor(xd * (double)c * qinv_d);
    const uint64_t k = kd > 0.0 ? (uint64_t)kd : 0u;
    // T = x c and K = k q as (low, middle, top) words
    const uint64_t tl = x.lo * c;
    const uint64_t th = __umul64hi(x.lo, (uint64_t)c);
    const uint64_t tm = x.hi * c + th;
    const uint64_t tt = __umul64hi(x.hi, (uint64_t)c) + (tm < th ? 1u : 0u);
    const uint64_t kl = q.lo * k;
    const uint64_t kh = __umul64hi(q.lo, k);
    const uint64_t km = q.hi * k + kh;
    const uint64_t kt = __umul64hi(q.hi, k) + (km < kh ? 1u : 0u);
    u128w r;
    r.lo = tl - kl;
    const uint64_t b0 = tl < kl ? 1u : 0u;
    r.hi = tm - km - b0;
    const uint64_t b1 = (tm < km || tm - km < b0) ? 1u : 0u;
    const uint64_t rt = tt - kt - b1;
    if ((int64_t)rt < 0) {
        // R in [-q, 0): R + q, computed modulo 2^128
        r.lo += q.lo;
        r.hi += q.hi + (r.lo < q.lo ? 1u : 0u);
    } else if (rt != 0 || !w_lt(r, q)) {
        r = w_sub(r, q);   // R in [q, 2q)
    }
    return r;
}

// Reciprocal of q in double precision.
GB_WIDE_FN double w_recip_d(u128w q)
{
    return 1.0 / ((double)q.hi * 18446744073709551616.0 + (double)q.lo);
}

// 2^rbits mod q for odd q > 1 and rbits >= the bit length L of q (the
// Montgomery form of 1 for R = 2^rbits): from 2^(L-1) < q, multiplied by
// 2^(rbits + 1 - L) in steps of at most 2^40.
GB_WIDE_FN u128w w_r_mod(u128w q, int rbits)
{
    const int L = q.hi ? 128 - __builtin_clzll(q.hi) : 64 - __builtin_clzll(q.lo);
    u128w x = L > 64 ? u128w{0, 1ull << (L - 65)} : u128w{1ull << (L - 1), 0};
    const double qinv_d = w_recip_d(q);
    for (int s = rbits + 1 - L; s > 0; s -= 40)
        x = w_mul_small(x, 1ull << (s < 40 ? s : 40), q, qinv_d);
    return x;
}
