// gb_wide_limbs.h -- Montgomery arithmetic modulo an odd q over N 28-bit limbs
// (R = 2^(28 N); N = 3, 4 or 5 for q below 2^72, 2^100 or 2^128), the inner
// arithmetic of the Baillie-PSW test past 2^64.
//
// With 28-bit limbs every 32x32-bit limb product fits 60 bits, so a column of
// the product accumulates in one 64-bit register by 32x32+64-bit multiply-adds
// alone: no carry is propagated inside a product, and no register pair has to
// be rebuilt for an addend.  Values are kept lazily: with q < R / 2^12, a
// Montgomery product takes operands with limbs below 2^30 and values below 8q,
// and returns normalized limbs (all but the top one below 2^28) with a value
// below a*b/R + q < 1.02 q; sums of such values stay within the operand bounds,
// and subtractions are written as additions of an exact 2q - y.  Only
// comparisons reduce fully.  A product costs 2 N^2 multiply-adds, so q gets the
// fewest limbs that leave it 12 bits below R (18 near 2^64, 50 near 2^128).
//
// Plain integer code: the functions are device functions in the kernels and
// compile for the host (GB_WIDE_FN defined before inclusion) in the tests.
#pragma once

#include <stdint.h>

#ifndef GB_WIDE_FN
#define GB_WIDE_FN __device__ __forceinline__
#endif

template <int N>
struct wl {
    uint32_t l[N];   // value = sum of l[j] * 2^(28 j)
};

constexpr uint32_t kLimbMask = (1u << 28) - 1;

// The limb count for moduli below 2^bits: the fewest N with bits <= 28 N - 12.
GB_WIDE_FN int wl_limbs_for(int bits)
{
    return bits <= 72 ? 3 : (bits <= 100 ? 4 : 5);
}

// Limbs of lo + 2^64 hi (normalized; the value must be below 2^(28 N)).
template <int N>
GB_WIDE_FN wl<N> wl_from(uint64_t lo, uint64_t hi)
{
    const uint32_t t[5] = {(uint32_t)lo & kLimbMask, (uint32_t)(lo >> 28) & kLimbMask,
                           (uint32_t)((lo >> 56) | (hi << 8)) & kLimbMask,
                           (uint32_t)(hi >> 20) & kLimbMask, (uint32_t)(hi >> 48)};
    wl<N> r;
#pragma unroll
    for (int j = 0; j < N; ++j)
        r.l[j] = t[j];
    if (N < 5)   // the top limb takes every bit above it
        r.l[N - 1] = (uint32_t)((N == 3 ? (lo >> 56) | (hi << 8) : hi >> 20));
    return r;
}

// -q^-1 mod 2^28 for odd q (Newton steps on the low 32 bits double the
// correct low bits: 3, 6, 12, 24, 48).
GB_WIDE_FN uint32_t wl_qinv(uint64_t q_lo)
{
    const uint32_t q0 = (uint32_t)q_lo;
    uint32_t inv = q0;
    for (int i = 0; i < 4; ++i)
        inv *= 2u - q0 * inv;
    return (0u - inv) & kLimbMask;
}

// Montgomery product a * b * 2^(-28 N) mod q (see the bounds above); qi = wl_qinv.
template <int N>
GB_WIDE_FN wl<N> wl_mont(const wl<N> &a, const wl<N> &b, const wl<N> &q, uint32_t qi)
{
    // c[j]: column i + j of the running value in row i (below 2^63: at most
    // five products below 2^60 and five below 2^56 each, plus carries)
    uint64_t c[N];
#pragma unroll
    for (int j = 0; j < N; ++j)
        c[j] = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const uint64_t bi = b.l[i];
#pragma unroll
        for (int j = 0; j < N; ++j)
            c[j] += a.l[j] * bi;
        const uint64_t m = ((uint32_t)c[0] * qi) & kLimbMask;   // the low limb becomes zero
#pragma unroll
        for (int j = 0; j < N; ++j)
            c[j] += m * q.l[j];
        const uint64_t carry = c[0] >> 28;
#pragma unroll
        for (int j = 0; j < N - 1; ++j)
            c[j] = c[j + 1];
        c[0] += carry;
        c[N - 1] = 0;
    }
    wl<N> r;
#pragma unroll
    for (int j = 0; j < N - 2; ++j) {
        r.l[j] = (uint32_t)c[j] & kLimbMask;
        c[j + 1] += c[j] >> 28;
    }
    r.l[N - 2] = (uint32_t)c[N - 2] & kLimbMask;
    r.l[N - 1] = (uint32_t)(c[N - 2] >> 28);
    return r;
}

// Q x mod q for a small signed integer Q (0 < |Q| < 2^15) and x normalized with
// a value below 1.02 q (a Montgomery product's output), in the Montgomery form
// of x's residue times Q; qrecip = 1/q in double precision.  The result is
// normalized with a value in [0, 3q].  The quotient t of |Q| x by q is below
// 2^16 and its double-precision estimate e has a relative error below 2^-49,
// so e is t - 1, t or t + 1; then |Q| x - (e - 1) q (e >= 1; |Q| x when e = 0,
// where t <= 1) lies in [0, 3q) and (e + 2) q - |Q| x in (0, 3q].  One pass of
// signed multiply-adds forms Q x + u q limb by limb, u = 1 - e or e + 2.
template <int N>
GB_WIDE_FN wl<N> wl_mul_q(const wl<N> &x, int32_t Q, const wl<N> &q, double qrecip)
{
    double xd = (double)x.l[N - 1];
#pragma unroll
    for (int j = N - 2; j >= 0; --j)
        xd = xd * 268435456.0 + (double)x.l[j];
    const uint32_t a = Q < 0 ? (uint32_t)(-Q) : (uint32_t)Q;
    const int32_t e = (int32_t)((double)a * xd * qrecip);
    const int32_t u = Q < 0 ? e + 2 : (e > 0 ? 1 - e : 0);
    wl<N> r;
    int64_t c = 0;
#pragma unroll
    for (int j = 0; j < N - 1; ++j) {
        c += (int64_t)(int32_t)x.l[j] * Q + (int64_t)(int32_t)q.l[j] * u;
        r.l[j] = (uint32_t)c & kLimbMask;
        c >>= 28;   // arithmetic: the floor of c / 2^28
    }
    r.l[N - 1] = (uint32_t)(c + (int64_t)(int32_t)x.l[N - 1] * Q + (int64_t)(int32_t)q.l[N - 1] * u);
    return r;
}

// x + y limb by limb (no carries: the caller keeps the operand bounds).
template <int N>
GB_WIDE_FN wl<N> wl_add(const wl<N> &x, const wl<N> &y)
{
    wl<N> r;
#pragma unroll
    for (int j = 0; j < N; ++j)
        r.l[j] = x.l[j] + y.l[j];
    return r;
}

// z - y for normalized z >= y (values), normalized result.
template <int N>
GB_WIDE_FN wl<N> wl_sub(const wl<N> &z, const wl<N> &y)
{
    wl<N> r;
    uint32_t b = 0;
#pragma unroll
    for (int j = 0; j < N - 1; ++j) {
        const uint32_t t = z.l[j] - y.l[j] - b;   // in (-2^28 - 1, 2^28)
        r.l[j] = t & kLimbMask;
        b = t >> 31;
    }
    r.l[N - 1] = z.l[N - 1] - y.l[N - 1] - b;
    return r;
}

// Carries propagated: all limbs but the top one below 2^28.
template <int N>
GB_WIDE_FN wl<N> wl_norm(const wl<N> &x)
{
    wl<N> r;
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < N - 1; ++j) {
        const uint32_t t = x.l[j] + c;
        r.l[j] = t & kLimbMask;
        c = t >> 28;
    }
    r.l[N - 1] = x.l[N - 1] + c;
    return r;
}

// x - q if x >= q, else x (x normalized, value below 2^(28 N - 9)).
template <int N>
GB_WIDE_FN wl<N> wl_csub(const wl<N> &x, const wl<N> &q)
{
    wl<N> d;
    uint32_t b = 0;
#pragma unroll
    for (int j = 0; j < N - 1; ++j) {
        const uint32_t t = x.l[j] - q.l[j] - b;
        d.l[j] = t & kLimbMask;
        b = t >> 31;
    }
    const uint32_t t = x.l[N - 1] - q.l[N - 1] - b;
    d.l[N - 1] = t;
    return (t >> 31) ? x : d;
}

// The residue of x in [0, q) for x (any limbs below 2^30) below (k + 1) q.
template <int N, int k>
GB_WIDE_FN wl<N> wl_canon(const wl<N> &x, const wl<N> &q)
{
    wl<N> r = wl_norm(x);
#pragma unroll
    for (int i = 0; i < k; ++i)
        r = wl_csub(r, q);
    return r;
}

template <int N>
GB_WIDE_FN bool wl_eq(const wl<N> &x, const wl<N> &y)
{
    uint32_t d = 0;
#pragma unroll
    for (int j = 0; j < N; ++j)
        d |= x.l[j] ^ y.l[j];
    return d == 0;
}

template <int N>
GB_WIDE_FN bool wl_zero(const wl<N> &x)
{
    uint32_t d = 0;
#pragma unroll
    for (int j = 0; j < N; ++j)
        d |= x.l[j];
    return d == 0;
}
