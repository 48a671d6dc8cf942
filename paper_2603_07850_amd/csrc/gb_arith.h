// gb_arith.h -- integer arithmetic of the gfx950 kernels: 64-by-32-bit
// remainders without a hardware divider, exact integer square roots, and the
// deterministic 64-bit Miller-Rabin test built on Montgomery multiplication.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// 1/p in double precision: the hardware reciprocal refined by two Newton steps
// (each squares the relative error), so the quotient estimates below are off
// by at most one.
__device__ __forceinline__ double gb_recip(uint32_t p)
{
    const double pd = (double)p;
    double r = __builtin_amdgcn_rcp(pd);
    double e = __builtin_fma(-pd, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-pd, r, 1.0);
    return __builtin_fma(r, e, r);
}

// Remainder of y by p when y < p * 2^32 (so y / p < 2^32): the double estimate
// of the quotient is within one of the truth and one signed step corrects it.
__device__ __forceinline__ uint32_t gb_mod_small_quot(uint64_t y, uint32_t p, double inv)
{
    const double yd = (double)y;
    const uint32_t q = __double2uint_rz(yd * inv);
    int64_t t = (int64_t)(y - (uint64_t)q * p);  // true value lies in (-p, 2p)
    if (t < 0)
        t += p;
    else if (t >= (int64_t)p)
        t -= p;
    return (uint32_t)t;
}

// x mod p for any 64-bit x and odd 3 <= p < 2^32, given inv = gb_recip(p).
// The high word is reduced first so that the second step's quotient fits 32
// bits.
__device__ __forceinline__ uint32_t gb_mod_u64_u32_inv(uint64_t x, uint32_t p, double inv)
{
    uint32_t xh = (uint32_t)(x >> 32);
    if (xh >= p)
        xh = gb_mod_small_quot(xh, p, inv);
    return gb_mod_small_quot(((uint64_t)xh << 32) | (uint32_t)x, p, inv);
}

__device__ __forceinline__ uint32_t gb_mod_u64_u32(uint64_t x, uint32_t p)
{
    return gb_mod_u64_u32_inv(x, p, gb_recip(p));
}

// Offset d in [0, p) of p's first odd multiple at or above the odd number
// Q = 2h + 1, i.e. p | Q + 2d, for odd 3 <= p < 2^32 and h < 2^63, in double
// precision and exactly.  Since 1/2 = (p + 1)/2 (mod p), d = (p - 1)/2 - h
// (mod p).  The caller passes h as hh = h rounded to double and hl = h - hh
// (|hl| <= 2^9, exact), and inv = gb_recip(p) (within an ulp of 1/p):
//  * q = floor(hh inv) is within h 2^-50 + 1 of h / p, and q p = ph + pl
//    exactly (the fma yields the product's rounding error);
//  * t = (p - 1)/2 - (h - q p) = (ph - hh) + (pl + ((p - 1)/2 - hl)): each
//    term and partial sum is an integer below 2^35 in magnitude (ph and hh lie
//    within (h 2^-50 + 2) p + 2^11 of each other), hence exact;
//  * f = floor(t inv) is floor(t / p) unless t is a multiple of p: |t| < 2^51
//    keeps the estimate's error below the 1/p that separates t / p from an
//    integer.  At a multiple, f may be one low; then d = t - f p (one exact
//    fma) comes out as p instead of 0, which the last step maps back.
// Contraction is off: a fused ph - hh would use the unrounded product and
// count its rounding error twice.
__device__ __forceinline__ uint32_t gb_first_odd_multiple(double hh, double hl, double pd,
                                                          double inv, double half)
{
#pragma clang fp contract(off)
    const double q = __builtin_floor(hh * inv);
    const double ph = q * pd;
    const double pl = __builtin_fma(q, pd, -ph);
    const double t = (ph - hh) + (pl + (half - hl));
    const double f = __builtin_floor(t * inv);
    const uint32_t d = (uint32_t)__builtin_fma(-f, pd, t);
    return d == (uint32_t)pd ? 0u : d;
}

// floor(sqrt(x)) exactly: a double estimate corrected with integer squares
// that cannot wrap (the root is at most 2^32 - 1).
__device__ __forceinline__ uint32_t gb_isqrt64(uint64_t x)
{
    uint64_t r = (uint64_t)__builtin_sqrt((double)x);
    if (r > 0xFFFFFFFFull)
        r = 0xFFFFFFFFull;
    while (r * r > x)
        --r;
    while (r < 0xFFFFFFFFull && (r + 1) * (r + 1) <= x)
        ++r;
    return (uint32_t)r;
}

// Montgomery product a*b*2^-64 mod n for odd n and a, b < n; ninv = -n^-1 mod 2^64.
// The 128-bit intermediate a*b + m*n is kept as (hi, lo) halves; its true
// value divided by 2^64 is below 2n and may exceed 2^64 when n > 2^63, which
// the carry flags track.
__device__ __forceinline__ uint64_t gb_mont_mul(uint64_t a, uint64_t b, uint64_t n, uint64_t ninv)
{
    const uint64_t lo = a * b;
    const uint64_t hi = __umul64hi(a, b);
    const uint64_t m = lo * ninv;
    const uint64_t mh = __umul64hi(m, n);
    const uint64_t s = hi + mh;
    const bool c1 = s < hi;
    const uint64_t s2 = s + (lo != 0 ? 1u : 0u);
    const bool c2 = s2 < s;
    return (c1 || c2 || s2 >= n) ? s2 - n : s2;
}

// Deterministic Miller-Rabin for 64-bit n with the first twelve primes as
// bases (the witness set the paper relies on for q < 2^64, Sec. 3.4).
__device__ inline bool gb_is_prime_u64(uint64_t n)
{
    if (n < 2)
        return false;
    if ((n & 1) == 0)
        return n == 2;
    const uint32_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        if (n == bases[i])
            return true;
        if (n % bases[i] == 0)
            return false;
    }
    if (n < 41ull * 41ull)
        return true;  // no prime factor <= 37 and below 41^2

    uint64_t inv = n;  // n * n == 1 (mod 8): three correct bits
#pragma unroll
    for (int i = 0; i < 5; ++i)
        inv *= 2 - n * inv;  // Newton: correct bits double each step
    const uint64_t ninv = 0 - inv;
    const uint64_t one = (0 - n) % n;  // 2^64 mod n: Montgomery form of 1
    uint64_t r2 = one;                 // becomes 2^128 mod n by 64 modular doublings
    for (int i = 0; i < 64; ++i) {
        const bool c = (r2 >> 63) != 0;
        uint64_t t = r2 << 1;
        if (c || t >= n)
            t -= n;
        r2 = t;
    }
    const uint64_t minus_one = n - one;
    uint64_t d = n - 1;
    const int s = __builtin_ctzll(d);
    d >>= s;
    for (int i = 0; i < 12; ++i) {
        uint64_t base = gb_mont_mul(bases[i], r2, n, ninv);  // bases[i] * 2^64 mod n
        uint64_t x = one;
        for (uint64_t e = d; e; e >>= 1) {
            if (e & 1)
                x = gb_mont_mul(x, base, n, ninv);
            base = gb_mont_mul(base, base, n, ninv);
        }
        if (x == one || x == minus_one)
            continue;
        bool witness = true;
        for (int j = 1; j < s; ++j) {
            x = gb_mont_mul(x, x, n, ninv);
            if (x == minus_one) {
                witness = false;
                break;
            }
        }
        if (witness)
            return false;
    }
    return true;
}
