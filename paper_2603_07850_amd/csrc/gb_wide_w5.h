// gb_wide_w5.h -- Montgomery arithmetic modulo an odd q < 2^128 over five
// 28-bit limbs (R = 2^140), the inner arithmetic of the Baillie-PSW test past
// 2^64.
//
// With 28-bit limbs every 32x32-bit limb product fits 60 bits, so a column of
// the product accumulates in one 64-bit register by 32x32+64-bit multiply-adds
// alone: no carry is propagated inside a product, and no register pair has to
// be rebuilt for an addend.  Values are kept lazily: a Montgomery product takes
// operands with limbs below 2^30 and values below 8q, and returns normalized
// limbs (the low four below 2^28) with a value below a*b/2^140 + q < 1.01 q;
// sums of such values stay within the operand bounds, and subtractions are
// written as additions of an exact 2q - y.  Only comparisons reduce fully.
//
// Plain integer code: the functions are device functions in the kernels and
// compile for the host (GB_W5_FN defined before inclusion) in the tests.
#pragma once

#include <stdint.h>

#ifndef GB_W5_FN
#define GB_W5_FN __device__ __forceinline__
#endif

struct w5 {
    uint32_t l[5];   // value = sum of l[j] * 2^(28 j)
};

constexpr uint32_t kW5Mask = (1u << 28) - 1;

// Limbs of lo + 2^64 hi (normalized).
GB_W5_FN w5 w5_from(uint64_t lo, uint64_t hi)
{
    w5 r;
    r.l[0] = (uint32_t)lo & kW5Mask;
    r.l[1] = (uint32_t)(lo >> 28) & kW5Mask;
    r.l[2] = (uint32_t)((lo >> 56) | (hi << 8)) & kW5Mask;
    r.l[3] = (uint32_t)(hi >> 20) & kW5Mask;
    r.l[4] = (uint32_t)(hi >> 48);
    return r;
}

// -q^-1 mod 2^28 for odd q (Newton steps on the low 32 bits double the
// correct low bits: 3, 6, 12, 24, 48).
GB_W5_FN uint32_t w5_qinv(uint64_t q_lo)
{
    const uint32_t q0 = (uint32_t)q_lo;
    uint32_t inv = q0;
    for (int i = 0; i < 4; ++i)
        inv *= 2u - q0 * inv;
    return (0u - inv) & kW5Mask;
}

// Montgomery product a * b * 2^-140 mod q (see the bounds above); qi = w5_qinv.
GB_W5_FN w5 w5_mont(const w5 &a, const w5 &b, const w5 &q, uint32_t qi)
{
    // c[j]: column i + j of the running value in row i (below 2^63: at most
    // five products below 2^60 and five below 2^56 each, plus carries)
    uint64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const uint64_t bi = b.l[i];
        c0 += a.l[0] * bi;
        c1 += a.l[1] * bi;
        c2 += a.l[2] * bi;
        c3 += a.l[3] * bi;
        c4 += a.l[4] * bi;
        const uint64_t m = ((uint32_t)c0 * qi) & kW5Mask;   // the low limb becomes zero
        c0 += m * q.l[0];
        c1 += m * q.l[1];
        c2 += m * q.l[2];
        c3 += m * q.l[3];
        c4 += m * q.l[4];
        c0 = c1 + (c0 >> 28);
        c1 = c2;
        c2 = c3;
        c3 = c4;
        c4 = 0;
    }
    w5 r;
    r.l[0] = (uint32_t)c0 & kW5Mask;
    c1 += c0 >> 28;
    r.l[1] = (uint32_t)c1 & kW5Mask;
    c2 += c1 >> 28;
    r.l[2] = (uint32_t)c2 & kW5Mask;
    c3 += c2 >> 28;
    r.l[3] = (uint32_t)c3 & kW5Mask;
    r.l[4] = (uint32_t)(c3 >> 28);
    return r;
}

// x + y limb by limb (no carries: the caller keeps the operand bounds).
GB_W5_FN w5 w5_add(const w5 &x, const w5 &y)
{
    w5 r;
#pragma unroll
    for (int j = 0; j < 5; ++j)
        r.l[j] = x.l[j] + y.l[j];
    return r;
}

// z - y for normalized z >= y (values), normalized result.
GB_W5_FN w5 w5_sub(const w5 &z, const w5 &y)
{
    w5 r;
    uint32_t b = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t t = z.l[j] - y.l[j] - b;   // in (-2^28 - 1, 2^28)
        r.l[j] = t & kW5Mask;
        b = t >> 31;
    }
    r.l[4] = z.l[4] - y.l[4] - b;
    return r;
}

// Carries propagated: the low four limbs below 2^28.
GB_W5_FN w5 w5_norm(const w5 &x)
{
    w5 r;
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t t = x.l[j] + c;
        r.l[j] = t & kW5Mask;
        c = t >> 28;
    }
    r.l[4] = x.l[4] + c;
    return r;
}

// x - q if x >= q, else x (x normalized, value below 2^131).
GB_W5_FN w5 w5_csub(const w5 &x, const w5 &q)
{
    w5 d;
    uint32_t b = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t t = x.l[j] - q.l[j] - b;
        d.l[j] = t & kW5Mask;
        b = t >> 31;
    }
    const uint32_t t = x.l[4] - q.l[4] - b;
    d.l[4] = t;
    return (t >> 31) ? x : d;
}

// The residue of x in [0, q) for x (any limbs below 2^30) below (k + 1) q.
template <int k>
GB_W5_FN w5 w5_canon(const w5 &x, const w5 &q)
{
    w5 r = w5_norm(x);
#pragma unroll
    for (int i = 0; i < k; ++i)
        r = w5_csub(r, q);
    return r;
}

GB_W5_FN bool w5_eq(const w5 &x, const w5 &y)
{
    return ((x.l[0] ^ y.l[0]) | (x.l[1] ^ y.l[1]) | (x.l[2] ^ y.l[2]) | (x.l[3] ^ y.l[3]) |
            (x.l[4] ^ y.l[4])) == 0;
}

GB_W5_FN bool w5_zero(const w5 &x)
{
    return (x.l[0] | x.l[1] | x.l[2] | x.l[3] | x.l[4]) == 0;
}
