// gb_wide.h -- 128-bit integer arithmetic of the kernels that verify past
// 2^64 (Sec. 5, future work: 128-bit sieve arithmetic with a Baillie-PSW
// test): u128 values as two 64-bit words, remainders by 32-bit primes,
// Montgomery multiplication modulo an odd 128-bit q (R = 2^128) and the
// Baillie-PSW probable-prime test (strong test to base 2, then the strong
// Lucas test with Selfridge's parameters D = 5, -7, 9, ...; P = 1,
// Q = (1 - D)/4, evaluated on the V sequence alone).
#pragma once

#include "gb_arith.h"
#include "gb_internal.h"
#include "gb_wide_types.h"

__device__ __forceinline__ bool w_lt(u128w a, u128w b)
{
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}
__device__ __forceinline__ bool w_eq(u128w a, u128w b) { return a.hi == b.hi && a.lo == b.lo; }
__device__ __forceinline__ bool w_zero(u128w a) { return (a.hi | a.lo) == 0; }

__device__ __forceinline__ u128w w_add64(u128w a, uint64_t b)
{
    u128w r;
    r.lo = a.lo + b;
    r.hi = a.hi + (r.lo < b ? 1u : 0u);
    return r;
}

__device__ __forceinline__ u128w w_sub64(u128w a, uint64_t b)
{
    u128w r;
    r.lo = a.lo - b;
    r.hi = a.hi - (a.lo < b ? 1u : 0u);
    return r;
}

__device__ __forceinline__ u128w w_sub(u128w a, u128w b)
{
    u128w r;
    r.lo = a.lo - b.lo;
    r.hi = a.hi - b.hi - (a.lo < b.lo ? 1u : 0u);
    return r;
}

// a mod p for an odd prime 3 <= p < 2^32: (hi mod p) * (2^64 mod p) + lo mod p.
__device__ __forceinline__ uint32_t w_mod_u32(u128w a, uint32_t p)
{
    const double inv = gb_recip(p);
    const uint32_t r32 = gb_mod_u64_u32_inv(1ull << 32, p, inv);           // 2^32 mod p
    const uint32_t r64 = gb_mod_u64_u32_inv((uint64_t)r32 * r32, p, inv);  // 2^64 mod p
    const uint32_t h = gb_mod_u64_u32_inv(a.hi, p, inv);
    const uint32_t l = gb_mod_u64_u32_inv(a.lo, p, inv);
    const uint32_t t = gb_mod_u64_u32_inv((uint64_t)h * r64, p, inv);
    const uint64_t s = (uint64_t)t + l;   // < 2p
    return (uint32_t)(s >= p ? s - p : s);
}

// (a + b) mod q and (a - b) mod q for a, b < q.
__device__ __forceinline__ u128w w_addmod(u128w a, u128w b, u128w q)
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

__device__ __forceinline__ u128w w_submod(u128w a, u128w b, u128w q)
{
    const u128w d = w_sub(a, b);
    if (!w_lt(a, b))
        return d;
    u128w r;
    r.lo = d.lo + q.lo;
    r.hi = d.hi + q.hi + (r.lo < q.lo ? 1u : 0u);
    return r;
}

// Montgomery product a * b * 2^-128 mod q for odd q and a, b < q: word-serial
// reduction over four 32-bit limbs (each limb product with its addends fits
// one 32x32+64-bit multiply-add, which issues at the full VALU rate);
// qinv = -q^-1 mod 2^64, of which the low 32 bits serve.  The running value
// stays below 2q, so a fifth limb holds its top bit.
__device__ __forceinline__ u128w w_mont_mul(u128w A, u128w B, u128w Q, uint64_t qinv)
{
    const uint32_t a[4] = {(uint32_t)A.lo, (uint32_t)(A.lo >> 32), (uint32_t)A.hi,
                           (uint32_t)(A.hi >> 32)};
    const uint32_t b[4] = {(uint32_t)B.lo, (uint32_t)(B.lo >> 32), (uint32_t)B.hi,
                           (uint32_t)(B.hi >> 32)};
    const uint32_t q[4] = {(uint32_t)Q.lo, (uint32_t)(Q.lo >> 32), (uint32_t)Q.hi,
                           (uint32_t)(Q.hi >> 32)};
    const uint32_t qi = (uint32_t)qinv;
    uint32_t t0 = 0, t1 = 0, t2 = 0, t3 = 0, t4 = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        // t += a * b[i] (six limbs)
        uint64_t uv = (uint64_t)a[0] * b[i] + t0;
        t0 = (uint32_t)uv;
        uv = (uint64_t)a[1] * b[i] + t1 + (uv >> 32);
        t1 = (uint32_t)uv;
        uv = (uint64_t)a[2] * b[i] + t2 + (uv >> 32);
        t2 = (uint32_t)uv;
        uv = (uint64_t)a[3] * b[i] + t3 + (uv >> 32);
        t3 = (uint32_t)uv;
        uv = (uint64_t)t4 + (uv >> 32);
        t4 = (uint32_t)uv;
        const uint32_t t5 = (uint32_t)(uv >> 32);
        // t = (t + m q) / 2^32 with m making the low limb zero
        const uint32_t m = t0 * qi;
        uv = (uint64_t)m * q[0] + t0;
        uv = (uint64_t)m * q[1] + t1 + (uv >> 32);
        t0 = (uint32_t)uv;
        uv = (uint64_t)m * q[2] + t2 + (uv >> 32);
        t1 = (uint32_t)uv;
        uv = (uint64_t)m * q[3] + t3 + (uv >> 32);
        t2 = (uint32_t)uv;
        uv = (uint64_t)t4 + (uv >> 32);
        t3 = (uint32_t)uv;
        t4 = t5 + (uint32_t)(uv >> 32);
    }
    u128w r = {((uint64_t)t1 << 32) | t0, ((uint64_t)t3 << 32) | t2};
    if (t4 != 0 || !w_lt(r, Q))
        r = w_sub(r, Q);
    return r;
}

// -q^-1 mod 2^64 for odd q (Newton steps double the correct low bits).
__device__ __forceinline__ uint64_t w_qinv(uint64_t q0)
{
    uint64_t inv = q0;   // q0 * q0 == 1 (mod 8)
#pragma unroll
    for (int i = 0; i < 5; ++i)
        inv *= 2 - q0 * inv;
    return 0 - inv;
}

// 2^128 mod q for odd q > 1: from 2^(L-1) < q (L the bit length of q), by
// 129 - L modular doublings.
__device__ __forceinline__ u128w w_r_mod(u128w q)
{
    const int L = q.hi ? 128 - __builtin_clzll(q.hi) : 64 - __builtin_clzll(q.lo);
    u128w x = L > 64 ? u128w{0, 1ull << (L - 65)} : u128w{1ull << (L - 1), 0};
    for (int i = L - 1; i < 128; ++i)
        x = w_addmod(x, x, q);
    return x;
}

// v * x mod q for a small v < 2^20 and x < q (double and add).
__device__ __forceinline__ u128w w_small_mul(uint32_t v, u128w x, u128w q)
{
    u128w r = {0, 0};
    for (int i = 19; i >= 0; --i) {
        r = w_addmod(r, r, q);
        if ((v >> i) & 1)
            r = w_addmod(r, x, q);
    }
    return r;
}

// Jacobi symbol (a / m) for odd 0 < m and 0 <= a < m, 32-bit.
__device__ __forceinline__ int jacobi32(uint32_t a, uint32_t m)
{
    int t = 1;
    while (a != 0) {
        while ((a & 1) == 0) {
            a >>= 1;
            const uint32_t r = m & 7;
            if (r == 3 || r == 5)
                t = -t;
        }
        const uint32_t tmp = a;
        a = m;
        m = tmp;
        if ((a & 3) == 3 && (m & 3) == 3)
            t = -t;
        a %= m;
    }
    return m == 1 ? t : 0;
}

// Jacobi symbol (D / q) for odd D = +-d (d odd, small) and odd q > d, by
// reciprocity: (d / q) = (q mod d / d) * (-1)^((d-1)/2 * (q-1)/2), and
// (-1 / q) = (-1)^((q-1)/2).
__device__ __forceinline__ int w_jacobi_small(int32_t D, u128w q)
{
    const uint32_t d = (uint32_t)(D < 0 ? -D : D);
    int t = 1;
    const bool q3 = (q.lo & 3) == 3;
    if (D < 0 && q3)
        t = -t;
    if (d == 1)
        return t;
    if ((d & 3) == 3 && q3)
        t = -t;
    return t * jacobi32(w_mod_u32(q, d), d);
}

// floor(sqrt(q)) == r exactly, for the perfect-square check (rarely taken).
__device__ inline bool w_is_square(u128w q)
{
    // the double estimate of sqrt(q) is within ~2^10 of the truth below 2^128
    const double qd = (double)q.hi * 18446744073709551616.0 + (double)q.lo;
    const double rd = __builtin_sqrt(qd);
    uint64_t r = rd >= 18446744073709551615.0 ? ~0ull : (uint64_t)rd;
    uint64_t lo = r > 4096 ? r - 4096 : 0, hi = r + 4096 < r ? ~0ull : r + 4096;
    while (lo < hi) {   // largest x in [lo, hi] with x^2 <= q
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        const u128w sq = {mid * mid, __umul64hi(mid, mid)};
        if (!w_lt(q, sq))
            lo = mid;
        else
            hi = mid - 1;
    }
    const u128w sq = {lo * lo, __umul64hi(lo, lo)};
    return w_eq(sq, q);
}

// The two halves of the Baillie-PSW test of an odd q > 2^64 that has no prime
// factor up to 97 (the sieve has removed every factor up to its bound), with
// qinv = w_qinv(q.lo) and one = w_r_mod(q).  First the strong probable-prime
// test to base 2:
__device__ inline bool w_sprp2(u128w q, uint64_t qinv, u128w one)
{
    const u128w minus_one = w_sub(q, one);
    // strong probable prime to base 2: q - 1 = d * 2^s
    u128w d = w_sub64(q, 1);
    int s = 0;
    while ((d.lo & 1) == 0) {
        d.lo = (d.lo >> 1) | (d.hi << 63);
        d.hi >>= 1;
        ++s;
    }
    const int top = d.hi ? 127 - __builtin_clzll(d.hi) : 63 - __builtin_clzll(d.lo);
    u128w x = one;
    for (int i = top; i >= 0; --i) {
        x = w_mont_mul(x, x, q, qinv);
        const uint64_t w = i >= 64 ? d.hi : d.lo;
        if ((w >> (i & 63)) & 1)
            x = w_addmod(x, x, q);   // times the base 2
    }
    bool pass = w_eq(x, one) || w_eq(x, minus_one);
    for (int r = 1; r < s && !pass; ++r) {
        x = w_mont_mul(x, x, q, qinv);
        pass = w_eq(x, minus_one);
    }
    return pass;
}

// then the strong Lucas test with Selfridge's parameters.
__device__ inline bool w_slucas(u128w q, uint64_t qinv, u128w one)
{
    // Selfridge: the first D of 5, -7, 9, -11, ... with (D / q) = -1
    int32_t D = 5;
    int tries = 0;
    for (;;) {
        const int j = w_jacobi_small(D, q);
        if (j == -1)
            break;
        if (j == 0)
            return false;   // |D| shares a factor with q (q > |D|)
        if (++tries == 16 && w_is_square(q))
            return false;   // a square has no such D
        if (tries >= (1 << 15))
            return false;   // a bound on the loop only: for a non-square the
                            // first such D comes after a few tries

        D = D > 0 ? -(D + 2) : -D + 2;
    }
    const int32_t Qs = (1 - D) / 4;
    // Montgomery form of Q
    u128w Qm = w_small_mul((uint32_t)(Qs < 0 ? -Qs : Qs), one, q);
    if (Qs < 0 && !w_zero(Qm))
        Qm = w_sub(q, Qm);
    // q + 1 = d * 2^s (q + 1 cannot wrap: q < 2^128 - 1)
    u128w d = w_add64(q, 1);
    int s = 0;
    while ((d.lo & 1) == 0) {
        d.lo = (d.lo >> 1) | (d.hi << 63);
        d.hi >>= 1;
        ++s;
    }
    // The ladder keeps (V_k, V_k+1, Q^k) and doubles k, adding one where the
    // bit of d is set:
    //   V_2k = V_k^2 - 2 Q^k,  V_2k+1 = V_k V_k+1 - P Q^k,  V_2k+2 = V_k+1^2 - 2 Q^k+1.
    // U is not carried: D U_k = 2 V_k+1 - P V_k, and D is a unit mod q
    // ((D / q) = -1), so U_d = 0 (mod q) exactly when 2 V_d+1 = P V_d.  Every
    // step is the same four products whatever the bit (no divergence).
    const int top = d.hi ? 127 - __builtin_clzll(d.hi) : 63 - __builtin_clzll(d.lo);
    u128w V = one;                                      // V_1 = P = 1
    u128w V1 = w_submod(one, w_addmod(Qm, Qm, q), q);   // V_2 = P^2 - 2Q
    u128w Qk = Qm;                                      // Q^1
    for (int i = top - 1; i >= 0; --i) {
        const uint64_t w = i >= 64 ? d.hi : d.lo;
        const bool bit = ((w >> (i & 63)) & 1) != 0;
        const u128w QkQ = w_mont_mul(Qk, Qm, q, qinv);
        const u128w Qb = bit ? QkQ : Qk;                // Q^(k + bit)
        const u128w x = bit ? V1 : V;
        const u128w prod = w_submod(w_mont_mul(V, V1, q, qinv), Qk, q);
        const u128w sq = w_submod(w_mont_mul(x, x, q, qinv), w_addmod(Qb, Qb, q), q);
        V = bit ? prod : sq;
        V1 = bit ? sq : prod;
        Qk = w_mont_mul(Qk, Qb, q, qinv);               // Q^(2k + bit)
    }
    if (w_eq(w_addmod(V1, V1, q), V) || w_zero(V))
        return true;   // U_d = 0 or V_d = 0
    for (int r = 1; r < s; ++r) {
        V = w_submod(w_mont_mul(V, V, q, qinv), w_addmod(Qk, Qk, q), q);
        Qk = w_mont_mul(Qk, Qk, q, qinv);
        if (w_zero(V))
            return true;
    }
    return false;
}

// Baillie-PSW: both halves.
__device__ inline bool w_bpsw(u128w q)
{
    const uint64_t qinv = w_qinv(q.lo);
    const u128w one = w_r_mod(q);   // R mod q: Montgomery form of 1
    return w_sprp2(q, qinv, one) && w_slucas(q, qinv, one);
}
