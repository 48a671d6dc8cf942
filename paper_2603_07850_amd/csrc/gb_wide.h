// gb_wide.h -- the primality arithmetic of the kernels that verify past 2^64
// (Sec. 5, future work: 128-bit sieve arithmetic with a Baillie-PSW test):
// remainders of u128 values (gb_wide_u128.h) by 32-bit primes, Jacobi
// symbols, and the Baillie-PSW probable-prime test (strong test to base 2,
// then the strong Lucas test with Selfridge's parameters D = 5, -7, 9, ...;
// P = 1, Q = (1 - D)/4, evaluated on the V sequence alone) over the Montgomery
// arithmetic of gb_wide_limbs.h (R = 2^(28 N)).
#pragma once

#include "gb_arith.h"
#include "gb_internal.h"
#include "gb_wide_types.h"
#include "gb_wide_u128.h"
#include "gb_wide_limbs.h"

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
// N limbs for q below 2^(28 N - 12), qi = wl_qinv(q.lo) and one = 2^(28 N) mod q
// = w_r_mod(q, 28 N).  First the strong probable-prime test to base 2:
template <int N>
__device__ inline bool w_sprp2(u128w q, uint32_t qi, u128w one_u)
{
    const wl<N> q5 = wl_from<N>(q.lo, q.hi);
    const wl<N> one = wl_from<N>(one_u.lo, one_u.hi);
    const wl<N> minus_one = wl_sub(q5, one);
    // q - 1 = d * 2^s
    u128w d = w_sub64(q, 1);
    int s = 0;
    while ((d.lo & 1) == 0) {
        d.lo = (d.lo >> 1) | (d.hi << 63);
        d.hi >>= 1;
        ++s;
    }
    const int top = d.hi ? 127 - __builtin_clzll(d.hi) : 63 - __builtin_clzll(d.lo);
    wl<N> x = one;
    for (int i = top; i >= 0; --i) {
        x = wl_mont(x, x, q5, qi);                 // below 1.02 q
        const uint64_t w = i >= 64 ? d.hi : d.lo;
        if ((w >> (i & 63)) & 1)
            x = wl_add(x, x);                      // times the base 2: below 2.04 q
    }
    x = wl_canon<N, 2>(x, q5);
    bool pass = wl_eq(x, one) || wl_eq(x, minus_one);
    for (int r = 1; r < s && !pass; ++r) {
        x = wl_canon<N, 1>(wl_mont(x, x, q5, qi), q5);
        pass = wl_eq(x, minus_one);
    }
    return pass;
}

// then the strong Lucas test with Selfridge's parameters.
template <int N>
__device__ inline bool w_slucas(u128w q, uint32_t qi, u128w one_u)
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
    // 0 < |Q| <= 2^14 + 1 (|D| < 2^16 + 5 by the bound on the search): the
    // Montgomery forms of Q and of V_2 = P^2 - 2Q come from a small-constant
    // product and a negation
    const double qr = w_recip_d(q);
    u128w Qm_u = w_mul_small(one_u, (uint32_t)(Qs < 0 ? -Qs : Qs), q, qr);
    if (Qs < 0 && !w_zero(Qm_u))
        Qm_u = w_sub(q, Qm_u);
    const u128w V2_u = w_submod(one_u, w_addmod(Qm_u, Qm_u, q), q);
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
    // step is the same three Montgomery products and one product by the small
    // integer Q (Q^k+1 = Q Q^k, at most 3q) whatever the bit (no divergence);
    // the subtractions are additions of 2q - Q^k and 2 (3q - Q^(k+bit)), so
    // V_k and V_k+1 stay below 7.02 q unreduced.
    const wl<N> q5 = wl_from<N>(q.lo, q.hi);
    const wl<N> twoq = wl_norm(wl_add(q5, q5));
    const wl<N> threeq = wl_norm(wl_add(twoq, q5));
    const wl<N> Qm = wl_from<N>(Qm_u.lo, Qm_u.hi);
    const int top = d.hi ? 127 - __builtin_clzll(d.hi) : 63 - __builtin_clzll(d.lo);
    wl<N> V = wl_from<N>(one_u.lo, one_u.hi);   // V_1 = P = 1
    wl<N> V1 = wl_from<N>(V2_u.lo, V2_u.hi);    // V_2
    wl<N> Qk = Qm;                              // Q^1
    for (int i = top - 1; i >= 0; --i) {
        const uint64_t w = i >= 64 ? d.hi : d.lo;
        const bool bit = ((w >> (i & 63)) & 1) != 0;
        const wl<N> QkQ = wl_mul_q(Qk, Qs, q5, qr);
        const wl<N> Qb = bit ? QkQ : Qk;        // Q^(k + bit), at most 3q
        const wl<N> x = bit ? V1 : V;
        const wl<N> prod = wl_add(wl_mont(V, V1, q5, qi), wl_sub(twoq, Qk));
        const wl<N> nb = wl_sub(threeq, Qb);
        const wl<N> sq = wl_add(wl_mont(x, x, q5, qi), wl_add(nb, nb));
        V = bit ? prod : sq;
        V1 = bit ? sq : prod;
        Qk = wl_mont(Qk, Qb, q5, qi);           // Q^(2k + bit)
    }
    V = wl_canon<N, 7>(V, q5);
    V1 = wl_canon<N, 7>(V1, q5);
    if (wl_eq(wl_canon<N, 1>(wl_add(V1, V1), q5), V) || wl_zero(V))
        return true;   // U_d = 0 or V_d = 0
    for (int r = 1; r < s; ++r) {
        const wl<N> nq = wl_sub(twoq, Qk);
        V = wl_canon<N, 5>(wl_add(wl_mont(V, V, q5, qi), wl_add(nq, nq)), q5);
        Qk = wl_mont(Qk, Qk, q5, qi);
        if (wl_zero(V))
            return true;
    }
    return false;
}

// Baillie-PSW: both halves, over the fewest limbs for q.
template <int N>
__device__ inline bool w_bpsw_n(u128w q)
{
    const uint32_t qi = wl_qinv(q.lo);
    const u128w one = w_r_mod(q, 28 * N);   // Montgomery form of 1
    return w_sprp2<N>(q, qi, one) && w_slucas<N>(q, qi, one);
}

__device__ inline bool w_bpsw(u128w q)
{
    const int L = q.hi ? 128 - __builtin_clzll(q.hi) : 64 - __builtin_clzll(q.lo);
    const int n = wl_limbs_for(L);
    return n == 3 ? w_bpsw_n<3>(q) : (n == 4 ? w_bpsw_n<4>(q) : w_bpsw_n<5>(q));
}
