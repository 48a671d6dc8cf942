/*
 * gb_oracle_wide.c -- plain, slow CPU oracle for Goldbach range verification
 * past 2^64 (the paper's future-work direction "pushing past the 64-bit
 * ceiling", Sec. 5: 128-bit arithmetic coupled with a Baillie-PSW test).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header, table or constant with the GPU
 * path.
 *
 * Beyond 2^64 no table of primes up to sqrt(q) exists, so primality of
 * q = n - p is decided by the Baillie-PSW test: a strong probable-prime test
 * to base 2 followed by a strong Lucas probable-prime test with Selfridge's
 * parameters (D the first of 5, -7, 9, -11, ... with Jacobi symbol
 * (D/q) = -1, P = 1, Q = (1 - D)/4).  No composite passing both is known, and
 * none exists below 2^64.  What this file computes, for every even n of an
 * inclusive u128 range [A, B]:
 *     p_min(n) = min { p prime : p <= n - 2, BPSW(n - p) },
 * searched first among the candidate primes p <= P_max (Phase 1), then among
 * the table primes P_max < p <= min(T, n/2) (Phase 2), with the same
 * aggregates as the 64-bit oracle: count verified, sum of p_min mod 2^64,
 * largest p_min with its smallest n, the Phase-1 misses in ascending order,
 * and the count of n with no p found.
 *
 * Method, with no blocking or reordering beyond the definition: for each n in
 * ascending order, each candidate p in ascending order, q = n - p is tested
 * by BPSW (a q with a prime factor below 1000 other than itself is rejected
 * first by trial division, which only saves time).  All arithmetic is on
 * unsigned __int128; modular products use double-and-add, so nothing
 * overflows for any modulus below 2^128.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define GBO_OK 0
#define GBO_EINVAL 1
#define GBO_ETRUNC 5

typedef struct gbo_result_wide {
    uint64_t A_lo, A_hi, B_lo, B_hi;   /* normalized bounds; A > B: empty */
    uint64_t P_max;
    uint64_t verified;
    uint64_t max_p;
    uint64_t max_p_n_lo, max_p_n_hi;
    uint64_t checksum;
    uint64_t n_unresolved;
    uint64_t n_failed;
} gbo_result_wide;

static u128 mk(uint64_t lo, uint64_t hi) { return ((u128)hi << 64) | lo; }

/* (a + b) mod m for a, b < m, without overflow */
static u128 addmod(u128 a, u128 b, u128 m)
{
    return a >= m - b ? a - (m - b) : a + b;
}

static u128 submod(u128 a, u128 b, u128 m)
{
    return a >= b ? a - b : a + (m - b);
}

/* a * b mod m by double-and-add over the bits of b (a, b < m) */
static u128 mulmod(u128 a, u128 b, u128 m)
{
    u128 r = 0;
    for (int i = 127; i >= 0; i--) {
        r = addmod(r, r, m);
        if ((b >> i) & 1)
            r = addmod(r, a, m);
    }
    return r;
}

static u128 powmod(u128 a, u128 e, u128 m)
{
    u128 r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1)
            r = mulmod(r, a, m);
        a = mulmod(a, a, m);
        e >>= 1;
    }
    return r;
}

/* floor(sqrt(x)) by bisection on r * r <= x (r < 2^64, so r * r fits) */
uint64_t gbo_isqrt128(uint64_t lo, uint64_t hi)
{
    u128 x = mk(lo, hi);
    uint64_t a = 0, b = UINT64_MAX;
    while (a < b) {
        uint64_t mid = a + (b - a) / 2 + 1;
        if ((u128)mid * mid <= x)
            a = mid;
        else
            b = mid - 1;
    }
    return a;
}

/* strong probable prime to base a (n odd, n > a) */
static int sprp(u128 n, u128 a)
{
    u128 d = n - 1;
    int s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        s++;
    }
    u128 x = powmod(a, d, n);
    if (x == 1 || x == n - 1)
        return 1;
    for (int r = 1; r < s; r++) {
        x = mulmod(x, x, n);
        if (x == n - 1)
            return 1;
    }
    return 0;
}

/* Jacobi symbol (a/n) for odd n > 0, with a given as a residue mod n */
static int jacobi(u128 a, u128 n)
{
    int t = 1;
    a %= n;
    while (a != 0) {
        while ((a & 1) == 0) {
            a >>= 1;
            unsigned r = (unsigned)(n & 7);
            if (r == 3 || r == 5)
                t = -t;
        }
        u128 tmp = a;
        a = n;
        n = tmp;
        if ((a & 3) == 3 && (n & 3) == 3)
            t = -t;
        a %= n;
    }
    return n == 1 ? t : 0;
}

/* x / 2 mod n for odd n */
static u128 half(u128 x, u128 n)
{
    return (x & 1) ? (x >> 1) + (n >> 1) + 1 : x >> 1;
}

/*
 * Strong Lucas probable prime with Selfridge's method A: D = 5, -7, 9, -11,
 * ... until (D/n) = -1; P = 1, Q = (1 - D)/4.  With n + 1 = d * 2^s, d odd,
 * n passes when U_d = 0 or V_{d 2^r} = 0 (mod n) for some 0 <= r < s.
 * n is odd, > 5 here, and not a perfect square.
 */
static int strong_lucas(u128 n)
{
    int64_t D = 5;
    for (;;) {
        u128 Dm = D > 0 ? (u128)D % n : n - ((u128)(-D) % n);
        int j = jacobi(Dm, n);
        if (j == -1)
            break;
        if (j == 0 && (u128)(D > 0 ? D : -D) != n)
            return 0;   /* a factor of n */
        D = D > 0 ? -(D + 2) : -D + 2;
    }
    const int64_t Qs = (1 - D) / 4;
    const u128 Dm = D > 0 ? (u128)D % n : n - ((u128)(-D) % n);
    const u128 Qm = Qs >= 0 ? (u128)Qs % n : n - ((u128)(-Qs) % n);
    u128 d = n + 1;   /* n < 2^128 - 1 here */
    int s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        s++;
    }
    /* U_1 = 1, V_1 = P = 1, Q^1; then the binary chain over the bits of d */
    int top = 127;
    while (!((d >> top) & 1))
        top--;
    u128 U = 1, V = 1, Qk = Qm;
    for (int i = top - 1; i >= 0; i--) {
        /* k -> 2k */
        U = mulmod(U, V, n);
        V = submod(mulmod(V, V, n), addmod(Qk, Qk, n), n);
        Qk = mulmod(Qk, Qk, n);
        if ((d >> i) & 1) {
            /* 2k -> 2k + 1 (P = 1) */
            u128 U2 = half(addmod(U, V, n), n);
            u128 V2 = half(addmod(mulmod(Dm, U, n), V, n), n);
            U = U2;
            V = V2;
            Qk = mulmod(Qk, Qm, n);
        }
    }
    if (U == 0 || V == 0)
        return 1;
    for (int r = 1; r < s; r++) {
        V = submod(mulmod(V, V, n), addmod(Qk, Qk, n), n);
        Qk = mulmod(Qk, Qk, n);
        if (V == 0)
            return 1;
    }
    return 0;
}

static const uint32_t kSmall[] = {2,  3,  5,  7,  11, 13, 17, 19, 23, 29, 31, 37, 41, 43,
                                  47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97};

/* Baillie-PSW: 1 for a probable prime, 0 for composite (n < 2^128 - 1). */
static int bpsw(u128 n)
{
    if (n < 2)
        return 0;
    for (unsigned i = 0; i < sizeof kSmall / sizeof kSmall[0]; i++) {
        if (n == kSmall[i])
            return 1;
        if (n % kSmall[i] == 0)
            return 0;
    }
    if (!sprp(n, 2))
        return 0;
    uint64_t r = gbo_isqrt128((uint64_t)n, (uint64_t)(n >> 64));
    if ((u128)r * r == n)
        return 0;
    return strong_lucas(n);
}

int gbo_bpsw(uint64_t lo, uint64_t hi) { return bpsw(mk(lo, hi)); }

/* q has a prime factor below 1000 other than q itself (a cheap composite test) */
static int small_factor(u128 q, const uint32_t *primes, uint64_t nprimes)
{
    for (uint64_t k = 0; k < nprimes && primes[k] < 1000; k++)
        if (q != primes[k] && q % primes[k] == 0)
            return 1;
    return 0;
}

static void account(gbo_result_wide *res, u128 n, uint64_t p)
{
    res->verified++;
    res->checksum += p;
    u128 bn = mk(res->max_p_n_lo, res->max_p_n_hi);
    if (p > res->max_p || (p == res->max_p && n < bn)) {
        res->max_p = p;
        res->max_p_n_lo = (uint64_t)n;
        res->max_p_n_hi = (uint64_t)(n >> 64);
    }
}

/*
 * Verify every even n in [A, B] (u128 bounds as lo/hi halves; inclusive,
 * rounded inward to even numbers, A raised to 4).
 *   primes/nprimes/T : every prime <= T ascending; candidates are the primes
 *                      <= P_max, Phase 2 uses the table primes above it
 *   unresolved       : 2 * cap u64 (lo, hi pairs), ascending Phase-1 misses
 *   pmin_out         : optional p_min per even in order (0 where none);
 *                      only for short ranges
 */
int gbo_verify_range_wide(uint64_t A_lo, uint64_t A_hi, uint64_t B_lo, uint64_t B_hi,
                          uint64_t P_max, const uint32_t *primes, uint64_t nprimes, uint64_t T,
                          gbo_result_wide *res, uint64_t *unresolved, uint64_t cap,
                          uint32_t *pmin_out)
{
    memset(res, 0, sizeof(*res));
    res->P_max = P_max;
    if (P_max < 2 || P_max > T || nprimes == 0)
        return GBO_EINVAL;
    u128 A = mk(A_lo, A_hi), B = mk(B_lo, B_hi);
    const u128 top = ~(u128)0;
    if (A & 1) {
        if (A == top) {
            res->A_lo = res->A_hi = UINT64_MAX;
            res->B_lo = (uint64_t)(B & ~(u128)1);
            res->B_hi = (uint64_t)((B & ~(u128)1) >> 64);
            return GBO_OK;
        }
        A += 1;
    }
    if (A < 4)
        A = 4;
    B &= ~(u128)1;
    res->A_lo = (uint64_t)A;
    res->A_hi = (uint64_t)(A >> 64);
    res->B_lo = (uint64_t)B;
    res->B_hi = (uint64_t)(B >> 64);
    if (A > B)
        return GBO_OK;
    uint64_t ncand = 0;
    while (ncand < nprimes && primes[ncand] <= P_max)
        ncand++;
    int status = GBO_OK;
    u128 count = (B - A) / 2 + 1;
    for (u128 i = 0; i < count; i++) {
        u128 n = A + 2 * i;
        uint64_t found = 0;
        if (n == 4) {
            found = 2;
        } else {
            for (uint64_t k = 1; k < ncand; k++) {
                uint64_t p = primes[k];
                if ((u128)p > n - 3)
                    break;
                u128 q = n - p;
                if (!small_factor(q, primes, nprimes) && bpsw(q)) {
                    found = p;
                    break;
                }
            }
        }
        if (!found) {
            if (res->n_unresolved < cap && unresolved) {
                unresolved[2 * res->n_unresolved] = (uint64_t)n;
                unresolved[2 * res->n_unresolved + 1] = (uint64_t)(n >> 64);
            } else {
                status = GBO_ETRUNC;
            }
            res->n_unresolved++;
            for (uint64_t k = ncand; k < nprimes; k++) {
                uint64_t p = primes[k];
                if ((u128)p > n / 2)
                    break;
                u128 q = n - p;
                if (!small_factor(q, primes, nprimes) && bpsw(q)) {
                    found = p;
                    break;
                }
            }
        }
        if (found)
            account(res, n, found);
        else
            res->n_failed++;
        if (pmin_out)
            pmin_out[(uint64_t)i] = (uint32_t)found;
    }
    (void)T;
    return status;
}
