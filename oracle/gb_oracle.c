/*
 * gb_oracle.c -- plain, slow, obviously-correct CPU oracle for Goldbach range
 * verification with a segmented double sieve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
 * its Python binding) may link, load or call this file; only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark do.  It shares no code,
 * header, table or constant with the GPU path.
 *
 * What it computes (paper, Sec. 1 problem statement and Sec. 3.3 / Sec. 3.1):
 * for every even n in [A, B] the minimal prime p such that n - p is prime,
 *     p_min(n) = min { p prime : n - p prime },
 * searched first among candidate primes p <= P_max ("Phase 1", Sec. 3.3), then,
 * for the n that Phase 1 leaves unresolved, among the remaining table primes
 * P_max < p <= min(T, n/2) with n - p tested for primality ("Phase 2",
 * Sec. 3.3).  Aggregates returned for the range:
 *   verified      number of n for which some p was found (either phase)
 *   checksum      sum of p_min over verified n, modulo 2^64
 *   max_p/max_p_n largest p_min, and the smallest n attaining it
 *   unresolved    ascending list of n with no prime p <= P_max (Phase 1 miss)
 *   n_failed      n with no p found even after Phase 2
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes): ranges are inclusive and rounded inward to even numbers, A is
 * clamped to 4; n = 4 is 2 + 2; for n >= 6 only odd p can work; the Phase-2
 * range is bounded by the prime table limit T and by n/2; max ties go to the
 * smallest n.
 *
 * Method, step by step, with no blocking or reordering beyond the plain
 * definition:
 *   1. base primes: plain sieve of Eratosthenes (gbo_primes);
 *   2. per oracle segment of evens, a byte array marks the odd q in the
 *      window [n_lo - P_max, n_hi - 3]; every base prime p with
 *      p <= q_hi / p (the division-bounded guard of Sec. 3.4) strikes its odd
 *      multiples from max(p*p, first multiple >= window low); loop variables
 *      are 128-bit so nothing wraps near 2^64;
 *   3. scalar probe: candidates ascending, stop at the first prime q;
 *   4. Phase 2: the next table primes ascending, q tested by gbo_is_prime
 *      (trial division below 2^32, deterministic Miller-Rabin with the first
 *      twelve primes as bases above it, Sec. 3.4).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define GBO_OK 0
#define GBO_EINVAL 1
#define GBO_ERANGE 2
#define GBO_ENOMEM 3
#define GBO_ETRUNC 5

typedef struct gbo_result {
    uint64_t A, B;          /* normalized bounds; A > B means the range is empty */
    uint64_t P_max;         /* candidate bound used */
    uint64_t verified;
    uint64_t max_p;
    uint64_t max_p_n;
    uint64_t checksum;
    uint64_t n_unresolved;
    uint64_t n_failed;
} gbo_result;

/* floor(sqrt(x)) by bisection on r*r <= x, in 128-bit so the square never wraps. */
uint64_t gbo_isqrt(uint64_t x)
{
    uint64_t lo = 0, hi = 0xFFFFFFFFull;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo + 1) / 2;
        if ((u128)mid * mid <= (u128)x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

/*
 * All primes <= limit (limit < 2^32 + 2^20), ascending, plain sieve of
 * Eratosthenes over odd numbers in blocks of one million bytes so that a limit
 * near 2^32 does not need a 4 GB array.  Returns the count; writes at most cap
 * entries to out when out is non-NULL.  Returns -1 when out is too small.
 */
int64_t gbo_primes(uint64_t limit, uint32_t *out, uint64_t cap)
{
    if (limit < 2)
        return 0;
    if (limit > 0xFFFFFFFFull)
        return -2;
    uint64_t r = gbo_isqrt(limit);
    /* seed primes <= r by the textbook sieve on a byte per integer */
    unsigned char *small = (unsigned char *)malloc(r + 1);
    if (!small)
        return -3;
    memset(small, 1, r + 1);
    small[0] = 0;
    if (r >= 1)
        small[1] = 0;
    for (uint64_t i = 2; i * i <= r; i++)
        if (small[i])
            for (uint64_t j = i * i; j <= r; j += i)
                small[j] = 0;
    uint64_t nseed = 0;
    for (uint64_t i = 3; i <= r; i++)
        nseed += small[i] && (i & 1);
    uint64_t *seed = (uint64_t *)malloc((nseed + 1) * sizeof(uint64_t));
    if (!seed) {
        free(small);
        return -3;
    }
    nseed = 0;
    for (uint64_t i = 3; i <= r; i++)
        if (small[i] && (i & 1))
            seed[nseed++] = i;
    free(small);

    int64_t count = 0;
    if (out) {
        if (cap < 1) {
            free(seed);
            return -1;
        }
        out[0] = 2;
    }
    count = 1;

    const uint64_t BLK = 1u << 20; /* odd numbers per block */
    unsigned char *blk = (unsigned char *)malloc(BLK);
    if (!blk) {
        free(seed);
        return -3;
    }
    /* block b covers odd numbers lo, lo+2, ..., lo + 2*(BLK-1), lo = 1 + 2*BLK*b */
    for (uint64_t lo = 1; lo <= limit; lo += 2 * BLK) {
        uint64_t hi = lo + 2 * (BLK - 1);
        if (hi > limit)
            hi = (limit & 1) ? limit : limit - 1;
        uint64_t len = (hi - lo) / 2 + 1;
        memset(blk, 1, len);
        if (lo == 1)
            blk[0] = 0; /* 1 is not prime */
        for (uint64_t k = 0; k < nseed; k++) {
            uint64_t p = seed[k];
            if (p > hi / p)
                break;
            uint64_t start = p * p;
            if (start < lo) {
                uint64_t m = (lo + p - 1) / p * p; /* first multiple >= lo */
                if ((m & 1) == 0)
                    m += p;                        /* odd multiple */
                start = m;
            }
            for (uint64_t m = start; m <= hi; m += 2 * p)
                blk[(m - lo) / 2] = 0;
        }
        for (uint64_t i = 0; i < len; i++) {
            if (blk[i]) {
                if (out) {
                    if ((uint64_t)count >= cap) {
                        free(blk);
                        free(seed);
                        return -1;
                    }
                    out[count] = (uint32_t)(lo + 2 * i);
                }
                count++;
            }
        }
    }
    free(blk);
    free(seed);
    return count;
}

/* (a * b) mod m with a full 128-bit product (Sec. 3.4). */
static uint64_t mulmod128(uint64_t a, uint64_t b, uint64_t m)
{
    return (uint64_t)(((u128)a * b) % m);
}

static uint64_t powmod128(uint64_t a, uint64_t e, uint64_t m)
{
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1)
            r = mulmod128(r, a, m);
        a = mulmod128(a, a, m);
        e >>= 1;
    }
    return r;
}

/*
 * Strong probable-prime test (Miller-Rabin) of odd n > 37 to base a:
 * write n - 1 = d * 2^s with d odd; n passes iff a^d = 1 or a^(d*2^j) = n-1
 * for some 0 <= j < s.
 */
static int strong_probable_prime(uint64_t n, uint64_t a)
{
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        s++;
    }
    uint64_t x = powmod128(a, d, n);
    if (x == 1 || x == n - 1)
        return 1;
    for (int j = 1; j < s; j++) {
        x = mulmod128(x, x, n);
        if (x == n - 1)
            return 1;
    }
    return 0;
}

/*
 * Primality of q < 2^64.  Below 2^32 the textbook definition: trial division
 * by every integer 3, 5, 7, ... up to floor(sqrt(q)).  At and above 2^32 the
 * deterministic Miller-Rabin test with the first twelve primes as bases, which
 * the paper uses for 64-bit q (Sec. 3.3, Sec. 3.4).
 */
int gbo_is_prime(uint64_t q)
{
    if (q < 2)
        return 0;
    if ((q & 1) == 0)
        return q == 2;
    if (q < 0x100000000ull) {
        for (uint64_t d = 3; d <= q / d; d += 2)
            if (q % d == 0)
                return 0;
        return 1;
    }
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (int i = 0; i < 12; i++)
        if (q % bases[i] == 0)
            return 0;
    for (int i = 0; i < 12; i++)
        if (!strong_probable_prime(q, bases[i]))
            return 0;
    return 1;
}

/*
 * Inward rounding of [A, B] to even bounds with A >= 4 (reading of the
 * inclusive range [start, LIMIT] of Sec. 3.5).  Returns 1 when non-empty.
 */
static int normalize(uint64_t A, uint64_t B, uint64_t *An, uint64_t *Bn)
{
    uint64_t b = B & ~(uint64_t)1;
    uint64_t a;
    if (A & 1) {
        if (A == UINT64_MAX) {
            *An = UINT64_MAX;
            *Bn = b;
            return 0;
        }
        a = A + 1;
    } else {
        a = A;
    }
    if (a < 4)
        a = 4;
    *An = a;
    *Bn = b;
    return a <= b;
}

static void account(gbo_result *res, uint64_t n, uint64_t p)
{
    res->verified++;
    res->checksum += p; /* modulo 2^64 by unsigned wraparound */
    if (p > res->max_p || (p == res->max_p && n < res->max_p_n)) {
        res->max_p = p;
        res->max_p_n = n;
    }
}

/*
 * Verify every even n in [A, B].
 *   primes, nprimes : all primes <= T ascending (from gbo_primes(T, ...))
 *   T               : the table limit; sieving needs T >= isqrt(B), and the
 *                     Phase-2 search uses table primes only
 *   P_max           : Phase-1 candidate bound, 2 <= P_max <= T
 *   seg_evens       : evens per oracle segment (any value >= 1; results do not
 *                     depend on it)
 *   res             : aggregates
 *   unresolved/cap  : ascending Phase-1 misses (first cap of them)
 *   pmin_out        : optional, p_min per n in order (0 where none), length
 *                     (B' - A')/2 + 1 -- used by tests on small ranges only
 */
int gbo_verify_range(uint64_t A, uint64_t B, uint64_t P_max,
                     const uint32_t *primes, uint64_t nprimes, uint64_t T,
                     uint64_t seg_evens, gbo_result *res,
                     uint64_t *unresolved, uint64_t cap, uint32_t *pmin_out)
{
    memset(res, 0, sizeof(*res));
    res->P_max = P_max;
    if (P_max < 2 || P_max > T || seg_evens == 0 || nprimes == 0)
        return GBO_EINVAL;
    uint64_t An, Bn;
    int nonempty = normalize(A, B, &An, &Bn);
    res->A = An;
    res->B = Bn;
    if (!nonempty)
        return GBO_OK;
    if (gbo_isqrt(Bn) > T)
        return GBO_ERANGE;

    /* index one past the last odd candidate prime <= P_max */
    uint64_t ncand = 0;
    while (ncand < nprimes && primes[ncand] <= P_max)
        ncand++;

    uint64_t total = (Bn - An) / 2 + 1;     /* number of evens, counted not looped to B */
    uint64_t nseg_max = seg_evens;
    /* window bytes: odd q in [n_lo - P_max, n_hi - 3] */
    uint64_t win_cap = nseg_max + P_max / 2 + 2;
    unsigned char *win = (unsigned char *)malloc(win_cap);
    uint64_t *pend = (uint64_t *)malloc(sizeof(uint64_t) * (nseg_max));
    if (!win || !pend) {
        free(win);
        free(pend);
        return GBO_ENOMEM;
    }
    int status = GBO_OK;
    uint64_t done = 0;
    while (done < total) {
        uint64_t cnt = total - done < seg_evens ? total - done : seg_evens;
        uint64_t n_lo = An + 2 * done;
        uint64_t n_hi = n_lo + 2 * (cnt - 1);
        /* window of odd q; q_lo may be 1 when n_lo <= P_max */
        uint64_t q_lo = n_lo > P_max ? n_lo - P_max : 1;
        q_lo |= 1;
        uint64_t q_hi = n_hi >= 3 ? n_hi - 3 : 1; /* n_hi >= 4 */
        uint64_t nq = q_hi >= q_lo ? (q_hi - q_lo) / 2 + 1 : 0;
        memset(win, 1, nq);
        if (q_lo == 1 && nq)
            win[0] = 0; /* 1 is not prime */
        for (uint64_t k = 1; k < nprimes; k++) { /* odd base primes */
            uint64_t p = primes[k];
            if (p > q_hi / p)
                break;
            u128 start = (u128)p * p;
            if (start < q_lo) {
                u128 m = ((u128)q_lo + p - 1) / p * p;
                if ((m & 1) == 0)
                    m += p;
                start = m;
            }
            for (u128 m = start; m <= q_hi; m += 2 * (u128)p)
                win[(uint64_t)(m - q_lo) / 2] = 0;
        }
        /* scalar probe, candidates ascending */
        uint64_t npend = 0;
        for (uint64_t i = 0; i < cnt; i++) {
            uint64_t n = n_lo + 2 * i;
            uint64_t found = 0;
            if (n == 4) {
                found = 2;
            } else {
                for (uint64_t k = 1; k < ncand; k++) {
                    uint64_t p = primes[k];
                    if (p > n - 3)
                        break;
                    uint64_t q = n - p;
                    if (win[(q - q_lo) / 2]) {
                        found = p;
                        break;
                    }
                }
            }
            if (found) {
                account(res, n, found);
                if (pmin_out)
                    pmin_out[done + i] = (uint32_t)found;
            } else {
                pend[npend++] = n;
                if (pmin_out)
                    pmin_out[done + i] = 0;
            }
        }
        /* Phase 2 for this segment's misses, in ascending n */
        for (uint64_t t = 0; t < npend; t++) {
            uint64_t n = pend[t];
            if (res->n_unresolved < cap && unresolved)
                unresolved[res->n_unresolved] = n;
            else
                status = GBO_ETRUNC;
            res->n_unresolved++;
            uint64_t found = 0;
            for (uint64_t k = ncand; k < nprimes; k++) {
                uint64_t p = primes[k];
                if (p > n / 2)
                    break;
                if (gbo_is_prime(n - p)) {
                    found = p;
                    break;
                }
            }
            if (found) {
                account(res, n, found);
                if (pmin_out)
                    pmin_out[(n - An) / 2] = (uint32_t)found;
            } else {
                res->n_failed++;
            }
        }
        done += cnt;
    }
    free(win);
    free(pend);
    return status;
}

/*
 * Per-q primality over a window by the independent method (gbo_is_prime), so a
 * test can compare it with the sieve on the same q: out[i] = is_prime(q0 + 2i).
 */
void gbo_is_prime_window(uint64_t q0, uint64_t count, unsigned char *out)
{
    for (uint64_t i = 0; i < count; i++)
        out[i] = (unsigned char)gbo_is_prime(q0 + 2 * i);
}

/*
 * The sieve of step 2 alone over odd q in [q0, q0 + 2(count-1)], exposed for
 * the two-method test near 2^64.  primes holds every prime <= T, and T must
 * reach isqrt of the window top.
 */
int gbo_sieve_window(uint64_t q0, uint64_t count, const uint32_t *primes,
                     uint64_t nprimes, uint64_t T, unsigned char *out)
{
    if ((q0 & 1) == 0 || count == 0)
        return GBO_EINVAL;
    uint64_t q_hi = q0 + 2 * (count - 1);
    if (q_hi < q0 || gbo_isqrt(q_hi) > T)
        return GBO_ERANGE;
    memset(out, 1, count);
    if (q0 == 1)
        out[0] = 0;
    for (uint64_t k = 1; k < nprimes; k++) {
        uint64_t p = primes[k];
        if (p > q_hi / p)
            break;
        u128 start = (u128)p * p;
        if (start < q0) {
            u128 m = ((u128)q0 + p - 1) / p * p;
            if ((m & 1) == 0)
                m += p;
            start = m;
        }
        for (u128 m = start; m <= q_hi; m += 2 * (u128)p)
            out[(uint64_t)(m - q0) / 2] = 0;
    }
    return GBO_OK;
}
