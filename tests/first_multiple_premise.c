/*
 * Host check of the double-precision first-multiple arithmetic the kernels
 * use (gb_first_odd_multiple, and the segment kernel's form for window starts
 * below 2^52): the offset d in [0, p) of p's first odd multiple at or above an
 * odd Q = 2h + 1, i.e. d = (p - 1)/2 - h (mod p), compared with 128-bit integer
 * remainders.  Contraction is off (-ffp-contract=off), as in the kernel; the
 * reciprocal is taken one ulp low, nearest and one ulp high in turn, the
 * kernels' Newton-refined reciprocal being within an ulp.  Prints the number of
 * mismatches; exit status 0 when there are none.
 *
 * Usage: first_multiple_premise N
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint64_t next(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
}

static double step_ulp(double x, int dir)
{
    uint64_t b;
    memcpy(&b, &x, 8);
    b += (uint64_t)(int64_t)dir;
    memcpy(&x, &b, 8);
    return x;
}

/* d = (p - 1)/2 - h (mod p) from h = hh + hl (hh = h rounded, hl exact) */
static uint32_t general(double hh, double hl, double pd, double inv, double half)
{
    const double q = floor(hh * inv);
    const double ph = q * pd;
    const double pl = fma(q, pd, -ph);
    const double t = (ph - hh) + (pl + (half - hl));
    const double f = floor(t * inv);
    const uint32_t d = (uint32_t)fma(-f, pd, t);
    return d == (uint32_t)pd ? 0u : d;
}

/* the same for h < 2^51 held exactly in hd */
static uint32_t small(double hd, double pd, double inv)
{
    const double q = floor(hd * inv);
    const double t = fma(q, pd, -hd) + fma(pd, 0.5, -0.5);
    const double f = floor(t * inv);
    const uint32_t d = (uint32_t)fma(-f, pd, t);
    return d == (uint32_t)pd ? 0u : d;
}

static uint64_t want(uint64_t Q, uint32_t p)
{
    const uint64_t r = (uint64_t)((unsigned __int128)Q % p);
    const uint64_t x = r ? p - r : 0;   /* 2d = -Q (mod p) */
    return (x & 1) ? (x + p) / 2 : x / 2;
}

int main(int argc, char **argv)
{
    const long n = argc > 1 ? atol(argv[1]) : 1000000;
    long bad = 0;
    for (long it = 0; it < n; ++it) {
        uint32_t p;
        switch (it % 5) {
        case 0: p = 3 + 2 * (uint32_t)(next() % 200); break;
        case 1: p = 0xFFFFFFFFu - 2 * (uint32_t)(next() % 100000); break;
        case 2: p = ((uint32_t)next() >> (next() % 30)) | 3u; break;
        default: p = (uint32_t)next() | 1u; if (p < 3) p = 3;
        }
        uint64_t Q;
        switch ((it / 5) % 4) {
        case 0: Q = next() | 1; break;
        case 1: Q = 0xFFFFFFFFFFFFFFFFull - 2 * (next() % 1000000); break;
        case 2: {   /* next to a multiple of p */
            const uint64_t k = next() % (0xFFFFFFFFFFFFFFF0ull / p);
            Q = (k * p + 2 * (next() % 3)) | 1;
            break;
        }
        default: Q = (next() >> (next() % 63)) | 1;
        }
        const uint64_t h = Q >> 1;
        const double pd = (double)p, half = (double)(p >> 1);
        const double inv = step_ulp(1.0 / pd, (int)(it % 3) - 1);
        const double hh = (double)h;
        const double hl = (double)(int64_t)(h - (uint64_t)hh);
        const uint64_t w = want(Q, p);
        if (general(hh, hl, pd, inv, half) != w) {
            if (bad < 5)
                printf("general: p=%u Q=%llu\n", p, (unsigned long long)Q);
            ++bad;
        }
        /* the small-window form: p < 2^26, Q < 2^52, p >= 37 as in the kernel */
        if (p >= 37 && p < (1u << 26)) {
            const uint64_t Qs = Q & ((1ull << 52) - 1);
            const double hs = (double)(Qs >> 1);
            if (small(hs, pd, inv) != want(Qs, p)) {
                if (bad < 5)
                    printf("small: p=%u Q=%llu\n", p, (unsigned long long)Qs);
                ++bad;
            }
        }
    }
    printf("%ld\n", bad);
    return bad != 0;
}
