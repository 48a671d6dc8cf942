// Host driver for the Montgomery arithmetic over N 28-bit limbs used by the
// Baillie-PSW test past 2^64 (paper_2603_07850_amd/csrc/gb_wide_limbs.h,
// compiled here as plain C++).  It draws seeded cases -- a limb count N of 3, 4
// or 5 and a modulus of the sizes it serves (61 to 72, 73 to 100, 101 to 128
// bits), operands at the limits of the documented bounds (limbs up to 2^30 - 1,
// values up to 8q - 1, in non-normalized limb forms) -- and prints operands and
// results in hex, one case per line, for tests/test_wide_limb_arith.py to check
// with exact integers.
#include <cstdio>
#include <cstdlib>
#include <cstdint>

#define GB_WIDE_FN static inline
#include "../paper_2603_07850_amd/csrc/gb_wide_limbs.h"

typedef unsigned __int128 u128;

static uint64_t s_state;
static uint64_t next64()
{
    // splitmix64
    uint64_t z = (s_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// A random value below lim (lim = lim_lo + 2^128 lim_top) as N limbs, then
// spread: some units moved from a limb to the one below, keeping every limb
// below 2^30.
template <int N>
static wl<N> draw(const u128 &lim_lo, uint32_t lim_top, bool spread)
{
    wl<N> x;
    for (;;) {
        u128 v = ((u128)next64() << 64) | next64();
        const uint32_t top = lim_top ? (uint32_t)(next64() % (lim_top + 1)) : 0;
        if (top == lim_top) {
            if (lim_lo == 0)
                continue;
            v %= lim_lo;
        }
        x = wl_from<N>((uint64_t)v, (uint64_t)(v >> 64));
        if (N == 5)
            x.l[N - 1] += top << 16;   // 2^128 = 2^(4*28 + 16)
        break;
    }
    if (spread) {
        for (int j = N - 1; j > 0; --j) {
            const uint32_t room = ((1u << 30) - 1 - x.l[j - 1]) >> 28;   // units of 2^28 that fit
            uint32_t t = room ? (uint32_t)(next64() % (room + 1)) : 0;
            if (t > x.l[j])
                t = x.l[j];
            x.l[j] -= t;
            x.l[j - 1] += t << 28;
        }
    }
    return x;
}

template <int N>
static void put(const wl<N> &x)
{
    for (int j = 0; j < N; ++j)
        printf(" %x", x.l[j]);
}

template <int N>
static void one_case()
{
    const int lo_bits = N == 3 ? 61 : (N == 4 ? 73 : 101), hi_bits = 28 * N - 12;
    const int bits = lo_bits + (int)(next64() % (hi_bits - lo_bits + 1));
    u128 q = ((u128)next64() << 64) | next64();
    if (bits < 128)
        q &= ((u128)1 << bits) - 1;
    q |= (u128)1 << (bits - 1);
    q |= 1;
    const wl<N> q5 = wl_from<N>((uint64_t)q, (uint64_t)(q >> 64));
    const uint32_t qi = wl_qinv((uint64_t)q);
    // bound 8q as (low 128 bits, top)
    const u128 q8 = q << 3;
    const uint32_t q8top = (uint32_t)(q >> 125);
    const int kind = (int)(next64() % 4);
    wl<N> a, b;
    if (kind == 0) {          // canonical operands
        a = draw<N>(q, 0, false);
        b = draw<N>(q, 0, false);
    } else {                  // lazy operands up to 8q - 1
        a = draw<N>(q8, q8top, true);
        b = draw<N>(q8, q8top, true);
    }
    const wl<N> r = wl_mont(a, b, q5, qi);
    printf("mont %d %x", N, qi);
    put(q5);
    put(a);
    put(b);
    put(r);
    printf("\n");
    // exact helpers on normalized values below 2q
    const wl<N> twoq = wl_norm(wl_add(q5, q5));
    const wl<N> y = wl_canon<N, 1>(r, q5);       // r < 1.02 q
    const wl<N> z = wl_sub(twoq, r);             // 2q - r
    const wl<N> s = wl_canon<N, 5>(wl_add(wl_add(r, z), wl_add(z, z)), q5);
    printf("help");
    put(y);
    put(z);
    put(s);
    printf("\n");
    // the product by a small signed Q (0 < |Q| <= 2^14 + 1) of the Montgomery
    // product's output (below 1.02 q), the edges of Q's range drawn often
    const int32_t edges[6] = {1, 2, 3, (1 << 14) - 1, 1 << 14, (1 << 14) + 1};
    const uint32_t pick = (uint32_t)(next64() % 8);
    int32_t Q = pick < 6 ? edges[pick] : 1 + (int32_t)(next64() % ((1 << 14) + 1));
    if (next64() & 1)
        Q = -Q;
    const double qrecip = 1.0 / ((double)(uint64_t)(q >> 64) * 18446744073709551616.0 +
                                 (double)(uint64_t)q);
    const wl<N> m = wl_mul_q(r, Q, q5, qrecip);
    printf("mulq %d", Q);
    put(m);
    printf("\n");
}

int main(int argc, char **argv)
{
    const long n = argc > 1 ? atol(argv[1]) : 10000;
    s_state = argc > 2 ? strtoull(argv[2], nullptr, 10) : 1;
    for (long c = 0; c < n; ++c) {
        const int N = 3 + (int)(next64() % 3);
        if (N == 3)
            one_case<3>();
        else if (N == 4)
            one_case<4>();
        else
            one_case<5>();
    }
    return 0;
}
