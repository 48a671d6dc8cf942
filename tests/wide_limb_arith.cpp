// Host driver for the Montgomery arithmetic over 28-bit limbs used by the
// Baillie-PSW test past 2^64 (paper_2603_07850_amd/csrc/gb_wide_w5.h, compiled
// here as plain C++).  It draws seeded cases -- moduli of 64 to 128 bits,
// operands at the limits of the documented bounds (limbs up to 2^30 - 1, values
// up to 8q - 1, in non-normalized limb forms) -- and prints operands and
// results in hex, one case per line, for tests/test_wide_limb_arith.py to check
// with exact integers.
#include <cstdio>
#include <cstdlib>
#include <cstdint>

#define GB_W5_FN static inline
#include "../paper_2603_07850_amd/csrc/gb_wide_w5.h"

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

// A random value below lim (lim < 2^131) as five limbs, then spread: some
// units moved from a limb to the one below, keeping every limb below 2^30.
static w5 draw(const u128 &lim_lo, uint32_t lim_top, bool spread)
{
    // value = r mod lim, lim = lim_lo + 2^128 lim_top
    w5 x;
    for (;;) {
        u128 v = ((u128)next64() << 64) | next64();
        const uint32_t top = lim_top ? (uint32_t)(next64() % (lim_top + 1)) : 0;
        if (top == lim_top) {
            if (lim_lo == 0)
                continue;
            v %= lim_lo;
        }
        x = w5_from((uint64_t)v, (uint64_t)(v >> 64));
        x.l[4] += top << 16;   // 2^128 = 2^(4*28 + 16)
        break;
    }
    if (spread) {
        for (int j = 4; j > 0; --j) {
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

static void put(const w5 &x)
{
    for (int j = 0; j < 5; ++j)
        printf(" %x", x.l[j]);
}

int main(int argc, char **argv)
{
    const long n = argc > 1 ? atol(argv[1]) : 10000;
    s_state = argc > 2 ? strtoull(argv[2], nullptr, 10) : 1;
    for (long c = 0; c < n; ++c) {
        const int bits = 64 + (int)(next64() % 65);   // 64 .. 128
        u128 q = ((u128)next64() << 64) | next64();
        if (bits < 128)
            q &= ((u128)1 << bits) - 1;
        q |= (u128)1 << (bits - 1);
        q |= 1;
        const w5 q5 = w5_from((uint64_t)q, (uint64_t)(q >> 64));
        const uint32_t qi = w5_qinv((uint64_t)q);
        // bound 8q as (low 128 bits, top)
        const u128 q8 = q << 3;
        const uint32_t q8top = (uint32_t)(q >> 125);
        const int kind = (int)(next64() % 4);
        w5 a, b;
        if (kind == 0) {          // canonical operands
            a = draw(q, 0, false);
            b = draw(q, 0, false);
        } else {                  // lazy operands up to 8q - 1
            a = draw(q8, q8top, true);
            b = draw(q8, q8top, true);
        }
        const w5 r = w5_mont(a, b, q5, qi);
        printf("mont %x", qi);
        put(q5);
        put(a);
        put(b);
        put(r);
        printf("\n");
        // exact helpers on normalized values below 2q
        const w5 twoq = w5_norm(w5_add(q5, q5));
        const w5 y = w5_canon<1>(r, q5);           // r < 1.01 q
        const w5 z = w5_sub(twoq, r);              // 2q - r
        const w5 s = w5_canon<5>(w5_add(w5_add(r, z), w5_add(z, z)), q5);
        printf("help");
        put(y);
        put(z);
        put(s);
        printf("\n");
    }
    return 0;
}
