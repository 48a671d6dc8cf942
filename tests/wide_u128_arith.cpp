// Host driver for the 128-bit helpers of the verification past 2^64
// (paper_2603_07850_amd/csrc/gb_wide_u128.h, compiled here as plain C++): the
// product of a residue by a constant below 2^40 reduced with a double-precision
// quotient estimate, and 2^(28 N) mod q.  Seeded cases -- moduli of 64 to 128 bits,
// residues near q, products next to multiples of q, constants of 1 to 40 bits
// and the small constants of the Lucas setup -- are printed in hex for
// tests/test_wide_limb_arith.py to check with exact integers.
#include <cstdio>
#include <cstdlib>
#include <cstdint>

#define GB_WIDE_FN static inline
static inline uint64_t __umul64hi(uint64_t a, uint64_t b)
{
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
}
#include "../paper_2603_07850_amd/csrc/gb_wide_u128.h"

typedef unsigned __int128 u128;

static uint64_t s_state;
static uint64_t next64()
{
    uint64_t z = (s_state += 0x9E3779B97F4A7C15ull);   // splitmix64
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int main(int argc, char **argv)
{
    const long n = argc > 1 ? atol(argv[1]) : 10000;
    s_state = argc > 2 ? strtoull(argv[2], nullptr, 10) : 1;
    for (long c = 0; c < n; ++c) {
        const int bits = 64 + (int)(next64() % 65);
        u128 q = ((u128)next64() << 64) | next64();
        if (bits < 128)
            q &= ((u128)1 << bits) - 1;
        q |= (u128)1 << (bits - 1);
        q |= 1;
        const u128w qw = {(uint64_t)q, (uint64_t)(q >> 64)};
        const double qinv = w_recip_d(qw);
        // the constant: 1 to 40 bits, or a power of two
        const int cb = 1 + (int)(next64() % 40);
        uint64_t k = (next64() % 3 == 0) ? (1ull << (cb - 1)) : (next64() >> (64 - cb)) | 1;
        // the residue: random, next to q, or next to a multiple of q divided by k
        u128 x;
        const int kind = (int)(next64() % 3);
        if (kind == 0) {
            x = (((u128)next64() << 64) | next64()) % q;
        } else if (kind == 1) {
            x = q - 1 - (next64() % 1000) % q;
        } else {
            // x k within a few units of m q for a random m < k
            const uint64_t m = next64() % k;
            const u128 t = (u128)m * (uint64_t)(q >> 40);   // avoids 168-bit arithmetic:
            x = (t << 40) / k;                             // about m q / k
            x = x % q;
        }
        const u128w xw = {(uint64_t)x, (uint64_t)(x >> 64)};
        const u128w r = w_mul_small(xw, k, qw, qinv);
        // R = 2^(28 N) for the limb count the probe gives q (N = 3, 4, 5 below
        // 2^72, 2^100, 2^128)
        const int rbits = bits <= 72 ? 84 : (bits <= 100 ? 112 : 140);
        const u128w one = w_r_mod(qw, rbits);
        printf("%llx %llx %llx %llx %llx %llx %llx %d %llx %llx\n", (unsigned long long)qw.hi,
               (unsigned long long)qw.lo, (unsigned long long)xw.hi, (unsigned long long)xw.lo,
               (unsigned long long)k, (unsigned long long)r.hi, (unsigned long long)r.lo, rbits,
               (unsigned long long)one.hi, (unsigned long long)one.lo);
    }
    return 0;
}
