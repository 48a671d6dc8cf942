// gb_wide_types.h -- types and launch wrappers shared by the kernels that
// verify past 2^64 (gb_wide.hip) and the runtime that drives them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gb_wide_u128.h"

// Partial aggregates of the evens one wide probe workgroup settled (summed
// over the chunks of a call).
struct GbWideRecord {
    uint64_t checksum;
    uint64_t verified;
    uint64_t max_p;
    uint64_t max_n_lo, max_n_hi;   // smallest n attaining max_p (0 if none)
    uint64_t nspill;
    uint64_t pad[2];
};

// An even past 2^64 that the candidates p <= P_max left open; p is set by the
// wide Phase-2 kernel (0: none found).
struct GbWideSpill {
    uint64_t n_lo, n_hi;
    uint64_t p;
    uint64_t pad;
};

struct GbWideResult {
    uint64_t verified, checksum, max_p, max_n_lo, max_n_hi, n_unresolved, n_failed, spills;
};

struct GbWideArgs {
    const uint32_t *primes;
    uint64_t nprimes;
    uint32_t nsieve;      // primes[1 .. nsieve) are sieved out of every window
    uint32_t ncand;       // candidates primes[1 .. ncand]
    uint32_t H;           // halo bits: hmax + 32, rounded up to a multiple of 32
    uint32_t hmax;        // (largest candidate - 1) / 2 (0: no candidate)
    uint32_t nsmall;      // primes[1 .. nsmall) (below 2^16) are struck in LDS
    uint32_t ncoop;       // primes[1 .. ncoop) (below 2^12) are struck by a whole wave
    uint32_t nrec;        // probe records (the probe grid's upper bound)
    u128w A;              // first even of the range
    uint64_t nE;          // evens of the range
    GbWideRecord *rec;
    GbWideSpill *spill;
    uint64_t spill_cap;
    unsigned long long *ctr;   // [0] probe claims in the current chunk, [1] spills appended
};

// One chunk of a wide range: its evens n0 + 2i (0 <= i < cnt) and the strike
// bitmap of the odd numbers q_lo + 2b (0 <= b < nbits = cnt + H) below them.
struct GbWideChunk {
    u128w n0;
    u128w qlo;            // n0 - 1 - 2H
    uint32_t cnt;
    uint32_t nbits;
    uint32_t *bits;       // ceil(nbits / 32) words and a spare one; bit b set: q_lo + 2b has a factor <= S
    uint32_t lucas_at;    // a wave runs its Lucas round once this many lanes are ready
};

constexpr int kWideThreads = 256;
constexpr uint32_t kWideCandWords = 1024;    // the probe's table of candidate half-offsets below 2^15
constexpr uint32_t kWideSieveWords = 1024;   // bitmap words per LDS pass of the small primes
constexpr uint32_t kWideChunkLog2Default = 26;
constexpr uint32_t kWideChunkLog2Min = 12, kWideChunkLog2Max = 30;

// The three kernels of one chunk: the primes below 2^16 struck in LDS and
// written as whole words, then the larger sieving primes OR-ed in by atomics,
// then the persistent probe (grid blocks, at most a.nrec) with its arithmetic
// over `limbs` 28-bit limbs (3, 4 or 5: every q of the chunk below
// 2^(28 limbs - 12)).
hipError_t gb_launch_wide_chunk(const GbWideArgs &a, const GbWideChunk &ch, uint32_t sieve_grid,
                                uint32_t fill_grid, int limbs, uint32_t grid, hipStream_t s);
// Probe blocks per CU for the given limb count.
int gb_wide_occupancy(int limbs);
hipError_t gb_launch_wide_phase2(const GbWideArgs &a, uint32_t grid, hipStream_t s);
hipError_t gb_launch_wide_reduce(const GbWideArgs &a, uint64_t P_max, GbWideResult *res,
                                 u128w *unres, hipStream_t s);
// Zero the counters and the a.nrec probe records.
hipError_t gb_launch_wide_reset(const GbWideArgs &a, hipStream_t s);
hipError_t gb_launch_bpsw(const u128w *q, uint64_t count, uint8_t *out, hipStream_t s);
