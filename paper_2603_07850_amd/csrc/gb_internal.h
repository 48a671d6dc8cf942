// gb_internal.h -- structures and launch entry points shared by the
// translation units of libgoldbach (device code and host runtime).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// One verification interval of a launch, as the device sees it.
struct GbInterval {
    uint64_t A;          // first even n (normalized)
    uint64_t nE;         // number of evens in the interval (0 for an empty one)
    uint64_t seg_first;  // index of the interval's first segment in the launch
    uint64_t nseg;       // number of segments of the interval
};

// Partial aggregates of one segment, written by the sieve+probe kernel.
struct GbSegRecord {
    uint64_t checksum;   // sum of p_min of the n resolved in the segment (mod 2^64)
    uint64_t verified;   // number of n resolved in the segment's probe
    uint64_t max_n;      // smallest n attaining max_p in the segment
    uint32_t max_p;      // largest p_min found in the segment (0 if none)
    uint32_t pad;
};

// An n the probe window did not resolve.  p is filled by the Phase-2 kernel
// (0 if no prime was found).
struct GbSpill {
    uint64_t n;
    uint32_t iv;
    uint32_t p;
};

// Final aggregates of one interval (device side).
struct GbIvResult {
    uint64_t verified;
    uint64_t checksum;
    uint64_t max_p;
    uint64_t max_p_n;
    uint64_t n_unresolved;
    uint64_t n_failed;
    uint64_t unres_first;  // position of the interval's list in the unresolved output
    uint64_t pad;
};

// Device counters of one launch; cleared by gb_launch_reset at the start.
struct GbCounters {
    unsigned long long claim;   // next segment to claim
    unsigned long long spills;  // spill entries appended (may exceed the capacity)
    unsigned long long pad[6];
};

// Arguments of the persistent sieve + probe kernel.
struct GbProbeArgs {
    const uint32_t *primes;   // the prime table, ascending, primes[0] = 2
    uint64_t nprimes;
    const GbInterval *iv;
    uint32_t k;               // number of intervals
    uint32_t H;               // halo in bits (multiple of 32)
    uint32_t ncand;           // odd candidates probed in LDS: primes[1 .. ncand]
    uint32_t pad;
    uint64_t total_segs;
    GbSegRecord *rec;
    GbSpill *spill;
    uint64_t spill_cap;
    GbCounters *ctr;
};

// Launch wrappers (each returns the hipError_t of its launch).
hipError_t gb_launch_seed(uint32_t *seed, uint32_t *nseed, hipStream_t s);
hipError_t gb_launch_table_count(const uint32_t *seed, const uint32_t *nseed, uint64_t T,
                                 uint32_t nsegs, uint32_t *counts, hipStream_t s);
hipError_t gb_launch_table_scan(uint32_t *counts, uint32_t nsegs, uint64_t *total, hipStream_t s);
hipError_t gb_launch_table_emit(const uint32_t *seed, const uint32_t *nseed, uint64_t T,
                                uint32_t nsegs, const uint32_t *offsets, uint32_t *primes,
                                hipStream_t s);
uint32_t gb_table_seg_log2();

hipError_t gb_launch_reset(GbCounters *ctr, hipStream_t s);
hipError_t gb_launch_probe(int seg_log2, int wg_size, uint32_t grid, const GbProbeArgs &a,
                           hipStream_t s);
int gb_probe_supported(int seg_log2, int wg_size);
hipError_t gb_probe_occupancy(int seg_log2, int wg_size, int *blocks_per_cu);

hipError_t gb_launch_phase2(const uint32_t *primes, uint64_t nprimes, uint64_t first_idx,
                            GbSpill *spill, uint64_t spill_cap, const GbCounters *ctr,
                            uint32_t grid, hipStream_t s);
hipError_t gb_launch_reduce(const GbInterval *iv, uint32_t k, const GbSegRecord *rec,
                            const GbSpill *spill, uint64_t spill_cap, const GbCounters *ctr,
                            uint64_t P_max, GbIvResult *res, hipStream_t s);
hipError_t gb_launch_unres_emit(const GbSpill *spill, uint64_t spill_cap, const GbCounters *ctr,
                                uint64_t P_max, uint64_t *out, uint32_t grid, hipStream_t s);
hipError_t gb_launch_is_prime(const uint64_t *q, uint64_t count, uint8_t *out, hipStream_t s);
