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
    unsigned long long claim;    // unused (each launch has its own queue head)
    unsigned long long spills;   // spill entries appended (may exceed the capacity)
    unsigned long long t_start;  // device wall clock when the launch sequence began
    unsigned long long pad[5];   // pad[0]: largest overflowing bucket count
};

// Per-interval completion: segments finished and the device wall clock when
// the interval's last segment finished (the batched form's latency).
struct GbIvDone {
    unsigned long long segs_done;
    unsigned long long t_done;
};

// Arguments of the persistent sieve + probe kernel.  One launch processes the
// segments [seg_base, seg_base + nsegs) of the global segment numbering.
struct GbProbeArgs {
    const uint32_t *primes;   // the prime table, ascending, primes[0] = 2
    uint64_t nprimes;
    const GbInterval *iv;
    uint32_t k;               // number of intervals
    uint32_t H;               // halo in bits (multiple of 32)
    uint32_t ncand;           // odd candidates probed in LDS: primes[1 .. ncand]
    uint32_t lb_count;        // primes[0 .. lb_count) are sieved in the segment
    uint64_t seg_base;
    uint64_t nsegs;
    GbSegRecord *rec;
    GbSpill *spill;
    uint64_t spill_cap;
    GbCounters *ctr;
    unsigned long long *claim;  // this launch's segment queue head
    GbIvDone *done;
    const uint32_t *bitmap;   // per segment 3 * wcu words (class layout): bits struck by large
                              // primes; null when the launch has no buckets
    const uint32_t *ctab;     // probe candidate tables, 3 words per entry (see below)
    const uint32_t *ptab;     // the candidate p of each table entry
    uint32_t wcu;             // class-array words in use per segment, (E + H)/96 + 1
    uint32_t nv[9];           // entries of table (r, t3) with p <= the probe window
};

// The segment window in LDS is stored by class: odd bit b (odd number
// q_lo + 2b) is bit b / 3 of class array b mod 3.  One class holds the
// multiples of 3 (the class t3 with q_lo + 2*t3 = 0 mod 3) and is not stored;
// classes t3 + 1 and t3 + 2 (mod 3) are kept in LDS slots 0 and 1.  The halo H is a multiple of 96, so class index
// b / 3 = i' + H/3 + (r - h - t)/3 for b = r + 3i' + H - h.
constexpr uint32_t kHaloMax = 32832;  // largest halo: multiple of 96 >= 32767 + 2

// Words of one class array in the LDS window of a 2^log2e-even segment (with
// room for the probe's reads past the last block).
constexpr uint32_t gb_class_words(int log2e)
{
    return (uint32_t)(((1u << log2e) + kHaloMax + 95) / 96) + 4;
}

// Probe candidate tables, one per (segment size 2^18 / 2^19 / 2^20, class r of
// the evens, class t3 of the multiples of 3): the odd primes p <= 65536 whose
// n - p avoids class t3 (the others cannot be prime, n - p = 3 aside), in
// ascending order.  Entry: {byte offset, to subtract from the lane's base,
// of the first LDS word holding bit(n - p), slot of its class included;
// funnel-shift amount; p minus the
// previous entry's p (0 before the first)}.  Table (lg, r, t3) starts at entry
// ((lg - 18) * 9 + r * 3 + t3) * kCandStride.
constexpr uint32_t kCandStride = 6560;

// A run of consecutive segments of one interval that the bucket-fill kernel
// treats as one window [Q0, Q0 + 2*dmax] of odd numbers.
struct GbChunk {
    uint64_t seg_first;   // global index of the chunk's first segment
    uint64_t Q0;          // odd number at window bit 0 of the first segment
    uint64_t dmax;        // last window bit any segment of the chunk reads
    uint32_t nseg;
    uint32_t p_root;      // one past the last table prime <= isqrt(Q0 + 2*dmax)
    double hh;            // h = (Q0 - 1) / 2 rounded to double
    double hl;            // h - hh, exact (|hl| <= 2^9)
    uint32_t sqrt_q0;     // isqrt(Q0): only larger primes can have p^2 above Q0
    uint32_t q0m3;        // Q0 mod 3
};

// One fill task: the table primes [p_first, p_first + np) of one band
// (2^b, 2^(b+1)] against nchunk consecutive chunks of the round; a tile is
// kFillThreads * kFillPerThread consecutive primes of the task, and each
// (prime, chunk) item takes one remainder and walks the prime's multiples
// across the chunk.
struct GbFillTask {
    uint64_t tile_first;  // first fill tile of the task (within the round)
    uint32_t chunk_first; // index into the round's chunks
    uint32_t nchunk;
    uint32_t p_first;
    uint32_t np;          // an upper bound; items past a chunk's p_root skip it
};

struct GbBucketArgs {
    const uint32_t *primes;
    const GbChunk *chunk;
    const GbFillTask *task;
    uint32_t ntask;
    uint32_t log2e;
    uint32_t H;
    uint32_t words;       // bitmap words per segment, 3 * wcu
    uint64_t ntiles;
    uint64_t seg_base;    // global index of the round's first segment
    uint32_t *bitmap;     // the round's strike bitmaps, segment after segment
    uint32_t wcu;         // class-array words per segment bitmap (three per segment)
};


// Set the calling thread's gb_last_error() message (host code).
void gb_internal_set_error(const char *msg);

// Launch wrappers (each returns the hipError_t of its launch).
hipError_t gb_launch_seed(uint32_t *seed, uint32_t *nseed, hipStream_t s);
hipError_t gb_launch_table_count(const uint32_t *seed, const uint32_t *nseed, uint64_t T,
                                 uint32_t nsegs, uint32_t *counts, uint32_t *stash, hipStream_t s);
hipError_t gb_launch_table_scan(uint32_t *counts, uint32_t nsegs, uint64_t *total, hipStream_t s);
hipError_t gb_launch_table_emit(const uint32_t *stash, uint32_t nsegs, const uint32_t *offsets,
                                uint32_t *primes, hipStream_t s);
uint32_t gb_table_seg_log2();
uint32_t gb_table_block_words();   // 32-bit words of one block's stored bits

hipError_t gb_launch_reset(GbCounters *ctr, GbIvDone *done, uint32_t k,
                           unsigned long long *claims, uint32_t nclaims, hipStream_t s);
hipError_t gb_launch_put_interval(GbInterval *dst, const GbInterval &v, hipStream_t s);
hipError_t gb_launch_pow2_counts(const uint32_t *primes, uint64_t nprimes, uint64_t *out33,
                                 hipStream_t s);
hipError_t gb_launch_chunk_roots(const uint32_t *primes, uint64_t nprimes, GbChunk *chunks,
                                 uint64_t nchunk, hipStream_t s);
hipError_t gb_launch_probe(int seg_log2, int wg_size, uint32_t grid, const GbProbeArgs &a,
                           hipStream_t s);
int gb_probe_supported(int seg_log2, int wg_size);
hipError_t gb_probe_occupancy(int seg_log2, int wg_size, int *blocks_per_cu);

constexpr uint32_t kFillThreads = 256;
constexpr uint32_t kFillPerThread = 4;   // work items per thread in one fill tile
constexpr uint32_t kFillChunks = 16;     // chunks of one fill task
hipError_t gb_launch_bucket_reset(uint32_t *bitmap, uint64_t words, hipStream_t s);
hipError_t gb_launch_bucket_fill(const GbBucketArgs &a, uint32_t grid, hipStream_t s);

hipError_t gb_launch_phase2(const uint32_t *primes, uint64_t nprimes, uint64_t first_idx,
                            GbSpill *spill, uint64_t spill_cap, const GbCounters *ctr,
                            uint32_t grid, hipStream_t s);
hipError_t gb_launch_reduce(const GbInterval *iv, uint32_t k, const GbSegRecord *rec,
                            const GbSpill *spill, uint64_t spill_cap, const GbCounters *ctr,
                            uint64_t P_max, GbIvResult *res, hipStream_t s);
hipError_t gb_launch_unres_emit(const GbSpill *spill, uint64_t spill_cap, const GbCounters *ctr,
                                uint64_t P_max, uint64_t *out, uint32_t grid, hipStream_t s);
// gb_result image and status word written by the finalize kernel (the status
// at this byte offset of the image buffer).
constexpr size_t kFinalizeStatusOffset = 96;
hipError_t gb_launch_finalize(const GbIvResult *res, const GbCounters *ctr, uint64_t spill_cap,
                              uint64_t A, uint64_t B, uint64_t P_max, uint64_t *unres,
                              uint64_t cap, void *img, hipStream_t s);
// Unresolved list by bitmap and scan (one bit per even of each interval; the
// bits of interval i start at word woff[i]), for lists too long for the
// pairwise ranking.
hipError_t gb_launch_unres_bitmap(const GbSpill *spill, uint64_t spill_cap, const GbCounters *ctr,
                                  uint64_t P_max, const GbInterval *iv, uint32_t k,
                                  const uint64_t *woff, uint64_t words, uint32_t *bitmap,
                                  uint64_t *blocksum, uint64_t *out, uint32_t grid, hipStream_t s);
uint64_t gb_unres_bitmap_blocks(uint64_t words);
hipError_t gb_launch_is_prime(const uint64_t *q, uint64_t count, uint8_t *out, hipStream_t s);
