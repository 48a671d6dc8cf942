/*
 * goldbach.h -- C ABI of libgoldbach, device-resident segmented double-sieve
 * verification of Goldbach's conjecture on one AMD Instinct MI355X (gfx950).
 *
 * The problem (paper Sec. 1): every even n > 2 is a sum of two primes.  For
 * every even n of a range the library finds the minimal prime p with n - p
 * prime,   p_min(n) = min { p prime : n - p prime },   and returns aggregates
 * of these minimal partitions.  Phase 1 (Sec. 3.1, Sec. 3.3) searches p among
 * candidate primes p <= P_max against a sieved bitset of the odd q = n - p;
 * Phase 2 (Sec. 3.3, Sec. 3.4) finishes the n that Phase 1 leaves unresolved
 * with larger table primes and a deterministic 64-bit Miller-Rabin test.
 *
 * Conventions shared by every entry point:
 *  - Plain C types only; no exceptions cross the ABI and nothing calls exit
 *    or abort (Sec. 3.4, graceful error handling).  Every call returns a
 *    gb_status; on failure gb_last_error() gives a message for the calling
 *    thread and everything the failing call allocated has been released.
 *  - Arguments are validated before any work is enqueued (Sec. 3.5, resource
 *    validation before launch).
 *  - `stream` is a hipStream_t (NULL = the default stream).  The calls below
 *    enqueue their kernels on that stream and, except for
 *    gb_verify_range_async, wait for it before returning, so results are in
 *    the caller's host structures on return.
 *  - All u64 bounds up to 2^64 - 1 are accepted; the arithmetic inside is
 *    guarded against wrap-around up to that ceiling (Sec. 3.4).
 *  - One device per process: the device current at gb_base_primes() holds the
 *    tables; later calls make it current again.  Calls are serialized by an
 *    internal lock.
 */
#ifndef GOLDBACH_H
#define GOLDBACH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gb_status {
    GB_OK = 0,
    GB_EINVAL = 1,   /* an argument is out of its documented domain */
    GB_ERANGE = 2,   /* the prime table does not reach isqrt(B), or P_max exceeds it */
    GB_ENOMEM = 3,   /* device or pinned-host allocation failed, or a budget is exceeded */
    GB_EHIP = 4,     /* the HIP runtime reported an error (launch, copy, sync) */
    GB_ETRUNC = 5,   /* an unresolved list did not fit its buffer; every count is still exact */
    GB_ENOTABLE = 6, /* gb_base_primes() has not been called (or gb_release() has) */
    GB_EBUSY = 7     /* server: no result ready yet, or the admission queue is full */
} gb_status;

/*
 * Result of one verified range.  Written by the library into caller-owned
 * host memory.  Field meanings:
 *   A, B          the range after normalization: inclusive, rounded inward to
 *                 even numbers, A raised to 4; A > B means the range was empty.
 *   P_max         the Phase-1 candidate bound used (echoed).
 *   verified      number of even n in [A, B] for which some p_min was found
 *                 (Phase 1 or Phase 2).
 *   max_p         largest p_min over the range (0 if nothing verified).
 *   max_p_n       the smallest n attaining max_p (0 if nothing verified).
 *   checksum      sum of p_min over all verified n, modulo 2^64.
 *   n_unresolved  number of n with no prime p <= P_max such that n - p is prime
 *                 (the n that Phase 1 hands to Phase 2, Sec. 3.3).
 *   n_failed      number of n for which Phase 2 also found nothing among the
 *                 table primes p <= min(T, n/2) (a counterexample candidate;
 *                 expected 0).
 *   unresolved    caller-owned host buffer that receives the first
 *                 unresolved_cap unresolved n in ascending order (may be NULL
 *                 when unresolved_cap is 0).  GB_ETRUNC when it is too small.
 */
typedef struct gb_result {
    uint64_t A, B;
    uint64_t P_max;
    uint64_t verified;
    uint64_t max_p;
    uint64_t max_p_n;
    uint64_t checksum;
    uint64_t n_unresolved;
    uint64_t n_failed;
    uint64_t *unresolved;
    uint64_t unresolved_cap;
} gb_result;

/*
 * Launch parameters of the segment sieve + probe kernel (scheduling only:
 * they never change a result field).
 *   seg_log2   log2 of the evens per segment: 18, 19 or 20; the segment's
 *              LDS window holds 2^seg_log2 + halo odd numbers as bits
 *              (about 32, 64 or 128 KB per workgroup).
 *   wg_size    threads per workgroup: 256, 512 or 1024.
 *   window     probe window: candidates p <= min(P_max, window) are tested in
 *              LDS by the probe; candidates window < p <= P_max are tested by
 *              the Phase-2 kernel for the (rare) n the window leaves open.
 *              0 means window = P_max.  Must be 0 or in [3, 65536].
 *   wg_per_cu  workgroups per compute unit in the persistent grid; 0 = the
 *              maximum that LDS allows.
 *   bucket_log2  primes above 2^bucket_log2 are not sieved segment by segment
 *              but through per-segment strike bitmaps in HBM, filled once per
 *              run of segments; 17..32 (32 = never) applies to every range
 *              whose isqrt(B) exceeds the bound; 0 = automatic: bound
 *              2^(seg_log2 + 4).
 *   bucket_mib HBM budget for the strike bitmaps of one round, in MiB;
 *              0 = automatic: 512 for the first round, 8192 for the next
 *              ones.  Larger batches run in several rounds.  Only the
 *              bitmaps of the segments a round holds are allocated.
 */
typedef struct gb_params {
    uint32_t seg_log2;
    uint32_t wg_size;
    uint32_t window;
    uint32_t wg_per_cu;
    uint32_t bucket_log2;
    uint32_t bucket_mib;
} gb_params;

/*
 * Build the device-resident prime table: every prime p <= T with
 * T = max(limit, 65536), ascending, as uint32 (Sec. 3.1: base primes resident
 * and read-only on the device; here generated on the device).  It serves as
 * the sieving primes (p <= isqrt(B) are needed), the Phase-1 candidates
 * (p <= P_max) and the Phase-2 primes.  limit must be <= 2^32 - 1
 * (GB_EINVAL otherwise).  Replaces any earlier table.  Library-owned until
 * gb_release().
 */
gb_status gb_base_primes(uint64_t limit);

/* T of the current table (0 if none) and the number of primes in it. */
uint64_t gb_table_limit(void);
uint64_t gb_table_count(void);

/*
 * Copy table entries [first, first + count) into host memory `out`
 * (count * 4 bytes, caller-owned).  GB_EINVAL when the slice is out of range.
 */
gb_status gb_table_read(uint32_t *out, uint64_t first, uint64_t count);

/*
 * Verify every even n in [A, B] (Sec. 3.1-3.4; Alg. 1 worker loop, with the
 * segment claim made by a device-side atomic counter instead of a host one).
 *   A, B   any u64; normalized as described for gb_result.
 *   P_max  Phase-1 candidate bound, 2 <= P_max <= T (GB_EINVAL / GB_ERANGE).
 *   stream hipStream_t or NULL.
 *   out    caller-owned; out->unresolved / out->unresolved_cap are read as
 *          inputs, every other field is written.
 * Errors: GB_ENOTABLE, GB_EINVAL, GB_ERANGE (T < isqrt(B)), GB_ENOMEM,
 * GB_EHIP, GB_ETRUNC (all counts still exact).
 */
gb_status gb_verify_range(uint64_t A, uint64_t B, uint64_t P_max, void *stream,
                          gb_result *out);

/*
 * Stream-ordered form of gb_verify_range (Sec. 3.1: device-resident work
 * structures, one asynchronous copy of the result at the end).  The whole
 * launch sequence is enqueued on `stream` after the device work of the
 * library's previous call, and ends with copies of the result record into
 * *out, of the status into *status and of the unresolved list into
 * out->unresolved; the call returns once everything is enqueued.  The caller
 * synchronizes `stream` (or an event after it) before reading *out or
 * *status.
 *   out, status, out->unresolved   pinned host memory (hipHostMalloc or
 *          registered); GB_EINVAL otherwise, before anything is enqueued.
 *          out->unresolved / out->unresolved_cap are read at the call.
 *   *status (written by the stream): GB_OK; GB_ETRUNC when the unresolved
 *          list did not fit (counts exact); GB_ENOMEM when more evens were
 *          left open by the probe window than the spill list of this form
 *          holds (the library's current list, at most 65536 entries): *out
 *          is then not valid, and the blocking gb_verify_range (which grows
 *          the list) gives the result.
 * Errors returned by the call itself as gb_verify_range (nothing enqueued).
 * The host waits only when a workspace must grow, or when strike-bitmap
 * descriptors still being uploaded by the previous call would be
 * overwritten.  gb_last_stats() is not updated.
 */
gb_status gb_verify_range_async(uint64_t A, uint64_t B, uint64_t P_max, void *stream,
                                gb_result *out, int32_t *status);

/*
 * Verify k ranges in one persistent launch (batched form): workgroups claim
 * segments of all k ranges from one device queue with an atomic counter (the
 * device-side form of the work pool of Sec. 3.2, Alg. 1), and the whole
 * launch sequence is a captured HIP graph (Sec. 5 names CUDA graphs as future
 * work), re-instantiated only when the batch's shape changes.  Results are
 * identical to k separate gb_verify_range() calls.  The workload it is built
 * and measured for: thousands of uneven intervals per launch, lengths spread
 * over 10^4..10^8 evens and starts over 10^9..2^64 - 2 (tables up to 2^32).
 *   AB     host array of 2k u64: A_0, B_0, A_1, B_1, ...
 *   outs   host array of k gb_result (unresolved buffers as in gb_verify_range).
 * Errors as gb_verify_range; GB_ETRUNC if any list was truncated.
 */
gb_status gb_verify_batch(const uint64_t *AB, uint64_t k, uint64_t P_max,
                          void *stream, gb_result *outs);

/*
 * Verification past 2^64 (paper Sec. 5, future work "pushing past the 64-bit
 * ceiling": 128-bit sieve arithmetic coupled with a Baillie-PSW test).
 * Bounds and n are unsigned 128-bit integers given as (lo, hi) halves.  Up to
 * 2^64 nothing changes: p_min(n) = min { p prime : n - p prime }, and the part
 * of [A, B] below 2^64 goes through gb_verify_range.  From 2^64 on no prime
 * table reaches sqrt(n - p), so primality of q = n - p is decided by the
 * Baillie-PSW test (a strong probable-prime test to base 2 and a strong Lucas
 * test with Selfridge's parameters; no composite passing it is known):
 *     p_min(n) = min { p prime : n - p passes Baillie-PSW }.
 * The range is taken in chunks (gb_set_wide_chunk_log2); each chunk's strike
 * bitmap, sieved by the table primes up to min(T, 2^28) with 128-bit offsets,
 * only removes q with small factors; the survivors are tested in ascending p.  P_max and Phase 2 as in
 * gb_verify_range (Phase 2 tests table primes above P_max by Baillie-PSW).
 *   A, B   any u128 pair (normalized inward to even numbers, A raised to 4;
 *          B = 2^128 - 1 rounds to 2^128 - 2).  At most 2^40 evens at or
 *          above 2^64 per call (GB_EINVAL).  No isqrt(B) condition on the
 *          table limit T beyond the 64-bit part.
 *   out    caller-owned; out->unresolved holds 2 * unresolved_cap u64, the
 *          (lo, hi) halves of each unresolved n in ascending order.
 * Errors as gb_verify_range; GB_ENOMEM when more than 65536 evens at or above
 * 2^64 are left open by P_max (a tiny P_max over a long range).  Blocks until
 * done.  gb_last_stats() describes the part past 2^64: segments = chunks,
 * seg_log2 = log2 of the chunk size, grid = probe blocks, probe_ms = the
 * chunks' sieve and probe kernels.
 */
typedef struct gb_result128 {
    uint64_t A_lo, A_hi, B_lo, B_hi;
    uint64_t P_max;
    uint64_t verified;
    uint64_t max_p;
    uint64_t max_p_n_lo, max_p_n_hi;
    uint64_t checksum;
    uint64_t n_unresolved;
    uint64_t n_failed;
    uint64_t *unresolved;
    uint64_t unresolved_cap;
} gb_result128;

gb_status gb_verify_range_u128(uint64_t A_lo, uint64_t A_hi, uint64_t B_lo, uint64_t B_hi,
                               uint64_t P_max, void *stream, gb_result128 *out);

/*
 * Evens per chunk of a range past 2^64: gb_verify_range_u128 sieves and
 * probes such a range chunk after chunk, each chunk with a strike bitmap of
 * 2^log2 + H bits in device memory (H <= 32768 halo bits below the chunk's
 * first n).  log2 in [12, 30]; 26 by default (an 8 MiB bitmap).  Results do not
 * depend on it; fewer, longer chunks keep more lanes busy at each chunk's end.
 * GB_EINVAL outside the range.  Applies to later calls.
 */
gb_status gb_set_wide_chunk_log2(uint32_t log2);
gb_status gb_get_wide_chunk_log2(uint32_t *log2);

/*
 * Primality of `count` u128 values q[2i] + 2^64 q[2i+1] (DEVICE pointers:
 * 16 * count and count bytes): the deterministic Miller-Rabin test below 2^64
 * and Baillie-PSW above, the tests of gb_verify_range_u128, exported so that
 * they can be checked on their own.
 */
gb_status gb_is_prime_u128(const uint64_t *q, uint64_t count, uint8_t *is_prime, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * verification as gb_verify_range, with every scratch structure of the call
 * (counters, descriptor, segment records, spill and unresolved lists) in a
 * static 64 MiB device array that the library holds on each device from
 * gb_base_primes() until the process ends.  The call makes no hipMalloc,
 * hipFree or other allocating call; the caller passes `out` (and its
 * unresolved buffer, host memory) as for gb_verify_range.
 * Differences from gb_verify_range:
 *  - every prime up to isqrt(B) is sieved inside the segments (no strike
 *    bitmaps), so ranges near 2^64 run slower; results are identical;
 *  - the range may span at most about 2.09 million segments of 2^seg_log2
 *    evens (5.5e11 evens at seg_log2 = 18, 2.2e12 at 20): longer ranges fail
 *    with GB_ENOMEM before anything is enqueued;
 *  - at most 65536 evens may be left open by the probe window (they share
 *    what the segment records leave of the array); more give GB_ENOMEM
 *    after the run (tiny P_max over long ranges), and the result is then not
 *    written;
 *  - gb_last_stats() and gb_last_latencies() are not updated.
 * All calls on one device share its array and leave their contents in it.
 * Calls are serialized by the library lock and each waits for its stream
 * before returning, so two calls of one process never overlap on the array;
 * work that overlapped on one GPU (for instance a kernel of the caller's
 * still writing through an address it kept) would race.
 */
gb_status gb_verify_range_noalloc(uint64_t A, uint64_t B, uint64_t P_max, void *stream,
                                  gb_result *out);

/*
 * Test hook for the failure paths (Sec. 3.4, graceful error handling: an
 * error is reported, the library stays usable).  Makes the next
 * gb_verify_range / gb_verify_batch call fail with GB_EHIP at point `where`:
 * 1 = after validation, before anything is enqueued; 2 = after its kernels
 * are enqueued, before the results are read.  A failed call returns only when
 * none of its work is still in flight, and the next call runs normally.
 * where = 0 clears a pending injection; other values give GB_EINVAL.  No
 * kernel is made to fail: the condition is forced on the host.
 */
gb_status gb_debug_fail_next(uint32_t where);

/* Set / read the launch parameters used by later verify calls.  GB_EINVAL on
 * values outside the documented sets. */
gb_status gb_set_params(const gb_params *p);
gb_status gb_get_params(gb_params *p);

/*
 * Autotuner: time a calibration run of [A, B] (at most 2^36 evens) under each
 * segment size (2^18, 2^19, 2^20 evens), workgroup size (256, 512, 1024) and
 * probe window (2^12, 2^14, 2^16) (and, when isqrt(B) > 2^22, with and without
 * strike bitmaps), keep the fastest as the current parameters
 * and write it to *best (may be NULL).  Results of later calls do not depend
 * on the choice.  Built for full ranges [4, N] as in the paper's Table 1
 * (N = 10^10 and 10^12 here): the calibration range is the top of the range.
 * The choice is cached per device, range magnitude and P_max: a later call
 * for the same key returns it without timing (gb_autotune_cache_clear()
 * forgets every choice).
 */
gb_status gb_autotune(uint64_t A, uint64_t B, uint64_t P_max, void *stream,
                      gb_params *best);

/*
 * Autotuner for the batched form (the calibration-batch tuner): time
 * gb_verify_batch over the k intervals AB[0..2k) (the caller passes a sample
 * of the batches it will run; at most 2^36 evens in all) under each segment
 * size, workgroup size, probe window and strike-bitmap bound (automatic,
 * 2^(seg_log2+3), 2^(seg_log2+5)), keep the fastest as the current
 * parameters and write it to *best (may be NULL).  Results of later calls do
 * not depend on the choice.  GB_EINVAL for an empty or oversized sample.
 * Built for the batched workload described at gb_verify_batch.  Cached like
 * gb_autotune's choice, per device, sample (count, evens, largest top) and
 * P_max.
 */
gb_status gb_autotune_batch(const uint64_t *AB, uint64_t k, uint64_t P_max, void *stream,
                            gb_params *best);

/* Forget every cached autotuner choice (the next gb_autotune /
 * gb_autotune_batch times the candidates again). */
gb_status gb_autotune_cache_clear(void);

/*
 * Deterministic Miller-Rabin primality of `count` u64 values (Sec. 3.4: the
 * first twelve primes as bases; 128-bit products).  q and is_prime are DEVICE
 * pointers (count * 8 and count bytes); is_prime[i] becomes 1 or 0.  This is
 * the primality test of the Phase-2 kernel, exported so that it can be checked
 * on its own.
 */
gb_status gb_is_prime_u64(const uint64_t *q, uint64_t count, uint8_t *is_prime,
                          void *stream);

/*
 * Measurements of the last gb_verify_range / gb_verify_batch call, for the
 * benchmark and the profiles.
 *   probe_ms     duration of the persistent sieve+probe kernel, from HIP events
 *                recorded on the caller's stream around that launch.
 *   total_ms     the whole launch sequence on the stream (events around it).
 *   segments     segments processed; evens = evens in all ranges.
 *   spills       evens left open by the probe window (handled by Phase 2).
 *   grid, wg_size, seg_log2, halo_bits, ncand   the launch shape used.
 *   intervals    number of intervals of the call.
 */
typedef struct gb_stats {
    double probe_ms;
    double total_ms;
    uint64_t segments;
    uint64_t evens;
    uint64_t spills;
    uint32_t grid;
    uint32_t wg_size;
    uint32_t seg_log2;
    uint32_t halo_bits;
    uint32_t ncand;
    uint32_t pad;
    uint64_t intervals;
} gb_stats;

gb_status gb_last_stats(gb_stats *out);

/*
 * Per-interval latency of the last verify call, in milliseconds: from the
 * start of its launch sequence on the device to the moment the interval's
 * last segment finished (device wall clock; 0 for an empty interval).
 * k must equal the number of intervals of that call; ms is caller-owned.
 */
gb_status gb_last_latencies(double *ms, uint64_t k);

/*
 * Served form (built for a Poisson stream of requests, 90 % of them 10^4..10^8
 * evens, the rest 10^9 and 10^10 evens, starts up to 1.8e19, with a 64 GB
 * admission budget; the work pool of Sec. 3.2 turned into a request loop): a
 * request loop with continuous batching.  A server thread
 * admits submitted ranges while active slots and the HBM budget allow, and
 * runs ticks in which every active request contributes its next piece
 * (piece_segments segments) to one batched launch (gb_verify_batch); requests
 * arriving during a tick join the next one.  Pieces of a request are taken in
 * ascending n and merged, so every result equals gb_verify_range of the same
 * range.  The prime table must exist (gb_base_primes) and must not be
 * rebuilt or released while a server is open.
 *
 *   hbm_budget_bytes  admission budget: the sum of the active requests'
 *                     reservations (strike bitmaps and records of one piece)
 *                     stays within it; a
 *                     request whose reservation alone exceeds it is refused
 *                     with GB_ENOMEM at submission.
 *   P_max             candidate bound for every request (as gb_verify_range).
 *   max_active        slots: requests verified concurrently.
 *   piece_segments    segments per request per tick (>= 1).
 *   max_pending       bound on queued, not yet admitted requests (0 = none);
 *                     GB_EBUSY at submission when full.
 */
typedef struct gb_server gb_server;

typedef struct gb_server_config {
    uint64_t hbm_budget_bytes;
    uint64_t P_max;
    uint32_t max_active;
    uint32_t piece_segments;
    uint32_t max_pending;
    uint32_t pad;
} gb_server_config;

/* Counters of a server since it was opened (wall_ms: time since open; busy_ms:
 * time spent inside batched launches). */
typedef struct gb_server_stats {
    uint64_t submitted, admitted, completed, completed_evens, ticks;
    uint64_t active, pending, reserved_bytes;
    double busy_ms, wall_ms;
} gb_server_stats;

/* Open a server on the current table and parameters; *out owns a host thread. */
gb_status gb_server_open(const gb_server_config *cfg, gb_server **out);

/* Queue [A, B] (any u64 pair, normalized as for gb_result); *id (may be NULL)
 * receives the request id.  Non-blocking. */
gb_status gb_server_submit(gb_server *s, uint64_t A, uint64_t B, uint64_t *id);

/* Take one finished request: waits up to wait_ms (0 = do not wait, < 0 = until
 * one finishes); GB_EBUSY if none.  *out as for gb_verify_range (its
 * unresolved buffer is filled, GB_ETRUNC if too small); *latency_ms is the
 * time from submission to completion. */
gb_status gb_server_poll(gb_server *s, int32_t wait_ms, uint64_t *id, gb_result *out,
                         double *latency_ms);

gb_status gb_server_get_stats(gb_server *s, gb_server_stats *out);

/* Finish the active requests, drop the queued ones, stop the thread, free s. */
gb_status gb_server_close(gb_server *s);

/*
 * Device memory allocator of the library (the resident tables and the
 * workspaces of the verify calls and the server).  Paper Sec. 3.1 keeps the
 * base primes and the work structures resident on the device; this hook lets
 * the host framework own that memory, e.g. PyTorch's caching allocator.
 *   alloc(bytes, stream, user)        returns device memory of at least
 *                                     `bytes` bytes, or NULL (the call that
 *                                     needed it then fails with GB_ENOMEM);
 *   free_(ptr, bytes, stream, user)   gives back what alloc returned.
 * The library passes stream = NULL: its buffers are used on any stream, and
 * the device is synchronized before any of them is given back.  Both
 * functions NULL restores hipMalloc / hipFree.  Setting an allocator first
 * releases everything the library holds (as gb_release(), each buffer going
 * back to the allocator that gave it), so it is called before
 * gb_base_primes() and never while a server is open.  The functions may be
 * called from the server's thread.  GB_EINVAL if exactly one is NULL.
 */
typedef void *(*gb_alloc_fn)(size_t bytes, void *stream, void *user);
typedef void (*gb_free_fn)(void *ptr, size_t bytes, void *stream, void *user);
gb_status gb_set_allocator(gb_alloc_fn alloc, gb_free_fn free_, void *user);

/* Free the prime table and every workspace.  Safe to call at any time. */
gb_status gb_release(void);

/* Message for the last failing call on this thread ("" if none). */
const char *gb_last_error(void);

/*
 * Measurement support for the roofline of the segment kernel (paper Sec. 4.3,
 * profiling validation): the LDS read bandwidth of the current device,
 * measured with conflict-free reads of `width` bytes per lane (16: the LDS
 * data path's width; 4: the probe's word reads) by two 1024-thread workgroups
 * per CU, each reading its own 64 KiB of LDS 20000 times over; *bytes_per_s is
 * the whole device's rate.  Runs on the null stream and waits for it;
 * allocates no device memory.  GB_EINVAL for another width or a NULL output,
 * GB_EHIP when a HIP call fails.
 */
gb_status gb_lds_peak(uint32_t width, double *bytes_per_s);

#ifdef __cplusplus
}
#endif

#endif /* GOLDBACH_H */
