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
 *    enqueue their kernels on that stream and wait for it before returning,
 *    so results are in the caller's host structures on return.
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
 *   seg_log2   log2 of the odd numbers held per segment bitset in LDS:
 *              18, 19 or 20 (32, 64 or 128 KB of LDS per workgroup).
 *   wg_size    threads per workgroup: 256, 512 or 1024.
 *   window     probe window: candidates p <= min(P_max, window) are tested in
 *              LDS by the probe; candidates window < p <= P_max are tested by
 *              the Phase-2 kernel for the (rare) n the window leaves open.
 *              0 means window = P_max.  Must be 0 or in [3, 65536].
 *   wg_per_cu  workgroups per compute unit in the persistent grid; 0 = the
 *              maximum that LDS allows.
 */
typedef struct gb_params {
    uint32_t seg_log2;
    uint32_t wg_size;
    uint32_t window;
    uint32_t wg_per_cu;
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
 * Verify k ranges in one persistent launch (batched form): workgroups claim
 * segments of all k ranges from one device queue with an atomic counter.
 * Results are identical to k separate gb_verify_range() calls.
 *   AB     host array of 2k u64: A_0, B_0, A_1, B_1, ...
 *   outs   host array of k gb_result (unresolved buffers as in gb_verify_range).
 * Errors as gb_verify_range; GB_ETRUNC if any list was truncated.
 */
gb_status gb_verify_batch(const uint64_t *AB, uint64_t k, uint64_t P_max,
                          void *stream, gb_result *outs);

/* Set / read the launch parameters used by later verify calls.  GB_EINVAL on
 * values outside the documented sets. */
gb_status gb_set_params(const gb_params *p);
gb_status gb_get_params(gb_params *p);

/*
 * Time a calibration run of [A, B] (at most 2^31 evens) under each supported
 * parameter set, keep the fastest as the current parameters and write it to
 * *best (may be NULL).  Results of later calls do not depend on the choice.
 */
gb_status gb_autotune(uint64_t A, uint64_t B, uint64_t P_max, void *stream,
                      gb_params *best);

/*
 * Deterministic Miller-Rabin primality of `count` u64 values (Sec. 3.4: the
 * first twelve primes as bases; 128-bit products).  q and is_prime are DEVICE
 * pointers (count * 8 and count bytes); is_prime[i] becomes 1 or 0.  This is
 * the primality test of the Phase-2 kernel, exported so that it can be checked
 * on its own.
 */
gb_status gb_is_prime_u64(const uint64_t *q, uint64_t count, uint8_t *is_prime,
                          void *stream);

/* Free the prime table and every workspace.  Safe to call at any time. */
gb_status gb_release(void);

/* Message for the last failing call on this thread ("" if none). */
const char *gb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GOLDBACH_H */
