// gb_base.hip -- device generation of the resident prime table (all primes
// <= T, T <= 2^32 - 1).  The paper precomputes its small-prime table on the
// host and copies it once (Sec. 3.1); here every step runs on the GPU:
//   1. seed:  one workgroup sieves the odd numbers below 2^16 in LDS;
//   2. count: one workgroup per 2^18 odd numbers sieves its block with the
//             seed primes, counts the survivors and stores the block's bits;
//   3. scan:  exclusive prefix sum of the counts (one workgroup);
//   4. emit:  each workgroup reads its stored bits and writes its primes at
//             its offset, in ascending order.
#include "gb_internal.h"

namespace {

constexpr int kSeedThreads = 1024;
constexpr uint32_t kSeedLimit = 65536;          // seed primes are < 2^16
constexpr int kTabLog2 = 18;                    // odd numbers per table block
constexpr uint32_t kTabBits = 1u << kTabLog2;
constexpr uint32_t kTabWords = kTabBits / 32;
constexpr int kTabThreads = 1024;

// Exclusive prefix sum over a workgroup of NT threads; returns the exclusive
// prefix of `v` and writes the workgroup total to *total.  `scratch` holds
// NT/64 + 1 words.
template <int NT>
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *scratch, uint32_t *total)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off)
            x += y;
    }
    if (lane == 63)
        scratch[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < NT / 64; ++w) {
            const uint32_t t = scratch[w];
            scratch[w] = run;
            run += t;
        }
        scratch[NT / 64] = run;
    }
    __syncthreads();
    const uint32_t res = scratch[wave] + x - v;
    *total = scratch[NT / 64];
    __syncthreads();
    return res;
}

__device__ bool small_is_prime(uint32_t p)
{
    if (p < 2)
        return false;
    for (uint32_t d = 2; d * d <= p; ++d)
        if (p % d == 0)
            return false;
    return true;
}

// Seed table: primes below 2^16, primes[0] = 2.  Bit b of the LDS bitset is
// the odd number 2b + 1.
__global__ __launch_bounds__(kSeedThreads) void seed_kernel(uint32_t *seed, uint32_t *nseed)
{
    __shared__ uint32_t bits[kSeedLimit / 64];
    __shared__ uint32_t scratch[kSeedThreads / 64 + 1];
    const uint32_t t = threadIdx.x;
    bits[t] = 0xFFFFFFFFu;
    __syncthreads();
    if (t == 0)
        atomicAnd(&bits[0], ~1u);  // 1 is not prime
    // odd p < 256 strike their odd multiples from p^2 (p^2 < 2^16 needs
    // p <= 255), the whole workgroup taking each prime's multiples in turn
    for (uint32_t p = 3; p < 256; p += 2) {
        if (!small_is_prime(p))
            continue;
        for (uint32_t m = p * p + 2 * p * t; m < kSeedLimit; m += 2 * p * kSeedThreads) {
            const uint32_t b = m >> 1;
            atomicAnd(&bits[b >> 5], ~(1u << (b & 31)));
        }
    }
    __syncthreads();
    const uint32_t w = bits[t];
    uint32_t total;
    const uint32_t off = block_excl_scan<kSeedThreads>(__popc(w), scratch, &total);
    uint32_t rank = 0;
    for (uint32_t m = w; m; m &= m - 1, ++rank)
        seed[1 + off + rank] = 2 * (32 * t + (__ffs(m) - 1)) + 1;
    if (t == 0) {
        seed[0] = 2;
        *nseed = total + 1;
    }
}

// Seed primes at least this large strike a block fewer than 128 times: one
// thread walks all multiples of such a prime; smaller ones are struck by the
// whole workgroup, thread t taking multiples t, t + NT, ...
constexpr uint32_t kTabSplit = kTabBits / 128;

// Sieve table block g (odd numbers 2b + 1 for b in [g*2^18, (g+1)*2^18)) into
// `bits` with the odd seed primes p, p^2 <= top; bits for numbers above T are
// cleared.  The first multiple of each prime is found once, by one thread,
// and kept in `first` (bit index, or nbits when the prime does not reach the
// block).  Returns after a barrier.
__device__ void sieve_table_block(uint32_t *bits, uint32_t *first, const uint32_t *seed,
                                  uint32_t nseed, uint64_t T, uint32_t g)
{
    const uint32_t t = threadIdx.x;
    const uint64_t b0 = (uint64_t)g * kTabBits;
    const uint64_t lo = 2 * b0 + 1;                 // first odd number of the block (< 2^32)
    uint64_t hi = lo + 2 * (uint64_t)(kTabBits - 1);
    const uint64_t Todd = (T & 1) ? T : T - 1;
    if (hi > Todd)
        hi = Todd;
    const uint32_t nbits = (uint32_t)((hi - lo) / 2 + 1);
    for (uint32_t w = t; w < kTabWords; w += kTabThreads) {
        uint32_t v = 0xFFFFFFFFu;
        const uint32_t f = 32 * w;
        if (f >= nbits)
            v = 0;
        else if (nbits - f < 32)
            v = (1u << (nbits - f)) - 1;
        bits[w] = v;
    }
    // first multiple of each odd seed prime: max(p^2, the first odd multiple
    // >= lo) (lo < 2^32, p < 2^16)
    for (uint32_t i = 1 + t; i < nseed; i += kTabThreads) {
        const uint32_t p = seed[i];
        uint32_t j = nbits;
        if ((uint64_t)p * p <= hi) {
            uint64_t start = (uint64_t)p * p;
            if (start < lo) {
                uint64_t m = lo + (p - (uint32_t)lo % p) % p;   // first multiple >= lo
                if ((m & 1) == 0)
                    m += p;
                start = m;
            }
            if (start <= hi)
                j = (uint32_t)((start - lo) >> 1);
        }
        first[i] = j;
    }
    __syncthreads();
    if (g == 0 && t == 0)
        atomicAnd(&bits[0], ~1u);  // 1 is not prime
    for (uint32_t i = 1; i < nseed; ++i) {
        const uint32_t p = seed[i];
        if (p >= kTabSplit)
            break;
        const uint32_t j0 = first[i];
        for (uint32_t j = j0 + t * p; j < nbits; j += kTabThreads * p)
            atomicAnd(&bits[j >> 5], ~(1u << (j & 31)));
    }
    for (uint32_t i = 1 + t; i < nseed; i += kTabThreads) {
        const uint32_t p = seed[i];
        if (p < kTabSplit)
            continue;
        for (uint32_t j = first[i]; j < nbits; j += p)
            atomicAnd(&bits[j >> 5], ~(1u << (j & 31)));
    }
    __syncthreads();
}

__global__ __launch_bounds__(kTabThreads) void table_count_kernel(const uint32_t *seed,
                                                                  const uint32_t *nseed, uint64_t T,
                                                                  uint32_t *counts, uint32_t *stash)
{
    __shared__ uint32_t bits[kTabWords];
    __shared__ uint32_t first[kSeedLimit / 8];   // at most 6542 odd seed primes
    __shared__ uint32_t scratch[kTabThreads / 64 + 1];
    const uint32_t g = blockIdx.x;
    sieve_table_block(bits, first, seed, *nseed, T, g);
    uint32_t c = 0;
    uint32_t *out = stash + (uint64_t)g * kTabWords;
    for (uint32_t w = threadIdx.x; w < kTabWords; w += kTabThreads) {
        const uint32_t v = bits[w];
        out[w] = v;
        c += __popc(v);
    }
    uint32_t total;
    block_excl_scan<kTabThreads>(c, scratch, &total);
    if (threadIdx.x == 0)
        counts[g] = total;
}

// In-place exclusive scan of nsegs counts; *total = pi(T) - 1 (odd primes).
__global__ __launch_bounds__(1024) void table_scan_kernel(uint32_t *counts, uint32_t nsegs,
                                                         uint64_t *total)
{
    __shared__ uint32_t scratch[1024 / 64 + 1];
    uint64_t run = 0;
    for (uint32_t base = 0; base < nsegs; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < nsegs ? counts[i] : 0;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<1024>(v, scratch, &tot);
        if (i < nsegs)
            counts[i] = (uint32_t)(run + ex);
        run += tot;
    }
    if (threadIdx.x == 0)
        *total = run;
}

__global__ __launch_bounds__(kTabThreads) void table_emit_kernel(const uint32_t *stash,
                                                                 const uint32_t *offsets,
                                                                 uint32_t *primes)
{
    __shared__ uint32_t scratch[kTabThreads / 64 + 1];
    const uint32_t g = blockIdx.x;
    constexpr uint32_t per = kTabWords / kTabThreads;   // consecutive words per thread
    const uint32_t w0 = threadIdx.x * per;
    const uint32_t *in = stash + (uint64_t)g * kTabWords + w0;
    uint32_t v[per];
    uint32_t c = 0;
#pragma unroll
    for (uint32_t k = 0; k < per; ++k) {
        v[k] = in[k];
        c += __popc(v[k]);
    }
    uint32_t total;
    uint32_t pos = block_excl_scan<kTabThreads>(c, scratch, &total);
    pos += 1 + offsets[g];  // primes[0] = 2
    if (g == 0 && threadIdx.x == 0)
        primes[0] = 2;
    const uint64_t b0 = (uint64_t)g * kTabBits;
#pragma unroll
    for (uint32_t k = 0; k < per; ++k)
        for (uint32_t m = v[k]; m; m &= m - 1)
            primes[pos++] = (uint32_t)(2 * (b0 + 32 * (w0 + k) + (__ffs(m) - 1)) + 1);
}

}  // namespace

uint32_t gb_table_seg_log2() { return kTabLog2; }
uint32_t gb_table_block_words() { return kTabWords; }

hipError_t gb_launch_seed(uint32_t *seed, uint32_t *nseed, hipStream_t s)
{
    hipLaunchKernelGGL(seed_kernel, dim3(1), dim3(kSeedThreads), 0, s, seed, nseed);
    return hipGetLastError();
}

hipError_t gb_launch_table_count(const uint32_t *seed, const uint32_t *nseed, uint64_t T,
                                 uint32_t nsegs, uint32_t *counts, uint32_t *stash, hipStream_t s)
{
    hipLaunchKernelGGL(table_count_kernel, dim3(nsegs), dim3(kTabThreads), 0, s, seed, nseed, T,
                       counts, stash);
    return hipGetLastError();
}

hipError_t gb_launch_table_scan(uint32_t *counts, uint32_t nsegs, uint64_t *total, hipStream_t s)
{
    hipLaunchKernelGGL(table_scan_kernel, dim3(1), dim3(1024), 0, s, counts, nsegs, total);
    return hipGetLastError();
}

hipError_t gb_launch_table_emit(const uint32_t *stash, uint32_t nsegs, const uint32_t *offsets,
                                uint32_t *primes, hipStream_t s)
{
    hipLaunchKernelGGL(table_emit_kernel, dim3(nsegs), dim3(kTabThreads), 0, s, stash, offsets,
                       primes);
    return hipGetLastError();
}
