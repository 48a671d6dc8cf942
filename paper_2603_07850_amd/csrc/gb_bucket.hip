// gb_bucket.hip -- strike bitmaps for the primes above the bucket bound.
//
// A prime p much larger than a segment window strikes a window at most once,
// so computing its first multiple in every segment (one 64-by-32-bit
// remainder per prime per segment) costs far more than the strikes
// themselves; near 2^64 there are 2*10^8 such primes per segment.  Here the
// remainder is taken once per chunk (a run of consecutive segments of one
// interval) and prime, the prime's multiples are walked across the chunk, and
// each strike sets its window bit in the strike bitmap of the segment that
// owns it -- and of the previous segment too when it falls in the halo the
// two windows share -- with one non-returning atomic OR.  Strikes of one
// segment land on words spread over its window, so they do not queue on one
// address.  The segment kernel folds its bitmap into the LDS window.
//
// Work is cut into items (prime, chunk): a task pairs the primes of one band
// (2^b, 2^(b+1)] with a group of consecutive chunks, and a thread loads each
// of its primes and its reciprocal once for the whole group.  Every offset is
// relative to the chunk's window start and bounded by the chunk's last odd
// number, so no absolute value beyond it is formed (the overflow guards of the
// paper's Sec. 3.4).
#include "gb_arith.h"
#include "gb_internal.h"

namespace {

// Set window bit off of segment g in its strike bitmap, stored by class like
// the LDS window: bit off / 3 of class array off mod 3.
__device__ __forceinline__ void strike(const GbBucketArgs &a, uint64_t g, uint32_t off)
{
    const uint64_t rel = g - a.seg_base;
    const uint32_t i = __umulhi(off, 0xAAAAAAABu) >> 1;  // off / 3
    const uint32_t t = off - 3 * i;
    atomicOr(&a.bitmap[rel * a.words + t * a.wcu + (i >> 5)], 1u << (i & 31));
}

// Tasks and chunks are read-only here: read through the constant address
// space, with uniform indices, they load as scalars.
typedef const __attribute__((address_space(4))) GbFillTask *ctask_t;
typedef const __attribute__((address_space(4))) GbChunk *cchunk_t;

__device__ void fill_tile(const GbBucketArgs &a, uint64_t tile)
{
    const ctask_t task = (ctask_t)a.task;
    const cchunk_t chunk = (cchunk_t)a.chunk;
    uint32_t lo = 0, hi = a.ntask - 1;   // last task whose first tile <= tile
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (task[mid].tile_first <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    const uint64_t t_first = task[lo].tile_first;
    const uint32_t c_first = task[lo].chunk_first;
    const uint32_t c_n = task[lo].nchunk;
    const uint32_t p_first = task[lo].p_first;
    const uint32_t np = task[lo].np;
    const uint32_t E = 1u << a.log2e;
    const uint32_t emask = E - 1;
    constexpr uint32_t PB = kFillThreads * kFillPerThread;
    const uint32_t pb = (uint32_t)(tile - t_first);
    for (uint32_t m = 0; m < kFillPerThread; ++m) {
        const uint32_t pi = pb * PB + threadIdx.x + m * kFillThreads;
        if (pi >= np)
            break;
        const uint64_t idx = (uint64_t)p_first + pi;
        const uint32_t p = a.primes[idx];
        const double pd = (double)p;
        const double inv = gb_recip(p);
        const double half = (double)(p >> 1);
        const uint32_t pm3 = p % 3;
        for (uint32_t cc = 0; cc < c_n; ++cc) {
            const uint32_t ci = c_first + cc;
            if (idx >= chunk[ci].p_root)
                continue;
            const uint64_t dmax = chunk[ci].dmax;
            // first odd multiple of p at or above Q0 = 2h + 1, as a window bit
            uint64_t d = gb_first_odd_multiple(chunk[ci].hh, chunk[ci].hl, pd, inv, half);
            // strikes start at p^2: only a prime above isqrt(Q0) can have its
            // square past the chunk's first odd number
            if (p > chunk[ci].sqrt_q0) {
                const uint64_t dsq = ((uint64_t)p * p - chunk[ci].Q0) >> 1;
                if (dsq > d)
                    d = dsq;
            }
            if (d > dmax)
                continue;
            const uint64_t seg_first = chunk[ci].seg_first;
            const uint32_t nseg = chunk[ci].nseg;
            // the odd number Q0 + 2d is a multiple of 3 when d = Q0 (mod 3):
            // the window does not store that class, so those bits are not struck
            const uint32_t q0m3 = chunk[ci].q0m3;
            uint32_t dm3 = (uint32_t)(d % 3);
            for (; d <= dmax; d += p) {
                if (dm3 != q0m3) {
                    const uint64_t sg = d >> a.log2e;
                    const uint32_t off = (uint32_t)d & emask;
                    if (sg < nseg)
                        strike(a, seg_first + sg, off);
                    if (off < a.H && sg >= 1 && sg - 1 < nseg)
                        strike(a, seg_first + sg - 1, off + E);
                }
                dm3 += pm3;
                dm3 = dm3 >= 3 ? dm3 - 3 : dm3;
            }
        }
    }
}

// Grid-stride over the round's tiles (the grid is capped well below the
// 2^32 work-item limit of one launch).
__global__ __launch_bounds__(kFillThreads) void bucket_fill_kernel(GbBucketArgs a)
{
    for (uint64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x)
        fill_tile(a, tile);
}

__global__ void bucket_reset_kernel(uint32_t *bitmap, uint64_t words)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
        bitmap[i] = 0;
}

// p_root of each chunk: the number of table primes <= isqrt(its top).
__global__ void chunk_roots_kernel(const uint32_t *primes, uint64_t nprimes, GbChunk *chunks,
                                   uint64_t nchunk)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nchunk; c += stride) {
        const uint32_t root = gb_isqrt64(chunks[c].Q0 + 2 * chunks[c].dmax);
        uint64_t lo = 0, hi = nprimes;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (primes[mid] <= root)
                lo = mid + 1;
            else
                hi = mid;
        }
        chunks[c].p_root = (uint32_t)lo;
    }
}

}  // namespace

hipError_t gb_launch_bucket_reset(uint32_t *bitmap, uint64_t words, hipStream_t s)
{
    uint64_t blocks = (words + 255) / 256;
    if (blocks < 1)
        blocks = 1;
    if (blocks > 16384)
        blocks = 16384;
    hipLaunchKernelGGL(bucket_reset_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, bitmap, words);
    return hipGetLastError();
}

hipError_t gb_launch_bucket_fill(const GbBucketArgs &a, uint32_t grid, hipStream_t s)
{
    if (grid == 0)
        return hipSuccess;
    hipLaunchKernelGGL(bucket_fill_kernel, dim3(grid), dim3(kFillThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t gb_launch_chunk_roots(const uint32_t *primes, uint64_t nprimes, GbChunk *chunks,
                                 uint64_t nchunk, hipStream_t s)
{
    if (nchunk == 0)
        return hipSuccess;
    uint64_t blocks = (nchunk + 255) / 256;
    if (blocks > 1024)
        blocks = 1024;
    hipLaunchKernelGGL(chunk_roots_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, primes, nprimes,
                       chunks, nchunk);
    return hipGetLastError();
}
