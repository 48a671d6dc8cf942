// gb_phase2.hip -- Phase 2 on the device and the final reductions.
//
// Phase 2 (Sec. 3.3): an even n that no candidate of the probe window resolves
// is finished here.  The paper copies such n back to the host and resolves
// them there with a prime table and a 128-bit Miller-Rabin test; here the
// kernel stays on the GPU, so there is no host round trip and the pipeline can
// be captured as a whole.  One wave takes one spilled n and tests 64 table
// primes p at a time, ascending from the first prime above the probe window,
// with q = n - p checked by the deterministic Miller-Rabin test (Sec. 3.4);
// the lowest lane with a prime q gives p_min.  The search stops at
// p > min(T, n/2).
//
// The reduction (Sec. 3.1 device reduction, generalized from a count of
// unverified n to the full aggregates) folds per-segment records and Phase-2
// results per interval; every operation in it (wrapping sums, max with the
// smallest-n tie-break, counts) is order-independent, so the result does not
// depend on which workgroup claimed which segment.
#include "gb_arith.h"
#include "gb_internal.h"
#include "goldbach.h"

namespace {

constexpr int kRedThreads = 256;

__global__ __launch_bounds__(256) void phase2_kernel(const uint32_t *__restrict__ primes,
                                                     uint64_t nprimes, uint64_t first_idx,
                                                     GbSpill *spill, uint64_t cap,
                                                     const GbCounters *ctr)
{
    const unsigned long long total = ctr->spills;
    const uint64_t count = total < cap ? total : cap;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t wid = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t e = wid; e < count; e += nw) {
        const uint64_t n = spill[e].n;
        const uint64_t half = n >> 1;
        uint32_t found = 0;
        for (uint64_t base = first_idx; base < nprimes; base += 64) {
            const uint64_t idx = base + lane;
            const uint32_t p = idx < nprimes ? primes[idx] : 0xFFFFFFFFu;
            const bool valid = idx < nprimes && p <= half;
            const unsigned long long vm = __ballot(valid);
            if (vm == 0)
                break;
            const bool isp = valid && gb_is_prime_u64(n - p);
            const unsigned long long pm = __ballot(isp);
            if (pm) {
                found = __shfl(p, __ffsll(pm) - 1, 64);
                break;
            }
            if (vm != ~0ull)
                break;  // valid lanes form a prefix: the table or n/2 ended here
        }
        if (lane == 0)
            spill[e].p = found;
    }
}

__device__ __forceinline__ void max_merge(uint64_t &bp, uint64_t &bn, uint64_t p, uint64_t n)
{
    if (p > bp || (p == bp && n < bn)) {
        bp = p;
        bn = n;
    }
}

__device__ __forceinline__ bool unresolved(const GbSpill &s, uint64_t P_max)
{
    return s.p == 0 || s.p > P_max;
}

__global__ __launch_bounds__(kRedThreads) void reduce_kernel(const GbInterval *iv,
                                                              const GbSegRecord *rec,
                                                              const GbSpill *spill, uint64_t cap,
                                                              const GbCounters *ctr, uint64_t P_max,
                                                              GbIvResult *res)
{
    __shared__ uint64_t sh[6][kRedThreads / 64];
    const uint32_t x = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const GbInterval I = iv[x];
    uint64_t s = 0, c = 0, bp = 0, bn = 0, failed = 0, unres = 0, before = 0;
    for (uint64_t g = I.seg_first + tid; g < I.seg_first + I.nseg; g += kRedThreads) {
        const GbSegRecord r = rec[g];
        s += r.checksum;
        c += r.verified;
        if (r.max_p)
            max_merge(bp, bn, r.max_p, r.max_n);
    }
    const unsigned long long total = ctr->spills;
    const uint64_t count = total < cap ? total : cap;
    for (uint64_t e = tid; e < count; e += kRedThreads) {
        const GbSpill sp = spill[e];
        const bool un = unresolved(sp, P_max);
        if (sp.iv < x && un)
            ++before;
        if (sp.iv != x)
            continue;
        if (sp.p) {
            ++c;
            s += sp.p;
            max_merge(bp, bn, sp.p, sp.n);
        } else {
            ++failed;
        }
        if (un)
            ++unres;
    }
    const uint32_t lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        c += __shfl_xor(c, off, 64);
        failed += __shfl_xor(failed, off, 64);
        unres += __shfl_xor(unres, off, 64);
        before += __shfl_xor(before, off, 64);
        const uint64_t op = __shfl_xor(bp, off, 64);
        const uint64_t on = __shfl_xor(bn, off, 64);
        if (op)
            max_merge(bp, bn, op, on);
    }
    __shared__ uint64_t shp[kRedThreads / 64], shn[kRedThreads / 64];
    if (lane == 0) {
        sh[0][wave] = s;
        sh[1][wave] = c;
        sh[2][wave] = failed;
        sh[3][wave] = unres;
        sh[4][wave] = before;
        shp[wave] = bp;
        shn[wave] = bn;
    }
    __syncthreads();
    if (tid == 0) {
        GbIvResult r = {};
        uint64_t p = 0, n = 0;
        for (int w = 0; w < kRedThreads / 64; ++w) {
            r.checksum += sh[0][w];
            r.verified += sh[1][w];
            r.n_failed += sh[2][w];
            r.n_unresolved += sh[3][w];
            r.unres_first += sh[4][w];
            if (shp[w])
                max_merge(p, n, shp[w], shn[w]);
        }
        r.max_p = p;
        r.max_p_n = p ? n : 0;
        res[x] = r;
    }
}

// Unresolved n in (interval, n) order: each unresolved entry's position is the
// number of unresolved entries that precede it in that order (a counting rank;
// n are distinct within an interval).
__global__ __launch_bounds__(256) void unres_emit_kernel(const GbSpill *spill, uint64_t cap,
                                                         const GbCounters *ctr, uint64_t P_max,
                                                         uint64_t *out)
{
    const unsigned long long total = ctr->spills;
    const uint64_t count = total < cap ? total : cap;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) {
        const GbSpill me = spill[e];
        if (!unresolved(me, P_max))
            continue;
        uint64_t rank = 0;
        for (uint64_t f = 0; f < count; ++f) {
            const GbSpill o = spill[f];
            if (unresolved(o, P_max) && (o.iv < me.iv || (o.iv == me.iv && o.n < me.n)))
                ++rank;
        }
        out[rank] = me.n;
    }
}

// Unresolved n in (interval, n) order for long lists: one bit per even of
// every interval (interval i's bits start at word woff[i]), set for each
// unresolved spill; a scan of the words' popcounts gives each bit its
// position.  Cost: linear in the evens of the launch and in the spills.
constexpr uint32_t kEmitWordsPerBlock = 4096;   // 4 words per thread, 1024 threads

__global__ __launch_bounds__(256) void emit_zero_kernel(uint32_t *bitmap, uint64_t words)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
        bitmap[i] = 0;
}

__global__ __launch_bounds__(256) void emit_mark_kernel(const GbSpill *spill, uint64_t cap,
                                                        const GbCounters *ctr, uint64_t P_max,
                                                        const GbInterval *iv,
                                                        const uint64_t *woff, uint32_t *bitmap)
{
    const unsigned long long total = ctr->spills;
    const uint64_t count = total < cap ? total : cap;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) {
        const GbSpill sp = spill[e];
        if (!unresolved(sp, P_max))
            continue;
        const uint64_t idx = (sp.n - iv[sp.iv].A) >> 1;   // the even's index in its interval
        atomicOr(&bitmap[woff[sp.iv] + (idx >> 5)], 1u << (idx & 31));
    }
}

// Per block of kEmitWordsPerBlock words: the number of set bits.
__global__ __launch_bounds__(1024) void emit_count_kernel(const uint32_t *bitmap, uint64_t words,
                                                         uint64_t *blocksum)
{
    __shared__ uint64_t sh[16];
    const uint64_t w0 = (uint64_t)blockIdx.x * kEmitWordsPerBlock;
    uint64_t c = 0;
    for (uint32_t t = threadIdx.x; t < kEmitWordsPerBlock; t += 1024)
        if (w0 + t < words)
            c += __popc(bitmap[w0 + t]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int i = 0; i < 16; ++i)
            s += sh[i];
        blocksum[blockIdx.x] = s;
    }
}

// Exclusive scan of the block sums in place (one workgroup).
__global__ __launch_bounds__(1024) void emit_scan_kernel(uint64_t *blocksum, uint64_t nblocks)
{
    __shared__ uint64_t sh[1024];
    uint64_t run = 0;
    for (uint64_t base = 0; base < nblocks; base += 1024) {
        const uint64_t i = base + threadIdx.x;
        const uint64_t v = i < nblocks ? blocksum[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (uint32_t off = 1; off < 1024; off <<= 1) {
            const uint64_t y = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < nblocks)
            blocksum[i] = run + sh[threadIdx.x] - v;
        run += sh[1023];
        __syncthreads();
    }
}

// Emit: thread t of block b holds words 4t..4t+3 of the block; the position
// of a bit is the block's offset + the set bits before it in the block.
__global__ __launch_bounds__(1024) void emit_write_kernel(const uint32_t *bitmap, uint64_t words,
                                                         const uint64_t *blockoff,
                                                         const GbInterval *iv, uint32_t k,
                                                         const uint64_t *woff, uint64_t *out)
{
    __shared__ uint64_t sh[1024];
    const uint64_t w0 = (uint64_t)blockIdx.x * kEmitWordsPerBlock + 4ull * threadIdx.x;
    uint32_t v[4];
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        v[q] = w0 + q < words ? bitmap[w0 + q] : 0u;
        c += __popc(v[q]);
    }
    sh[threadIdx.x] = c;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint64_t y = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += y;
        __syncthreads();
    }
    uint64_t pos = blockoff[blockIdx.x] + sh[threadIdx.x] - c;
    if (c == 0)
        return;
    // the interval of word w0: last i with woff[i] <= w0
    uint32_t lo = 0, hi = k - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (woff[mid] <= w0)
            lo = mid;
        else
            hi = mid - 1;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint64_t w = w0 + q;
        while (lo + 1 < k && woff[lo + 1] <= w)
            ++lo;
        for (uint32_t m = v[q]; m; m &= m - 1) {
            const uint64_t idx = (w - woff[lo]) * 32 + (uint32_t)(__ffs(m) - 1);
            out[pos++] = iv[lo].A + 2 * idx;
        }
    }
}

__global__ __launch_bounds__(256) void is_prime_kernel(const uint64_t *q, uint64_t count,
                                                       uint8_t *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        out[i] = gb_is_prime_u64(q[i]) ? 1 : 0;
}

// The stream-ordered end of gb_verify_range_async: the caller's gb_result
// image and status word, built on the device from the reduced result and the
// launch counters, for one copy to the caller's pinned memory.
__global__ void finalize_kernel(const GbIvResult *res, const GbCounters *ctr, uint64_t spill_cap,
                                uint64_t A, uint64_t B, uint64_t P_max, uint64_t *unres,
                                uint64_t cap, gb_result *img, int32_t *status)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    const GbIvResult r = *res;
    gb_result o;
    o.A = A;
    o.B = B;
    o.P_max = P_max;
    o.verified = r.verified;
    o.max_p = r.max_p;
    o.max_p_n = r.max_p_n;
    o.checksum = r.checksum;
    o.n_unresolved = r.n_unresolved;
    o.n_failed = r.n_failed;
    o.unresolved = unres;
    o.unresolved_cap = cap;
    *img = o;
    *status = ctr->spills > spill_cap ? GB_ENOMEM : (r.n_unresolved > cap ? GB_ETRUNC : GB_OK);
}

}  // namespace

hipError_t gb_launch_finalize(const GbIvResult *res, const GbCounters *ctr, uint64_t spill_cap,
                              uint64_t A, uint64_t B, uint64_t P_max, uint64_t *unres,
                              uint64_t cap, void *img, hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(64), 0, s, res, ctr, spill_cap, A, B, P_max,
                       unres, cap, (gb_result *)img,
                       (int32_t *)((char *)img + kFinalizeStatusOffset));
    return hipGetLastError();
}

hipError_t gb_launch_phase2(const uint32_t *primes, uint64_t nprimes, uint64_t first_idx,
                            GbSpill *spill, uint64_t spill_cap, const GbCounters *ctr,
                            uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(phase2_kernel, dim3(grid), dim3(256), 0, s, primes, nprimes, first_idx,
                       spill, spill_cap, ctr);
    return hipGetLastError();
}

hipError_t gb_launch_reduce(const GbInterval *iv, uint32_t k, const GbSegRecord *rec,
                            const GbSpill *spill, uint64_t spill_cap, const GbCounters *ctr,
                            uint64_t P_max, GbIvResult *res, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(k), dim3(kRedThreads), 0, s, iv, rec, spill, spill_cap,
                       ctr, P_max, res);
    return hipGetLastError();
}

hipError_t gb_launch_unres_emit(const GbSpill *spill, uint64_t spill_cap, const GbCounters *ctr,
                                uint64_t P_max, uint64_t *out, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(unres_emit_kernel, dim3(grid), dim3(256), 0, s, spill, spill_cap, ctr,
                       P_max, out);
    return hipGetLastError();
}

hipError_t gb_launch_unres_bitmap(const GbSpill *spill, uint64_t spill_cap, const GbCounters *ctr,
                                  uint64_t P_max, const GbInterval *iv, uint32_t k,
                                  const uint64_t *woff, uint64_t words, uint32_t *bitmap,
                                  uint64_t *blocksum, uint64_t *out, uint32_t grid, hipStream_t s)
{
    const uint64_t nb = (words + kEmitWordsPerBlock - 1) / kEmitWordsPerBlock;
    if (nb == 0)
        return hipSuccess;
    hipLaunchKernelGGL(emit_zero_kernel, dim3(grid), dim3(256), 0, s, bitmap, words);
    hipLaunchKernelGGL(emit_mark_kernel, dim3(grid), dim3(256), 0, s, spill, spill_cap, ctr, P_max,
                       iv, woff, bitmap);
    hipLaunchKernelGGL(emit_count_kernel, dim3((uint32_t)nb), dim3(1024), 0, s, bitmap, words,
                       blocksum);
    hipLaunchKernelGGL(emit_scan_kernel, dim3(1), dim3(1024), 0, s, blocksum, nb);
    hipLaunchKernelGGL(emit_write_kernel, dim3((uint32_t)nb), dim3(1024), 0, s, bitmap, words,
                       blocksum, iv, k, woff, out);
    return hipGetLastError();
}

uint64_t gb_unres_bitmap_blocks(uint64_t words)
{
    return (words + kEmitWordsPerBlock - 1) / kEmitWordsPerBlock;
}

hipError_t gb_launch_is_prime(const uint64_t *q, uint64_t count, uint8_t *out, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    uint64_t blocks = (count + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    hipLaunchKernelGGL(is_prime_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, q, count, out);
    return hipGetLastError();
}
