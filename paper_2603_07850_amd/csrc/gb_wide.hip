// gb_wide.hip -- verification past 2^64 (the paper's future-work direction
// of Sec. 5: 128-bit sieve arithmetic coupled with a Baillie-PSW test).
//
// Beyond 2^64 the table of primes up to 2^32 no longer reaches sqrt(q), so the
// segment window is a pre-filter: a persistent kernel claims segments of
// 2^16 evens, strikes from the LDS window every odd q = n - p with a prime
// factor up to the sieve bound S (the table primes up to min(T, 2^28); the
// window start is a 128-bit number, so each prime's first multiple comes from
// a 128-by-32 remainder), and then decides the survivors, in ascending p for
// each n, with the Baillie-PSW test.  The first survivor that passes gives
// p_min(n).  Survivors are prime with probability about 0.9, so an even costs
// about one Baillie-PSW test, and a wave keeps all its lanes busy by handing
// a finished lane the next even of its share (no lockstep over a block).
// Evens that no candidate p <= P_max resolves are spilled to the wide
// Phase-2 kernel, which continues with the table primes above P_max.
#include "gb_wide.h"

namespace {

constexpr uint32_t kE = 1u << kWideLog2E;
// window words: E evens plus the halo (at most 32768 bits) and one spare word
constexpr uint32_t kWideWords = (kE + 32768) / 32 + 2;

__device__ __forceinline__ void max_merge_w(uint64_t &bp, u128w &bn, uint64_t p, u128w n)
{
    if (p > bp || (p == bp && w_lt(n, bn))) {
        bp = p;
        bn = n;
    }
}

__global__ __launch_bounds__(kWideThreads) void wide_sieve_probe_kernel(GbWideArgs a)
{
    constexpr uint32_t NWAVE = kWideThreads / 64;
    __shared__ uint32_t bits[kWideWords];   // bit b: odd q_lo + 2b has a factor <= S
    __shared__ unsigned long long sh_seg;
    __shared__ uint64_t red_sum[NWAVE], red_cnt[NWAVE], red_p[NWAVE], red_nl[NWAVE],
        red_nh[NWAVE], red_sp[NWAVE];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t H = a.H;

    for (;;) {
        if (tid == 0)
            sh_seg = atomicAdd(&a.ctr[0], 1ull);
        __syncthreads();
        const uint64_t seg = sh_seg;
        if (seg >= a.nsegs)
            break;
        const uint64_t rem = a.nE - (uint64_t)kE * seg;
        const uint32_t cnt = (uint32_t)(rem < kE ? rem : kE);
        // n0 = A + 2 E seg; q_lo = n0 - 1 - 2H (no wrap: n0 >= 2^64)
        const u128w n0 = w_add64(a.A, 2ull * kE * seg);
        const u128w qlo = w_sub64(n0, 1ull + 2ull * H);
        const uint32_t nbits = cnt + H;          // odd bits [0, nbits) hold every q probed
        const uint32_t nwords = (nbits + 31) / 32;
        for (uint32_t w = tid; w < nwords; w += kWideThreads)
            bits[w] = 0;
        __syncthreads();
        // strikes: every odd multiple of each sieving prime in the window
        // (q_lo + 2j = 0 mod p  <=>  2j = -q_lo mod p)
        for (uint32_t k = 1 + tid; k < a.nsieve; k += kWideThreads) {
            const uint32_t p = a.primes[k];
            const uint32_t r = w_mod_u32(qlo, p);
            const uint32_t x = r ? p - r : 0u;                    // -q_lo mod p
            uint32_t j = (x & 1) ? (x >> 1) + (p >> 1) + 1 : (x >> 1);   // x / 2 mod p
            for (; j < nbits; j += p)
                atomicOr(&bits[j >> 5], 1u << (j & 31));
        }
        __syncthreads();

        // probe: each wave takes a contiguous share of the segment's evens;
        // a lane holds one even (index i) and its next candidate k, and takes
        // the next even of the share when its current one is settled
        const uint32_t share = (cnt + NWAVE - 1) / NWAVE;
        const uint32_t i0 = wave * share;
        const uint32_t i1 = i0 + share < cnt ? i0 + share : cnt;
        uint64_t sum = 0, nres = 0, bp = 0, nsp = 0;
        u128w bn = {0, 0};
        uint32_t next = i0 + 64;    // first even of the share not yet handed out
        uint32_t i = i0 + lane;
        uint32_t k = 1;
        bool active = i < i1;
        while (__ballot(active) != 0) {
            bool settled = false;
            if (active) {
                // next surviving candidate: bit(n - p) = i + H - (p - 1)/2 clear
                uint32_t p = 0;
                for (; k <= a.ncand; ++k) {
                    p = a.primes[k];
                    const uint32_t b = i + H - (p >> 1);
                    if (((bits[b >> 5] >> (b & 31)) & 1u) == 0)
                        break;
                }
                const u128w n = w_add64(n0, 2ull * i);
                if (k > a.ncand) {
                    // no candidate p <= P_max: to Phase 2
                    const unsigned long long e = atomicAdd(&a.ctr[1], 1ull);
                    if (e < a.spill_cap) {
                        a.spill[e].n_lo = n.lo;
                        a.spill[e].n_hi = n.hi;
                        a.spill[e].p = 0;
                    }
                    ++nsp;
                    settled = true;
                } else if (w_bpsw(w_sub64(n, p))) {
                    sum += p;
                    ++nres;
                    max_merge_w(bp, bn, p, n);
                    settled = true;
                } else {
                    ++k;
                }
            }
            // settled lanes take the next evens of the share, in lane order
            const unsigned long long need = __ballot(active && settled);
            if (active && settled) {
                const uint32_t rank = (uint32_t)__popcll(need & ((1ull << lane) - 1));
                i = next + rank;
                k = 1;
                active = i < i1;
            }
            next += (uint32_t)__popcll(need);
        }
        // workgroup reduction of the segment's aggregates
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            sum += __shfl_xor(sum, off, 64);
            nres += __shfl_xor(nres, off, 64);
            nsp += __shfl_xor(nsp, off, 64);
            const uint64_t op = __shfl_xor(bp, off, 64);
            u128w on;
            on.lo = __shfl_xor(bn.lo, off, 64);
            on.hi = __shfl_xor(bn.hi, off, 64);
            if (op)
                max_merge_w(bp, bn, op, on);
        }
        if (lane == 0) {
            red_sum[wave] = sum;
            red_cnt[wave] = nres;
            red_p[wave] = bp;
            red_nl[wave] = bn.lo;
            red_nh[wave] = bn.hi;
            red_sp[wave] = nsp;
        }
        __syncthreads();
        if (tid == 0) {
            GbWideRecord r = {};
            u128w n = {0, 0};
            uint64_t p = 0;
            for (uint32_t w = 0; w < NWAVE; ++w) {
                r.checksum += red_sum[w];
                r.verified += red_cnt[w];
                r.nspill += red_sp[w];
                if (red_p[w])
                    max_merge_w(p, n, red_p[w], u128w{red_nl[w], red_nh[w]});
            }
            r.max_p = p;
            r.max_n_lo = n.lo;
            r.max_n_hi = n.hi;
            a.rec[seg] = r;
        }
        // the next claim is published by the barrier at the top of the loop,
        // after which the window is cleared: every wave is past its probe here
        __syncthreads();
    }
}

// Wide Phase 2: one wave per spilled n tests 64 table primes above P_max at a
// time (ascending), q = n - p by trial division up to 97 and Baillie-PSW; the
// lowest lane with a probable prime gives p_min.  n / 2 > 2^63 exceeds every
// table prime, so the search ends only with the table.
__global__ __launch_bounds__(256) void wide_phase2_kernel(GbWideArgs a)
{
    const unsigned long long total = a.ctr[1];
    const uint64_t count = total < a.spill_cap ? total : a.spill_cap;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t wid = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    constexpr uint32_t kTd[23] = {5,  7,  11, 13, 17, 19, 23, 29, 31, 37, 41, 43,
                                  47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97};
    for (uint64_t e = wid; e < count; e += nw) {
        const u128w n = {a.spill[e].n_lo, a.spill[e].n_hi};
        uint64_t found = 0;
        for (uint64_t base = (uint64_t)a.ncand + 1; base < a.nprimes; base += 64) {
            const uint64_t idx = base + lane;
            const bool valid = idx < a.nprimes;
            bool isp = false;
            uint32_t p = 0;
            if (valid) {
                p = a.primes[idx];
                const u128w q = w_sub64(n, p);
                bool small = w_mod_u32(q, 3) == 0;
                for (int t = 0; t < 23 && !small; ++t)
                    small = w_mod_u32(q, kTd[t]) == 0;
                isp = !small && w_bpsw(q);
            }
            const unsigned long long pm = __ballot(isp);
            if (pm) {
                found = __shfl(p, __ffsll(pm) - 1, 64);
                break;
            }
            if (__ballot(valid) != ~0ull)
                break;   // the table ended inside this group
        }
        if (lane == 0)
            a.spill[e].p = found;
    }
}

// One workgroup: fold the segment records and the Phase-2 results, and write
// the unresolved evens (p = 0 or p > P_max) in ascending order by counting
// rank (the spill list holds at most 2^16 entries on this path).
__global__ __launch_bounds__(256) void wide_reduce_kernel(GbWideArgs a, uint64_t P_max,
                                                          GbWideResult *res, u128w *unres)
{
    __shared__ uint64_t sh[5][4];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t s = 0, c = 0, bp = 0, failed = 0, un = 0;
    u128w bn = {0, 0};
    for (uint64_t g = tid; g < a.nsegs; g += 256) {
        const GbWideRecord r = a.rec[g];
        s += r.checksum;
        c += r.verified;
        if (r.max_p)
            max_merge_w(bp, bn, r.max_p, u128w{r.max_n_lo, r.max_n_hi});
    }
    const unsigned long long total = a.ctr[1];
    const uint64_t count = total < a.spill_cap ? total : a.spill_cap;
    for (uint64_t e = tid; e < count; e += 256) {
        const GbWideSpill sp = a.spill[e];
        const u128w n = {sp.n_lo, sp.n_hi};
        if (sp.p) {
            ++c;
            s += sp.p;
            max_merge_w(bp, bn, sp.p, n);
        } else {
            ++failed;
        }
        if (sp.p == 0 || sp.p > P_max) {
            ++un;
            uint64_t rank = 0;
            for (uint64_t f = 0; f < count; ++f) {
                const GbWideSpill o = a.spill[f];
                if ((o.p == 0 || o.p > P_max) && w_lt(u128w{o.n_lo, o.n_hi}, n))
                    ++rank;
            }
            unres[rank] = n;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        c += __shfl_xor(c, off, 64);
        failed += __shfl_xor(failed, off, 64);
        un += __shfl_xor(un, off, 64);
        const uint64_t op = __shfl_xor(bp, off, 64);
        u128w on;
        on.lo = __shfl_xor(bn.lo, off, 64);
        on.hi = __shfl_xor(bn.hi, off, 64);
        if (op)
            max_merge_w(bp, bn, op, on);
    }
    if (lane == 0) {
        sh[0][wave] = s;
        sh[1][wave] = c;
        sh[2][wave] = failed;
        sh[3][wave] = un;
        sh[4][wave] = bp;
    }
    __shared__ u128w shn[4];
    if (lane == 0)
        shn[wave] = bn;
    __syncthreads();
    if (tid == 0) {
        GbWideResult r = {};
        uint64_t p = 0;
        u128w n = {0, 0};
        for (int w = 0; w < 4; ++w) {
            r.checksum += sh[0][w];
            r.verified += sh[1][w];
            r.n_failed += sh[2][w];
            r.n_unresolved += sh[3][w];
            if (sh[4][w])
                max_merge_w(p, n, sh[4][w], shn[w]);
        }
        r.max_p = p;
        r.max_n_lo = n.lo;
        r.max_n_hi = n.hi;
        r.spills = total;
        *res = r;
    }
}

__global__ void wide_reset_kernel(unsigned long long *ctr)
{
    if (threadIdx.x < 2)
        ctr[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void bpsw_kernel(const u128w *q, uint64_t count, uint8_t *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const u128w v = q[i];
        bool r;
        if (v.hi == 0) {
            r = gb_is_prime_u64(v.lo);   // deterministic below 2^64
        } else if ((v.lo & 1) == 0 || w_mod_u32(v, 3) == 0) {
            r = false;
        } else {
            r = w_bpsw(v);
        }
        out[i] = r ? 1 : 0;
    }
}

}  // namespace

hipError_t gb_launch_wide(const GbWideArgs &a, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(wide_sieve_probe_kernel, dim3(grid), dim3(kWideThreads), 0, s, a);
    return hipGetLastError();
}

int gb_wide_occupancy()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, wide_sieve_probe_kernel, kWideThreads,
                                                     0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n < 1 ? 1 : n;
}

hipError_t gb_launch_wide_phase2(const GbWideArgs &a, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(wide_phase2_kernel, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t gb_launch_wide_reduce(const GbWideArgs &a, uint64_t P_max, GbWideResult *res,
                                 u128w *unres, hipStream_t s)
{
    hipLaunchKernelGGL(wide_reduce_kernel, dim3(1), dim3(256), 0, s, a, P_max, res, unres);
    return hipGetLastError();
}

hipError_t gb_launch_wide_reset(unsigned long long *ctr, hipStream_t s)
{
    hipLaunchKernelGGL(wide_reset_kernel, dim3(1), dim3(64), 0, s, ctr);
    return hipGetLastError();
}

hipError_t gb_launch_bpsw(const u128w *q, uint64_t count, uint8_t *out, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    uint64_t blocks = (count + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    hipLaunchKernelGGL(bpsw_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, q, count, out);
    return hipGetLastError();
}
