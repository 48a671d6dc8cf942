// gb_wide.hip -- verification past 2^64 (the paper's future-work direction
// of Sec. 5: 128-bit sieve arithmetic coupled with a Baillie-PSW test).
//
// Beyond 2^64 the table of primes up to 2^32 no longer reaches sqrt(q), so the
// sieve is a pre-filter: it marks every odd q = n - p with a prime factor up to
// the sieve bound S (the table primes up to min(T, 2^28)), and the survivors
// are decided, in ascending p for each n, by the Baillie-PSW test; the first
// survivor that passes gives p_min(n).  A range is taken in chunks of up to
// 2^26 evens (a runtime setting), each with a strike bitmap in device memory
// over the odd numbers from n0 - 1 - 2H, and three kernels per chunk:
//   * the primes below 2^16 strike 2^15-bit passes of the bitmap in LDS
//     (below 2^12 a whole wave per prime, above one thread per prime), and
//     each pass is written out as whole words;
//   * the larger sieving primes, one thread each, locate their first multiple
//     once per chunk (a 128-by-32 remainder) and OR their strikes into the
//     bitmap with device atomics (about 0.56 per bit of the chunk in all);
//   * a persistent probe over all CUs: a lane holds two evens, each with its
//     next candidate, reads a candidate's bit from the bitmap, and runs
//     Baillie-PSW on the first survivor (the base-2 test and the Lucas test in
//     rounds of their own, so that lanes whose survivor fails the base-2 test
//     do not wait through a Lucas test; two evens per lane, so that a lane
//     whose one even waits for the Lucas round works on the other); a settled
//     even's slot claims the next unclaimed even of the chunk (one atomic per
//     wave and round), so every lane stays busy until the chunk runs out.
// A survivor of the sieve to S is prime with probability about 1.78 ln S / ln q
// (0.8 near 2^64, 0.4 near 2^128), so an even costs one Baillie-PSW test and
// a few base-2 tests of composite survivors.  Evens that no candidate
// p <= P_max resolves are spilled to the wide Phase-2 kernel, which continues
// with the table primes above P_max.
#include "gb_wide.h"

namespace {

__device__ __forceinline__ void max_merge_w(uint64_t &bp, u128w &bn, uint64_t p, u128w n)
{
    if (p > bp || (p == bp && w_lt(n, bn))) {
        bp = p;
        bn = n;
    }
}

// The first bit b >= 0 with q0 + 2b = 0 (mod p), q0 odd, p an odd prime:
// 2b = -q0 (mod p), so b = x / 2 mod p for x = -q0 mod p.
__device__ __forceinline__ uint32_t wide_first_bit(u128w q0, uint32_t p)
{
    const uint32_t r = w_mod_u32(q0, p);
    const uint32_t x = r ? p - r : 0u;
    return (x & 1) ? (x >> 1) + (p >> 1) + 1 : (x >> 1);
}

// Strikes of the primes below 2^16, one 2^15-bit pass of the chunk's bitmap
// per workgroup iteration, written out as whole words (every word of the
// bitmap is written, so nothing needs clearing).  Block 0 also resets the
// chunk's probe claim counter.
__global__ __launch_bounds__(256) void wide_small_sieve_kernel(GbWideArgs a, GbWideChunk ch)
{
    __shared__ uint32_t w[kWideSieveWords];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (blockIdx.x == 0 && tid == 0)
        a.ctr[0] = 0;
    const uint32_t nwords = (ch.nbits + 31) / 32;
    for (uint32_t w0 = blockIdx.x * kWideSieveWords; w0 < nwords; w0 += gridDim.x * kWideSieveWords) {
        const uint32_t nw = nwords - w0 < kWideSieveWords ? nwords - w0 : kWideSieveWords;
        const uint32_t sbits = ch.nbits - 32 * w0 < 32 * nw ? ch.nbits - 32 * w0 : 32 * nw;
        for (uint32_t x = tid; x < kWideSieveWords; x += 256)
            w[x] = 0;
        __syncthreads();
        const u128w q0 = w_add64(ch.qlo, 64ull * w0);   // odd number of the pass's bit 0
        for (uint32_t k = 1 + wave; k < a.ncoop; k += 4) {
            const uint32_t p = a.primes[k];
            for (uint32_t j = wide_first_bit(q0, p) + lane * p; j < sbits; j += 64 * p)
                atomicOr(&w[j >> 5], 1u << (j & 31));
        }
        for (uint32_t k = a.ncoop + tid; k < a.nsmall; k += 256) {
            const uint32_t p = a.primes[k];
            for (uint32_t j = wide_first_bit(q0, p); j < sbits; j += p)
                atomicOr(&w[j >> 5], 1u << (j & 31));
        }
        __syncthreads();
        for (uint32_t x = tid; x < nw; x += 256)
            ch.bits[w0 + x] = w[x];
        __syncthreads();
    }
}

// Strikes of the sieving primes from 2^16 to S: one thread per prime, its
// first multiple in the chunk from one 128-by-32 remainder, then every odd
// multiple OR-ed into the bitmap.
__global__ __launch_bounds__(256) void wide_large_fill_kernel(GbWideArgs a, GbWideChunk ch)
{
    const uint32_t stride = gridDim.x * 256;
    for (uint32_t k = a.nsmall + blockIdx.x * 256 + threadIdx.x; k < a.nsieve; k += stride) {
        const uint32_t p = a.primes[k];
        for (uint64_t j = wide_first_bit(ch.qlo, p); j < ch.nbits; j += p)
            atomicOr(&ch.bits[j >> 5], 1u << (j & 31));
    }
}

// The probe of one chunk (persistent; the records accumulate over the chunks),
// its Baillie-PSW arithmetic over N 28-bit limbs (every q of the chunk below
// 2^(28 N - 12)).
template <int N>
__global__ __launch_bounds__(kWideThreads) void wide_probe_kernel(GbWideArgs a, GbWideChunk ch)
{
    constexpr uint32_t NWAVE = kWideThreads / 64;
    __shared__ uint64_t red_sum[NWAVE], red_cnt[NWAVE], red_p[NWAVE], red_nl[NWAVE],
        red_nh[NWAVE], red_sp[NWAVE];
    // bit h: 2h + 1 is a candidate (an odd prime <= P_max); one spare word
    __shared__ uint32_t cand[kWideCandWords + 1];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t H = a.H, hmax = a.hmax;
    const uint32_t *bits = ch.bits;
    for (uint32_t t = tid; t <= kWideCandWords; t += kWideThreads)
        cand[t] = 0;
    __syncthreads();
    for (uint32_t t = 1 + tid; t <= a.ncand; t += kWideThreads) {
        const uint32_t h = a.primes[t] >> 1;
        atomicOr(&cand[h >> 5], 1u << (h & 31));
    }
    __syncthreads();
    uint64_t sum = 0, nres = 0, bp = 0, nsp = 0;
    u128w bn = {0, 0};
    // A lane holds two evens (slots 0 and 1), each with a half-offset h: the
    // candidates p = 2h + 1 below it are settled.  A slot is `ready` when its
    // candidate 2h + 1 has passed the base-2 test (qi and one kept for the
    // Lucas test).  A wave runs base-2 rounds,
    // in which every lane with a slot lacking a ready candidate scans that
    // slot to its next survivor and tests it, until lucas_at of its active
    // lanes hold a ready slot, then one Lucas round in which every such lane
    // tests one ready slot: the base-2 failures (most composite survivors)
    // cost a base-2 test, not a whole Baillie-PSW round, and a lane whose one
    // even is ready still has the other to work on in the base-2 rounds.
    uint64_t claim = 0;
    if (lane == 0)
        claim = atomicAdd(&a.ctr[0], 128ull);
    claim = __shfl(claim, 0, 64);
    bool act0 = claim + lane < ch.cnt, act1 = claim + 64 + lane < ch.cnt;
    uint32_t i0 = (uint32_t)(claim + lane), i1 = (uint32_t)(claim + 64 + lane);   // below 2^31
    uint32_t k0 = 1, k1 = 1, qi0 = 0, qi1 = 0;   // half-offsets: p = 3 first
    bool rdy0 = false, rdy1 = false;
    u128w one0 = {0, 0}, one1 = {0, 0};
    for (;;) {
        const bool need0 = act0 && !rdy0, need1 = act1 && !rdy1;
        const bool has_rdy = (act0 && rdy0) || (act1 && rdy1);
        const unsigned long long act = __ballot(act0 || act1);
        if (act == 0)
            break;
        const uint32_t nact = (uint32_t)__popcll(act);
        const uint32_t nrdy = (uint32_t)__popcll(__ballot(has_rdy));
        const bool base2 = nrdy < (nact < ch.lucas_at ? nact : ch.lucas_at);
        // the slot this lane works on in this round
        const bool s1 = base2 ? !need0 : !(act0 && rdy0);
        const bool work = base2 ? (need0 || need1) : has_rdy;
        const uint32_t i = s1 ? i1 : i0;
        uint32_t k = s1 ? k1 : k0;
        uint32_t qi = s1 ? qi1 : qi0;
        u128w one = s1 ? one1 : one0;
        bool ready = false, settled = false;
        if (work) {
            const u128w n = w_add64(ch.n0, 2ull * i);
            if (base2) {
                // next surviving candidate, 32 half-offsets h at a time:
                // bit(n - p) = i + H - h for p = 2h + 1, so the 32 bits from
                // i + H - h - 31 up, reversed, are the strikes of h, h + 1, ...,
                // h + 31 (H >= hmax + 32 keeps the first bit at or above 0; the
                // bitmap has a spare word for the pair read)
                bool hit = false;
                while (k <= hmax) {
                    const uint32_t b0 = i + H - k - 31;
                    const uint32_t w = b0 >> 5;
                    const uint64_t pair = ((uint64_t)bits[w + 1] << 32) | bits[w];
                    const uint32_t struck = __builtin_bitreverse32((uint32_t)(pair >> (b0 & 31)));
                    const uint32_t cw = k >> 5;
                    const uint64_t cpair = ((uint64_t)cand[cw + 1] << 32) | cand[cw];
                    const uint32_t surv = (uint32_t)(cpair >> (k & 31)) & ~struck;
                    if (surv) {
                        k += (uint32_t)__builtin_ctz(surv);
                        hit = true;
                        break;
                    }
                    k += 32;
                }
                const uint32_t p = 2 * k + 1;
                if (!hit) {
                    // no candidate p <= P_max: to Phase 2
                    const unsigned long long e = atomicAdd(&a.ctr[1], 1ull);
                    if (e < a.spill_cap) {
                        a.spill[e].n_lo = n.lo;
                        a.spill[e].n_hi = n.hi;
                        a.spill[e].p = 0;
                    }
                    ++nsp;
                    settled = true;
                } else {
                    const u128w q = w_sub64(n, p);
                    qi = wl_qinv(q.lo);
                    one = w_r_mod(q, 28 * N);
                    if (w_sprp2<N>(q, qi, one))
                        ready = true;
                    else
                        ++k;
                }
            } else {
                const uint32_t p = 2 * k + 1;
                if (w_slucas<N>(w_sub64(n, p), qi, one)) {
                    sum += p;
                    ++nres;
                    max_merge_w(bp, bn, p, n);
                    settled = true;
                } else {
                    ++k;
                }
            }
            if (s1) {
                k1 = k;
                qi1 = qi;
                one1 = one;
                rdy1 = ready;
            } else {
                k0 = k;
                qi0 = qi;
                one0 = one;
                rdy0 = ready;
            }
        }
        // settled slots take the next evens of the chunk, in lane order
        const unsigned long long need = __ballot(work && settled);
        if (need) {
            uint64_t base = 0;
            if (lane == 0)
                base = atomicAdd(&a.ctr[0], (unsigned long long)__popcll(need));
            base = __shfl(base, 0, 64);
            if (work && settled) {
                const uint64_t ni = base + (uint64_t)__popcll(need & ((1ull << lane) - 1));
                const bool more = ni < ch.cnt;
                if (s1) {
                    i1 = (uint32_t)ni;
                    k1 = 1;
                    act1 = more;
                } else {
                    i0 = (uint32_t)ni;
                    k0 = 1;
                    act0 = more;
                }
            }
        }
    }
    // workgroup reduction, merged into this block's record
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
        GbWideRecord r = a.rec[blockIdx.x];
        u128w n = {r.max_n_lo, r.max_n_hi};
        uint64_t p = r.max_p;
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
        a.rec[blockIdx.x] = r;
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

// One workgroup: fold the probe records and the Phase-2 results, and write
// the unresolved evens (p = 0 or p > P_max) in ascending order by counting
// rank (the spill list holds at most 2^16 entries on this path).
__global__ __launch_bounds__(256) void wide_reduce_kernel(GbWideArgs a, uint64_t P_max,
                                                          GbWideResult *res, u128w *unres)
{
    __shared__ uint64_t sh[5][4];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t s = 0, c = 0, bp = 0, failed = 0, un = 0;
    u128w bn = {0, 0};
    for (uint64_t g = tid; g < a.nrec; g += 256) {
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

__global__ __launch_bounds__(256) void wide_reset_kernel(GbWideArgs a)
{
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t < 2)
        a.ctr[t] = 0;
    if (t < a.nrec)
        a.rec[t] = GbWideRecord{};
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

hipError_t gb_launch_wide_chunk(const GbWideArgs &a, const GbWideChunk &ch, uint32_t sieve_grid,
                                uint32_t fill_grid, int limbs, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(wide_small_sieve_kernel, dim3(sieve_grid), dim3(256), 0, s, a, ch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (fill_grid) {
        hipLaunchKernelGGL(wide_large_fill_kernel, dim3(fill_grid), dim3(256), 0, s, a, ch);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (limbs == 3)
        hipLaunchKernelGGL(wide_probe_kernel<3>, dim3(grid), dim3(kWideThreads), 0, s, a, ch);
    else if (limbs == 4)
        hipLaunchKernelGGL(wide_probe_kernel<4>, dim3(grid), dim3(kWideThreads), 0, s, a, ch);
    else
        hipLaunchKernelGGL(wide_probe_kernel<5>, dim3(grid), dim3(kWideThreads), 0, s, a, ch);
    return hipGetLastError();
}

int gb_wide_occupancy(int limbs)
{
    int n = 0;
    const hipError_t e =
        limbs == 3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, wide_probe_kernel<3>,
                                                                   kWideThreads, 0)
        : limbs == 4 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, wide_probe_kernel<4>,
                                                                     kWideThreads, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, wide_probe_kernel<5>,
                                                                     kWideThreads, 0);
    if (e != hipSuccess) {
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

hipError_t gb_launch_wide_reset(const GbWideArgs &a, hipStream_t s)
{
    const uint32_t n = a.nrec > 2 ? a.nrec : 2;
    hipLaunchKernelGGL(wide_reset_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a);
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
