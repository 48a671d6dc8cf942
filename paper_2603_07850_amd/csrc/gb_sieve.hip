// gb_sieve.hip -- the hot path: one persistent kernel whose workgroups claim
// segments of evens from a device queue (an atomic counter in HBM, the
// device-side counterpart of the paper's fetch_add work pool, Sec. 3.2 and
// Alg. 1), sieve the segment's odd window into an LDS bitset (Sec. 3.1) and
// probe every even n of the segment against the ascending candidate primes
// (Phase 1, Sec. 3.3).
//
// Geometry of one segment (E = 2^LOG2E evens, halo H bits, window W = E + H
// bits of LDS):
//   evens    n = n0 + 2i, 0 <= i < cnt <= E
//   bit b    odd q = q_lo + 2b,  q_lo = n0 - 1 - 2H   (q_lo may be negative
//            for the first segments; every q <= 1 is marked composite)
//   then     bit(n0 + 2i - p) = i + H - (p - 1)/2, so every candidate
//            p <= 2H + 1 reads inside the window.
// Segment s of an interval starts E*s bits after segment 0, so consecutive
// windows overlap by H bits and a window bit d of the interval belongs to
// segment d >> LOG2E (and to the previous one when d mod E < H).
//
// Sieve (every q is odd):
//   * primes 3..31   periodic 32-bit word masks, one word write per 32 odds;
//   * primes >= 37   strided clears from max(p^2, first multiple in the
//                    window) with LDS atomic AND; primes up to E/1024 are
//                    cleared by one wave each (each lane keeps one bit
//                    position, so its mask is loop-invariant), larger ones one
//                    prime per thread with several table loads in flight;
//   * primes above the bucket bound (when the launch has buckets) are not
//                    visited here: the bucket-fill kernel has set the window
//                    bits they strike in the segment's strike bitmap in HBM,
//                    which the presieve folds into the LDS window.
// Probe (bit-parallel): a thread owns 64 consecutive evens.  For candidate p
// the 64 bits q = n - p of those evens are 64 consecutive window bits, so two
// funnel shifts of three LDS words test p against all 64 evens at once; hits are
// removed from the thread's unresolved mask and the wave stops when no lane
// has an unresolved even left.  Ascending p makes the first hit the minimal
// one.  Evens still open after the window are appended to the spill list for
// the Phase-2 kernel.
#include "gb_arith.h"
#include "gb_internal.h"

namespace {

constexpr uint32_t kPre[10] = {3, 5, 7, 11, 13, 17, 19, 23, 29, 31};
constexpr uint32_t kHaloMax = 32768;  // largest halo: candidates up to 65536
constexpr uint32_t kFirstStrided = 11;  // primes[11] == 37
constexpr uint32_t kPrimesInFlight = 8;  // thread-tier table loads issued together

// One probe candidate: the byte offset of the LDS word holding bit(n - p)
// below the word of bit(n), the funnel-shift amount that aligns the bits
// n - p of a lane's evens, and the gap to the previous candidate.
struct Cand {
    uint32_t off, sh, gap;
};
struct CandGroup {
    Cand c[4];
};
// The candidate and prime tables seen through the constant address space:
// loads with a uniform index compile to scalar loads.
typedef const __attribute__((address_space(4))) Cand *ccand_t;
typedef const __attribute__((address_space(4))) CandGroup *cgroup_t;
typedef const __attribute__((address_space(4))) uint32_t *cprime_t;

// Test one candidate against a lane's 64 open evens (ul, uh; bit i: even
// n0 + 128j + 2i): xl, xh hold the primality bits of the 64 numbers n - p,
// funnel-shifted out of three LDS words; the hits leave the open masks.
__device__ __forceinline__ void probe_one(const char *lds, uint32_t base4, uint32_t off,
                                          uint32_t sh, uint32_t gap, uint32_t &ul, uint32_t &uh,
                                          uint32_t &acc)
{
    const uint32_t addr = base4 - off;
    const uint32_t w0 = *(const uint32_t *)(lds + addr);
    const uint32_t w1 = *(const uint32_t *)(lds + addr + 4);
    const uint32_t w2 = *(const uint32_t *)(lds + addr + 8);
    const uint32_t xl = __builtin_amdgcn_alignbit(w1, w0, sh);
    const uint32_t xh = __builtin_amdgcn_alignbit(w2, w1, sh);
    acc = __umul24(gap, (uint32_t)(__popc(ul) + __popc(uh))) + acc;
    ul &= ~xl;
    uh &= ~xh;
}

__device__ __forceinline__ void probe_group(const char *lds, uint32_t base4, cgroup_t G,
                                            uint32_t k, uint32_t &ul, uint32_t &uh,
                                            uint32_t &acc, uint32_t &lastg, uint32_t &gl,
                                            uint32_t &gh)
{
    const uint32_t sl = ul, sh = uh;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        probe_one(lds, base4, G->c[t].off, G->c[t].sh, G->c[t].gap, ul, uh, acc);
    const bool any = (ul != sl) | (uh != sh);
    lastg = any ? k : lastg;
    gl = any ? sl : gl;
    gh = any ? sh : gh;
}

__host__ __device__ constexpr uint32_t word_pattern(uint32_t p)
{
    uint32_t m = 0;
    for (uint32_t b = 0; b < 32; b += p)
        m |= 1u << b;
    return m;
}

// Smallest bit index j of the window whose odd number q_lo + 2j is a multiple
// of p and at least p^2 (saturated to 2^32 - 1).  The window start is q_lo
// when !neg and -qneg when neg.
__device__ __forceinline__ uint32_t first_bit(uint64_t qlo, uint64_t qneg, bool neg, uint32_t p)
{
    uint32_t x;  // -q_lo mod p
    if (neg) {
        x = gb_mod_u64_u32(qneg, p);
    } else {
        const uint32_t r = gb_mod_u64_u32(qlo, p);
        x = r ? p - r : 0;
    }
    // 2*beta == x (mod p)
    const uint32_t beta = (x & 1) ? (x >> 1) + (p >> 1) + 1 : (x >> 1);
    const uint64_t p2 = (uint64_t)p * p;
    uint64_t jsq = 0;
    if (neg)
        jsq = (p2 + qneg) >> 1;
    else if (p2 > qlo)
        jsq = (p2 - qlo) >> 1;
    const uint64_t j = jsq > beta ? jsq : (uint64_t)beta;
    return j > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)j;
}

// First window bit as above for a window start 0 < q_lo < 2^52, which a
// double holds exactly (qd = q_lo, qlo32 = its low word, sq = isqrt(q_lo)),
// and p < 2^26: one double quotient estimate, within one of floor(q_lo / p),
// and an exact fma remainder in (-p, 2p) that one step corrects.  When
// p > sq, p^2 lies past q_lo by less than the window, so the distance fits
// 32 bits.
__device__ __forceinline__ uint32_t first_bit_d(double qd, uint32_t qlo32, uint32_t sq, uint32_t p)
{
    const double pd = (double)p;
    double inv = __builtin_amdgcn_rcp(pd);
    double e = __builtin_fma(-pd, inv, 1.0);
    inv = __builtin_fma(inv, e, inv);
    e = __builtin_fma(-pd, inv, 1.0);
    inv = __builtin_fma(inv, e, inv);
    const double qt = __builtin_floor(qd * inv);
    int32_t r = (int32_t)__builtin_fma(-qt, pd, qd);
    r += r < 0 ? (int32_t)p : 0;
    r -= r >= (int32_t)p ? (int32_t)p : 0;
    const uint32_t x = r ? p - (uint32_t)r : 0u;  // -q_lo mod p
    uint32_t j = (x & 1) ? (x >> 1) + (p >> 1) + 1 : (x >> 1);
    const uint32_t jsq = (p * p - qlo32) >> 1;
    return (p > sq && jsq > j) ? jsq : j;
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
           __builtin_amdgcn_readfirstlane((uint32_t)v);
}

// Number of table entries <= x (upper bound), x < 2^32.
__device__ __forceinline__ uint32_t count_le(const uint32_t *primes, uint64_t nprimes, uint32_t x)
{
    uint64_t lo = 0, hi = nprimes;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (primes[mid] <= x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (uint32_t)lo;
}

// Clear the window bits j, j + p, ... below weff (one prime, one thread).
__device__ __forceinline__ void strike_prime(uint32_t *bits, uint32_t weff, uint32_t p, uint32_t j)
{
    if (p < weff) {
        for (uint32_t jj = j; jj < weff; jj += p)
            atomicAnd(&bits[jj >> 5], ~(1u << (jj & 31)));
    } else if (j < weff) {
        atomicAnd(&bits[j >> 5], ~(1u << (j & 31)));
    }
}

// The same count found by one wave: each round its 64 lanes test 64 evenly
// spaced entries of the bracket that holds the answer, and the ballot of the
// (monotone) outcomes narrows the bracket 64-fold.  Uniform result.
__device__ __forceinline__ uint32_t count_le_wave(const uint32_t *primes, uint64_t nprimes,
                                                 uint32_t x, uint32_t lane)
{
    uint64_t lo = 0, hi = nprimes;   // the count lies in [lo, hi]
    while (lo < hi) {
        const uint64_t step = (hi - lo + 63) >> 6;
        const uint64_t idx = lo + (uint64_t)lane * step;
        const bool le = idx < hi && primes[idx] <= x;
        const uint32_t L = (uint32_t)__popcll(__ballot(le));
        if (L == 0) {
            hi = lo;
        } else {
            const uint64_t nlo = lo + (uint64_t)(L - 1) * step + 1;
            const uint64_t nhi = lo + (uint64_t)L * step;
            lo = nlo;
            hi = nhi < hi ? nhi : hi;
        }
    }
    return (uint32_t)lo;
}

__device__ __forceinline__ bool small_prime_35(int64_t q)
{
    return q == 3 || q == 5 || q == 7 || q == 11 || q == 13 || q == 17 || q == 19 || q == 23 ||
           q == 29 || q == 31;
}

// Waves per SIMD that the LDS window allows (160 KB of LDS per CU, four SIMDs,
// at most eight waves each): the register budget is set to match it.
constexpr uint32_t lds_waves_per_simd(int log2e, int nt)
{
    const uint32_t wg_bytes = (uint32_t)(((1u << log2e) + kHaloMax) / 8) + 1024;
    const uint32_t wgs = (160u * 1024u) / wg_bytes;
    const uint32_t w = wgs * (uint32_t)(nt / 64) / 4;
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

template <int LOG2E, int NT>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(lds_waves_per_simd(LOG2E, NT)))) void sieve_probe_kernel(GbProbeArgs a)
{
    constexpr uint64_t E = 1ull << LOG2E;
    constexpr uint32_t NW = (uint32_t)((E + kHaloMax) / 32);
    constexpr uint32_t NWAVE = NT / 64;
    // primes up to this bound strike a window >= 1024 times: one wave each
    constexpr uint32_t kWaveTierMax = (uint32_t)(E >> 9);
    __shared__ uint32_t bits[NW];
    __shared__ unsigned long long sh_seg;
    __shared__ uint32_t sh_nroot;
    __shared__ unsigned long long red_sum[NWAVE];
    __shared__ uint32_t red_cnt[NWAVE];
    __shared__ uint32_t red_p[NWAVE];
    __shared__ unsigned long long red_n[NWAVE];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    const uint32_t wave = tid >> 6;
    const uint32_t H = a.H;
    const uint32_t H32 = H >> 5;
    const uint32_t NWr = (uint32_t)((E + H) >> 5);  // window words in use
    const uint32_t *__restrict__ primes = a.primes;
    const cprime_t cp = (cprime_t)primes;
    // primes[kFirstStrided .. nwave) are cleared one prime per wave
    const uint32_t nwave = count_le(primes, a.nprimes, kWaveTierMax);

    for (;;) {
        if (tid == 0)
            sh_seg = atomicAdd(a.claim, 1ull);
        __syncthreads();
        const uint64_t claim = uniform64(sh_seg);
        if (claim >= a.nsegs)
            break;
        const uint64_t seg = a.seg_base + claim;

        // ---- locate the interval and the segment geometry (uniform) ----
        uint32_t lo = 0, hi = a.k - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (a.iv[mid].seg_first <= seg)
                lo = mid;
            else
                hi = mid - 1;
        }
        const uint32_t ivx = lo;
        const GbInterval I = a.iv[ivx];
        const uint64_t js = seg - I.seg_first;
        const uint64_t n0 = I.A + 2 * E * js;
        const uint64_t rem = I.nE - E * js;
        const uint32_t cnt = (uint32_t)(rem < E ? rem : E);
        const uint32_t weff = cnt - 1 + H;          // bits [0, weff) are read by the probe
        const bool neg = n0 <= 2ull * H;            // q_lo < 0
        const uint64_t qlo = n0 - 1 - 2ull * H;     // valid when !neg
        const uint64_t qneg = 2ull * H + 1 - n0;    // valid when neg
        const uint64_t qhi = n0 + 2ull * cnt - 5;   // largest q any n of the segment needs
        // windows starting in (0, 2^52) take the double-precision first-bit path
        const bool small = !neg && qlo < (1ull << 52);
        const double qd = (double)qlo;
        const uint32_t sq = small ? gb_isqrt64(qlo) : 0u;
        if (wave == 0) {
            const uint32_t c = count_le_wave(primes, a.nprimes, gb_isqrt64(qhi), lane);
            if (lane == 0)
                sh_nroot = c;
        }

        // ---- presieve: periodic masks of 3..31 ----
        {
            uint32_t ph[10];
            uint32_t dec[10];
#pragma unroll
            for (int i = 0; i < 10; ++i) {
                const uint32_t p = kPre[i];
                const uint32_t x = neg ? (uint32_t)(qneg % p) : (uint32_t)((p - qlo % p) % p);
                const uint32_t beta = (x & 1) ? (x + p) >> 1 : x >> 1;
                ph[i] = (beta + p - (32u * tid) % p) % p;   // (beta - 32w) mod p at w = tid
                dec[i] = (32u * NT) % p;
            }
            // bits struck by the primes above the bucket bound (if any)
            const uint32_t *__restrict__ bm =
                a.bitmap ? a.bitmap + (seg - a.seg_base) * (uint64_t)NWr : nullptr;
            for (uint32_t w = tid; w < NWr; w += NT) {
                uint32_t m = bm ? bm[w] : 0u;
#pragma unroll
                for (int i = 0; i < 10; ++i) {
                    m |= word_pattern(kPre[i]) << ph[i];
                    ph[i] = ph[i] >= dec[i] ? ph[i] - dec[i] : ph[i] + kPre[i] - dec[i];
                }
                bits[w] = ~m;
            }
        }
        // restore the primes 3..31 and clear q <= 1 where the window reaches them
        if (neg || qlo <= 35) {
            __syncthreads();
            const uint64_t bmax = neg ? (35 + qneg) >> 1 : (35 - qlo) >> 1;
            for (uint64_t w = tid; w <= (bmax >> 5); w += NT) {
                uint32_t v = bits[w];
                for (uint32_t k = 0; k < 32; ++k) {
                    const uint64_t b = 32 * w + k;
                    if (b > bmax)
                        break;
                    const int64_t q = neg ? (int64_t)(2 * b) - (int64_t)qneg : (int64_t)(qlo + 2 * b);
                    v = small_prime_35(q) ? (v | (1u << k)) : (v & ~(1u << k));
                }
                bits[w] = v;
            }
        }
        __syncthreads();

        const uint32_t nroot = __builtin_amdgcn_readfirstlane(sh_nroot);  // published by the barrier above
        const uint32_t nsieve = nroot < a.lb_count ? nroot : a.lb_count;  // primes cleared here
        const uint32_t wend = (weff + 31) >> 5;

        // ---- strided clears, one prime per wave: 37 <= p <= kWaveTierMax ----
        // Lane l strikes bits j0 + l*p + m*64p; 64p is a multiple of 32, so a
        // lane's bit position within its words, and its mask, never change.
        {
            const uint32_t wv = __builtin_amdgcn_readfirstlane(wave);
            const uint32_t wave_end = nwave < nsieve ? nwave : nsieve;
            for (uint32_t i = kFirstStrided + wv; i < wave_end; i += NWAVE) {
                const uint32_t p = cp[i];
                const uint32_t j0 = small ? first_bit_d(qd, (uint32_t)qlo, sq, p)
                                          : first_bit(qlo, qneg, neg, p);
                const uint64_t jt = (uint64_t)j0 + (uint64_t)lane * p;
                if (jt < weff) {
                    const uint32_t mask = ~(1u << (jt & 31));
                    const uint32_t step = 2 * p;  // words per 64p bits
                    for (uint32_t w = (uint32_t)(jt >> 5); w < wend; w += step)
                        atomicAnd(&bits[w], mask);
                }
            }
        }
        // ---- strided clears, one prime per thread: kWaveTierMax < p <= min(isqrt(q_hi), bound) ----
        // kPrimesInFlight table loads are issued before the first is used.
        {
            const uint32_t first = nwave > kFirstStrided ? nwave : kFirstStrided;
            for (uint32_t i0 = first + tid; i0 < nsieve; i0 += kPrimesInFlight * NT) {
                uint32_t pv[kPrimesInFlight];
#pragma unroll
                for (uint32_t t = 0; t < kPrimesInFlight; ++t) {
                    const uint32_t ii = i0 + t * NT;
                    pv[t] = ii < nsieve ? primes[ii] : 0u;
                }
                if (small) {
#pragma unroll
                    for (uint32_t t = 0; t < kPrimesInFlight; ++t)
                        if (pv[t])
                            strike_prime(bits, weff, pv[t], first_bit_d(qd, (uint32_t)qlo, sq, pv[t]));
                } else {
#pragma unroll
                    for (uint32_t t = 0; t < kPrimesInFlight; ++t)
                        if (pv[t])
                            strike_prime(bits, weff, pv[t], first_bit(qlo, qneg, neg, pv[t]));
                }
            }
        }
        __syncthreads();

        // ---- probe ----
        // A lane owns a block of 64 consecutive evens, n0 + 128j + 2i for
        // i < 64, as two mask words (lo: i < 32).  Candidate k (p = primes[k],
        // k >= 1) comes from the candidate table as three words: the byte
        // offset of the word holding bit(n - p) below the lane's first word,
        // the funnel-shift amount and the gap p_k - p_(k-1) (p_0 = 0); four
        // candidates make one 48-byte group, read with two scalar loads.  Per
        // candidate a lane reads three LDS words, funnel-shifts the 64 bits
        // n - p of its evens, counts its open evens and removes the hits.  The
        // checksum of a block is accumulated in gap form: the sum of p_min
        // over the evens resolved by candidates 1..K equals the sum over k of
        // gap_k * (evens open before k), minus p_K per even still open after K.
        const cgroup_t gt = (cgroup_t)a.ctab;
        const ccand_t ct = (ccand_t)a.ctab;
        const uint32_t ncand = a.ncand;
        const uint32_t ngrp = ncand >> 2;
        const char *lds = (const char *)bits;
        const uint32_t nblk = (cnt + 63) >> 6;
        uint64_t sum = 0;
        uint32_t nres = 0;
        uint32_t bestp = 0;
        uint64_t bestn = 0;
        if (n0 == 4 && tid == 0) {  // 4 = 2 + 2, the only n whose p_min is even
            sum = 2;
            nres = 1;
            bestp = 2;
            bestn = 4;
        }
        for (uint32_t jb = 0; jb < nblk; jb += NT) {
            const uint32_t j = jb + tid;
            const bool act = j < nblk;
            uint32_t ul = 0, uh = 0;
            if (act) {
                ul = 0xFFFFFFFFu;
                uh = 0xFFFFFFFFu;
                const uint32_t r = cnt & 63;
                if (j == nblk - 1 && r) {
                    if (r < 32) {
                        ul = (1u << r) - 1;
                        uh = 0;
                    } else {
                        uh = r == 32 ? 0u : (1u << (r - 32)) - 1;
                    }
                }
                if (n0 == 4 && j == 0)
                    ul &= ~1u;
            }
            const uint32_t open0 = (uint32_t)(__popc(ul) + __popc(uh));
            const uint32_t base4 = ((act ? 2 * j : 0) + H32) * 4;  // byte address of the lane's first word
            uint32_t acc = 0;     // gap-form checksum, < 64 * 2^16 per block
            uint32_t lastg = 0;   // first candidate of the last group with a hit
            uint32_t gl = 0;      // open evens at the start of that group
            uint32_t gh = 0;
            uint32_t k = 1;       // next candidate
            for (uint32_t g = 0; g < ngrp; ++g) {
                probe_group(lds, base4, gt + g, k, ul, uh, acc, lastg, gl, gh);
                k += 4;
                if (__ballot((ul | uh) != 0) == 0)
                    break;
            }
            // the candidates after the last full group, one at a time
            if (__ballot((ul | uh) != 0) != 0) {
                for (; k <= ncand; ++k) {
                    const uint32_t sl = ul, sh = uh;
                    probe_one(lds, base4, ct[k - 1].off, ct[k - 1].sh, ct[k - 1].gap, ul, uh, acc);
                    const bool any = (ul != sl) | (uh != sh);
                    lastg = any ? k : lastg;
                    gl = any ? sl : gl;
                    gh = any ? sh : gh;
                    if (__ballot((ul | uh) != 0) == 0) {
                        ++k;
                        break;
                    }
                }
            }
            // k - 1 is the last candidate the wave tested
            const uint32_t open = (uint32_t)(__popc(ul) + __popc(uh));
            if (open && k > 1)
                acc -= cp[k - 1] * open;
            sum += acc;
            nres += open0 - open;
            // Replay the last group with a hit: its last hitting candidate is
            // the block's largest p_min, and the lowest bit of that hit is the
            // smallest n attaining it.  Every candidate replayed here was also
            // tested above, so the replay reproduces the same hits.
            if (lastg) {
                uint32_t vl = gl, vh = gh, lastp = 0, hl = 0, hh = 0;
                const uint32_t kend = lastg + 3 < ncand ? lastg + 3 : ncand;
                const uint32_t *tab = a.ctab;
                for (uint32_t kk = lastg; kk <= kend && (vl | vh); ++kk) {
                    const uint32_t *e = tab + 3 * (kk - 1);
                    const uint32_t addr = base4 - e[0];
                    const uint32_t w0 = *(const uint32_t *)(lds + addr);
                    const uint32_t w1 = *(const uint32_t *)(lds + addr + 4);
                    const uint32_t w2 = *(const uint32_t *)(lds + addr + 8);
                    const uint32_t xl = __builtin_amdgcn_alignbit(w1, w0, e[1]) & vl;
                    const uint32_t xh = __builtin_amdgcn_alignbit(w2, w1, e[1]) & vh;
                    if (xl | xh) {
                        vl ^= xl;
                        vh ^= xh;
                        lastp = primes[kk];
                        hl = xl;
                        hh = xh;
                    }
                }
                if (lastp > bestp) {
                    bestp = lastp;
                    const uint32_t bit = hl ? (uint32_t)(__ffs(hl) - 1) : 32u + (uint32_t)(__ffs(hh) - 1);
                    bestn = n0 + 128ull * j + 2ull * bit;
                }
            }
            while (ul | uh) {
                uint32_t bit;
                if (ul) {
                    bit = __ffs(ul) - 1;
                    ul &= ul - 1;
                } else {
                    bit = 32 + __ffs(uh) - 1;
                    uh &= uh - 1;
                }
                const unsigned long long idx = atomicAdd(&a.ctr->spills, 1ull);
                if (idx < a.spill_cap) {
                    a.spill[idx].n = n0 + 128ull * j + 2ull * bit;
                    a.spill[idx].iv = ivx;
                    a.spill[idx].p = 0;
                }
            }
        }

        // ---- workgroup reduction of the segment's partial aggregates ----
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            sum += __shfl_xor(sum, off, 64);
            nres += __shfl_xor(nres, off, 64);
            const uint32_t op = __shfl_xor(bestp, off, 64);
            const uint64_t on = __shfl_xor(bestn, off, 64);
            if (op > bestp || (op == bestp && on < bestn)) {
                bestp = op;
                bestn = on;
            }
        }
        if (lane == 0) {
            red_sum[wave] = sum;
            red_cnt[wave] = nres;
            red_p[wave] = bestp;
            red_n[wave] = bestn;
        }
        __syncthreads();
        if (tid == 0) {
            uint64_t s = 0, c = 0, bn = 0;
            uint32_t bp = 0;
            for (uint32_t w = 0; w < NWAVE; ++w) {
                s += red_sum[w];
                c += red_cnt[w];
                if (red_p[w] > bp || (red_p[w] == bp && red_n[w] < bn)) {
                    bp = red_p[w];
                    bn = red_n[w];
                }
            }
            GbSegRecord r;
            r.checksum = s;
            r.verified = c;
            r.max_p = bp;
            r.max_n = bp ? bn : 0;
            r.pad = 0;
            a.rec[seg] = r;
            // the interval is complete when its last segment record is written
            __threadfence();
            if (atomicAdd(&a.done[ivx].segs_done, 1ull) + 1 == I.nseg)
                a.done[ivx].t_done = wall_clock64();
        }
        __syncthreads();
    }
}

__global__ void reset_kernel(GbCounters *ctr, GbIvDone *done, uint32_t k,
                             unsigned long long *claims, uint32_t nclaims)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < sizeof(GbCounters) / 8)
        reinterpret_cast<unsigned long long *>(ctr)[t] = t == 2 ? wall_clock64() : 0;
    for (uint32_t i = t; i < nclaims; i += gridDim.x * blockDim.x)
        claims[i] = 0;
    for (uint32_t i = t; i < k; i += gridDim.x * blockDim.x) {
        done[i].segs_done = 0;
        done[i].t_done = 0;
    }
}

// Number of table primes <= 2^j for j = 0..32 (the planner's bucket bounds).
__global__ void pow2_counts_kernel(const uint32_t *primes, uint64_t nprimes, uint64_t *out)
{
    const uint32_t j = threadIdx.x;
    if (j <= 32) {
        const uint64_t x = j == 32 ? 0xFFFFFFFFull : (1ull << j);
        out[j] = count_le(primes, nprimes, (uint32_t)x);
    }
}

template <int LOG2E, int NT>
hipError_t launch_t(uint32_t grid, const GbProbeArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((sieve_probe_kernel<LOG2E, NT>), dim3(grid), dim3(NT), 0, s, a);
    return hipGetLastError();
}

template <int LOG2E, int NT>
hipError_t occ_t(int *n)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, sieve_probe_kernel<LOG2E, NT>, NT, 0);
}

}  // namespace

int gb_probe_supported(int seg_log2, int wg_size)
{
    return (seg_log2 >= 18 && seg_log2 <= 20) && (wg_size == 256 || wg_size == 512 || wg_size == 1024);
}

#define GB_DISPATCH(FN, ...)                                                   \
    switch (seg_log2 * 4096 + wg_size) {                                       \
    case 18 * 4096 + 256: return FN<18, 256>(__VA_ARGS__);                     \
    case 18 * 4096 + 512: return FN<18, 512>(__VA_ARGS__);                     \
    case 18 * 4096 + 1024: return FN<18, 1024>(__VA_ARGS__);                   \
    case 19 * 4096 + 256: return FN<19, 256>(__VA_ARGS__);                     \
    case 19 * 4096 + 512: return FN<19, 512>(__VA_ARGS__);                     \
    case 19 * 4096 + 1024: return FN<19, 1024>(__VA_ARGS__);                   \
    case 20 * 4096 + 256: return FN<20, 256>(__VA_ARGS__);                     \
    case 20 * 4096 + 512: return FN<20, 512>(__VA_ARGS__);                     \
    case 20 * 4096 + 1024: return FN<20, 1024>(__VA_ARGS__);                   \
    default: return hipErrorInvalidValue;                                      \
    }

hipError_t gb_launch_probe(int seg_log2, int wg_size, uint32_t grid, const GbProbeArgs &a,
                           hipStream_t s)
{
    GB_DISPATCH(launch_t, grid, a, s)
}

hipError_t gb_probe_occupancy(int seg_log2, int wg_size, int *blocks_per_cu)
{
    GB_DISPATCH(occ_t, blocks_per_cu)
}

hipError_t gb_launch_reset(GbCounters *ctr, GbIvDone *done, uint32_t k,
                           unsigned long long *claims, uint32_t nclaims, hipStream_t s)
{
    const uint32_t blocks = k > 256 * 64 ? 64 : (k + 255) / 256 + 1;
    hipLaunchKernelGGL(reset_kernel, dim3(blocks), dim3(256), 0, s, ctr, done, k, claims, nclaims);
    return hipGetLastError();
}

hipError_t gb_launch_pow2_counts(const uint32_t *primes, uint64_t nprimes, uint64_t *out33,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(pow2_counts_kernel, dim3(1), dim3(64), 0, s, primes, nprimes, out33);
    return hipGetLastError();
}
