// gb_sieve.hip -- the hot path: one persistent kernel whose workgroups claim
// segments of evens from a device queue (an atomic counter in HBM, the
// device-side counterpart of the paper's fetch_add work pool, Sec. 3.2 and
// Alg. 1), sieve the segment's odd window into an LDS bitset (Sec. 3.1) and
// probe every even n of the segment against the ascending candidate primes
// (Phase 1, Sec. 3.3).
//
// Geometry of one segment (E = 2^LOG2E evens, halo H odd bits, H a multiple
// of 96, window W = E + H odd numbers):
//   evens    n = n0 + 2i, 0 <= i < cnt <= E
//   bit b    odd q = q_lo + 2b,  q_lo = n0 - 1 - 2H   (q_lo may be negative
//            for the first segments; every q <= 1 is marked composite)
//   then     bit(n0 + 2i - p) = i + H - (p - 1)/2, so every candidate
//            p <= 2H + 1 reads inside the window.
// Segment s of an interval starts E*s bits after segment 0, so consecutive
// windows overlap by H bits and a window bit d of the interval belongs to
// segment d >> LOG2E (and to the previous one when d mod E < H).
//
// LDS layout: odd bit b is bit b / 3 of class array b mod 3.  The class t3
// with q_lo + 2*t3 = 0 (mod 3) holds exactly the odd multiples of 3 and is
// not stored; the other two classes are LDS slots 0 and 1.  A bit is a strike
// mark: 1 = struck (not prime), 0 = prime, the convention of the strike
// bitmaps in HBM, so a strike is one OR.
//
// Sieve (every q is odd):
//   * primes 5..31   periodic 32-bit word masks per class, one word write per
//                    32 class bits;
//   * primes >= 37   strikes from max(p^2, first multiple in the window) with
//                    LDS atomic OR, class by class (a prime's
//                    multiples in one class are p class bits apart); primes up
//                    to E/512 are struck by one wave each (each lane keeps one
//                    bit position, so its mask is loop-invariant), larger ones
//                    one prime per thread with several table loads in flight;
//   * primes above the bucket bound (when the launch has buckets) are not
//                    visited here: the bucket-fill kernel has set the window
//                    bits they strike in the segment's strike bitmap in HBM,
//                    which the presieve folds into the LDS window.
// Probe (bit-parallel): evens of one residue class r (n = n0 + 2r + 6i') go
// to a wave together, a lane owning 64 consecutive i'.  For candidate p the 64
// bits q = n - p of those evens are 64 consecutive bits of one class array, so
// two funnel shifts of three LDS words test p against all 64 evens at once;
// candidates whose n - p falls in class t3 are skipped.  Hits are removed
// from the lane's open masks and the wave stops when no lane has an open even
// left; ascending p makes the first hit the minimal one.  A first pass gives
// every block a fixed number of candidates, a second pass finishes the few
// still-open blocks packed 64 per wave.  Evens still open after the window
// are appended to the spill list for the Phase-2 kernel.
#include "gb_arith.h"
#include "gb_internal.h"

namespace {

constexpr uint32_t kPre[10] = {3, 5, 7, 11, 13, 17, 19, 23, 29, 31};
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
typedef const __attribute__((address_space(4))) GbInterval *civ_t;

// Open evens of a lane's block.
__device__ __forceinline__ uint32_t open_count(uint32_t ul, uint32_t uh)
{
    return (uint32_t)(__popc(ul) + __popc(uh));
}

// Test one candidate against a lane's 64 open evens (ul, uh; bit i: even
// n0 + 128j + 2i): xl, xh hold the strike bits of the 64 numbers n - p
// (1 = not prime), funnel-shifted out of three LDS words; an even stays open
// only where n - p is struck.  c is the lane's open count before the entry
// (the gap-form checksum term).
__device__ __forceinline__ void probe_one(const char *lds, uint32_t base4, uint32_t off,
                                          uint32_t sh, uint32_t gap, uint32_t c, uint32_t &ul,
                                          uint32_t &uh, uint32_t &acc)
{
    const uint32_t addr = base4 - off;
    const uint32_t w0 = *(const uint32_t *)(lds + addr);
    const uint32_t w1 = *(const uint32_t *)(lds + addr + 4);
    const uint32_t w2 = *(const uint32_t *)(lds + addr + 8);
    const uint32_t xl = __builtin_amdgcn_alignbit(w1, w0, sh);
    const uint32_t xh = __builtin_amdgcn_alignbit(w2, w1, sh);
    acc = __umul24(gap, c) + acc;
    ul &= xl;
    uh &= xh;
}

// Four entries; c is the open count before the first.
__device__ __forceinline__ void probe_group(const char *lds, uint32_t base4, cgroup_t G, uint32_t c,
                                            uint32_t &ul, uint32_t &uh, uint32_t &acc)
{
    probe_one(lds, base4, G->c[0].off, G->c[0].sh, G->c[0].gap, c, ul, uh, acc);
#pragma unroll
    for (int t = 1; t < 4; ++t)
        probe_one(lds, base4, G->c[t].off, G->c[t].sh, G->c[t].gap, open_count(ul, uh), ul, uh,
                  acc);
}

// State of the group loop of one probe pass: the wave's last group with a
// hit (lastk, uniform: its first entry, 0 if none) and the lane's open masks
// at its start (gl, gh), plus the first entry pk (uniform, 0: none) of the
// group just run.  That group's start masks and count live in one of two
// register sets that the loop uses in turn, so no copy is made per group.
struct ProbeTrack {
    uint32_t lastk, gl, gh, pk;
};

// Settle the group just run, whose start state is (tl, th, pc): it hit
// somewhere in the wave iff some lane's open count fell below pc.  c is the
// lane's open count now.
__device__ __forceinline__ void settle_group(ProbeTrack &T, uint32_t c, uint32_t tl, uint32_t th,
                                             uint32_t pc)
{
    if (T.pk != 0 && __ballot(c != pc) != 0) {
        T.lastk = T.pk;
        T.gl = tl;
        T.gh = th;
    }
    T.pk = 0;
}

__host__ __device__ constexpr uint32_t word_pattern(uint32_t p)
{
    uint32_t m = 0;
    for (uint32_t b = 0; b < 32; b += p)
        m |= 1u << b;
    return m;
}

// 6^-1 mod p for p = 5..31 (6 * inv = 1 mod p).
__host__ __device__ constexpr uint32_t inv6_mod(uint32_t p)
{
    uint32_t x = 1;
    while ((6 * x) % p != 1)
        ++x;
    return x;
}

constexpr uint32_t kInv6[9] = {inv6_mod(5),  inv6_mod(7),  inv6_mod(11), inv6_mod(13), inv6_mod(17),
                               inv6_mod(19), inv6_mod(23), inv6_mod(29), inv6_mod(31)};

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

// First window bit as above for a window start 0 < q_lo < 2^52, q_lo = 2h + 1
// with hd = h and qd = q_lo exact doubles, and p < 2^26.  Since 1/2 = (p + 1)/2
// (mod p), the offset is d = (p - 1)/2 - h (mod p): q = floor(hd / p) from the
// estimate is within one of the true quotient (h / p < 2^46 keeps the
// estimate's error far below one), q p - h is exact by one fma, so
// t = (q p - h) + (p - 1)/2 lies in (-2p, 3p/2), and d = t - floor(t / p) p is
// exact except that a multiple t of p may give p instead of 0.  Only a prime
// above sq_lo = isqrt(q_lo) can have p^2 past q_lo; its bit (p^2 - q_lo)/2 is
// exact in double (p^2 < 2^52).
__device__ __forceinline__ uint32_t first_bit_d(double hd, double qd, uint32_t sq_lo, uint32_t p)
{
    const double pd = (double)p;
    double inv = __builtin_amdgcn_rcp(pd);
    double e = __builtin_fma(-pd, inv, 1.0);
    inv = __builtin_fma(inv, e, inv);
    e = __builtin_fma(-pd, inv, 1.0);
    inv = __builtin_fma(inv, e, inv);
    const double q = __builtin_floor(hd * inv);
    const double t = __builtin_fma(q, pd, -hd) + __builtin_fma(pd, 0.5, -0.5);
    const double f = __builtin_floor(t * inv);
    uint32_t j = (uint32_t)__builtin_fma(-f, pd, t);
    j = j == p ? 0u : j;
    // a real branch (the empty asm keeps the compiler from computing the rare
    // case for every prime)
    if (p > sq_lo) {
        asm volatile("" : "+v"(j));
        const double dsq = __builtin_fmin(__builtin_fma(pd, pd, -qd) * 0.5, 4294967295.0);
        const uint32_t jsq = (uint32_t)dsq;
        j = jsq > j ? jsq : j;
    }
    return j;
}

// First window bit as above for a window start q_lo >= 2^52 (q_lo = 2h + 1,
// h = hh + hl as a rounded double and its exact remainder): the first odd
// multiple from gb_first_odd_multiple, raised to the bit of p^2 when p^2 lies
// past q_lo (p > sq_lo = isqrt(q_lo) >= 2^26), saturated to 2^32 - 1.
__device__ __forceinline__ uint32_t first_bit_h(double hh, double hl, uint64_t qlo, uint32_t sq_lo,
                                                uint32_t p)
{
    const double pd = (double)p;
    uint32_t j = gb_first_odd_multiple(hh, hl, pd, gb_recip(p), (double)(p >> 1));
    if (p > sq_lo) {
        const uint64_t jsq = ((uint64_t)p * p - qlo) >> 1;
        if (jsq > j)
            j = jsq > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)jsq;
    }
    return j;
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

// floor(x / 3) for x < 2^23 in single precision (full-rate conversions and
// multiply; a 32-bit high multiply is quarter rate).  The float nearest 1/3
// exceeds it by less than 1e-8, so x times it lies in [x/3, x/3 + 0.09) and
// its rounding (half an ulp, at most 1/8 below 2^22) keeps the product in
// [floor(x/3), floor(x/3) + 1): truncation gives the quotient.
__device__ __forceinline__ uint32_t div3(uint32_t x)
{
    return (uint32_t)((float)x * (1.0f / 3.0f));
}

// x mod 3 given q = floor(x / 3) < 2^23: one 24-bit multiply-add (the empty
// asm keeps the compiler from merging it into a 64-bit multiply-add).
__device__ __forceinline__ uint32_t mod3(uint32_t x, uint32_t q)
{
    uint32_t r = (uint32_t)__mul24((int32_t)q, -3) + x;
    asm("" : "+v"(r));
    return r;
}

// The multiples j + k*p (p prime to 3) run through the three classes as k
// does mod 3; the one in class t is k = (t - j) * p mod 3 (p is its own
// inverse mod 3).  kt_table(t) holds that k for every (j mod 3, p mod 3) as
// 2-bit fields at bit 2 * (j mod 3) + 6 * (p mod 3).
__host__ __device__ constexpr uint32_t kt_table(uint32_t t)
{
    uint32_t K = 0;
    for (uint32_t jm = 0; jm < 3; ++jm)
        for (uint32_t pm = 1; pm < 3; ++pm)
            K |= (((t + 3 - jm) * pm) % 3) << (2 * jm + 6 * pm);
    return K;
}

// Uniform class geometry of one window: the class kept in slot 0 (slot 1
// holds the other one that is not t3), the class indices of each slot inside
// the window, and each slot's kt_table.
struct ClassGeo {
    uint32_t t3, tA;
    uint32_t lim[2];
    uint32_t ktab[2];
};

__device__ __forceinline__ ClassGeo class_geo(uint32_t t3, uint32_t weff)
{
    constexpr uint32_t K0 = kt_table(0), K1 = kt_table(1), K2 = kt_table(2);
    ClassGeo g;
    g.t3 = t3;
    g.tA = t3 == 2 ? 0u : t3 + 1;
    const uint32_t tB = t3 == 0 ? 2u : t3 - 1;
    g.lim[0] = (weff + 2 - g.tA) / 3;
    g.lim[1] = (weff + 2 - tB) / 3;
    g.ktab[0] = g.tA == 0 ? K0 : (g.tA == 1 ? K1 : K2);
    g.ktab[1] = tB == 0 ? K0 : (tB == 1 ? K1 : K2);
    return g;
}

// Strike the odd bits j, j + p, ... below weff (one prime, one thread) in the
// class arrays of the window.  A prime below the window strikes many bits:
// its multiples in one stored class are the class indices i, i + p, ..., one
// strided loop per class.  A larger prime strikes at most once.
template <uint32_t WC>
__device__ __forceinline__ void strike_prime(uint32_t *bits, const ClassGeo &g, uint32_t weff,
                                             uint32_t p, uint32_t j)
{
    if (j >= weff)
        return;
    if (p < weff) {
        // here j, p < weff < 2^21, so j + 2p < 2^23
        const uint32_t jm = mod3(j, div3(j));
        const uint32_t pm = mod3(p, div3(p));
        const uint32_t sh = 2 * jm + __umul24(pm, 6u);
#pragma unroll
        for (uint32_t s = 0; s < 2; ++s) {
            const uint32_t kt = (g.ktab[s] >> sh) & 3u;
            uint32_t *cw = bits + s * WC;
            for (uint32_t i = div3(j + __umul24(kt, p)); i < g.lim[s]; i += p)
                atomicOr(&cw[i >> 5], 1u << (i & 31));
        }
    } else {
        const uint32_t i = div3(j);
        const uint32_t t = mod3(j, i);
        if (t != g.t3)
            atomicOr(&bits[(t == g.tA ? 0u : WC) + (i >> 5)], 1u << (i & 31));
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

// Settle a lane's block after its grouped entries (called by whole waves):
// the entries after the last full group one at a time, the gap-form checksum
// correction for evens still open, the replay of the wave's last group with a
// hit (all lanes of a wave read one table, so that group holds the wave's
// largest p_min; a lane replays it from its open masks at the group's start,
// and the lowest bit of its last hit is its smallest n with that p; every
// entry replayed was tested before, so the replay reproduces the same hits),
// and the spill of evens still open.  lastk (uniform) is the first entry of
// that group, 0 if none; gl, gh the lane's masks at its start.  Bit i of the
// block is the even nbase + 6i.
__device__ __forceinline__ void finish_block(const GbProbeArgs &a, const char *lds, uint32_t base4,
                                             uint32_t tab, uint32_t nv, uint32_t k, uint32_t ul,
                                             uint32_t uh, uint32_t acc, uint32_t lastk,
                                             uint32_t gl, uint32_t gh, uint32_t open0,
                                             uint64_t nbase, uint32_t ivx, uint64_t &sum,
                                             uint32_t &nres, uint32_t &bestp, uint64_t &bestn)
{
    const ccand_t ct = (ccand_t)(a.ctab + (uint64_t)tab * 3 * kCandStride);
    const cprime_t pt = (cprime_t)(a.ptab + (uint64_t)tab * kCandStride);
    if (__ballot((ul | uh) != 0) != 0) {
        for (; k <= nv; ++k) {
            const uint32_t sl = ul, sh = uh;
            probe_one(lds, base4, ct[k - 1].off, ct[k - 1].sh, ct[k - 1].gap, open_count(ul, uh),
                      ul, uh, acc);
            if (__ballot((ul != sl) | (uh != sh)) != 0) {
                lastk = k;
                gl = sl;
                gh = sh;
            }
            if (__ballot((ul | uh) != 0) == 0) {
                ++k;
                break;
            }
        }
    }
    // entry k - 1 is the last one the wave tested
    const uint32_t open = (uint32_t)(__popc(ul) + __popc(uh));
    if (open && k > 1)
        acc -= pt[k - 2] * open;
    // a second-pass block's share is negative when it only spills evens (the
    // first pass already counted their entries), so acc is a signed value of
    // magnitude < 2^31 and is added sign-extended
    sum += (uint64_t)(int64_t)(int32_t)acc;
    nres += open0 - open;
    if (lastk) {
        uint32_t vl = gl, vh = gh, lastp = 0, hl = 0, hh = 0;
        const uint32_t kend = lastk + 3 < nv ? lastk + 3 : nv;
        const uint32_t *tabv = a.ctab + (uint64_t)tab * 3 * kCandStride;
        const uint32_t *ptv = a.ptab + (uint64_t)tab * kCandStride;
        for (uint32_t kk = lastk; kk <= kend && (vl | vh); ++kk) {
            const uint32_t *e = tabv + 3 * (kk - 1);
            const uint32_t addr = base4 - e[0];
            const uint32_t w0 = *(const uint32_t *)(lds + addr);
            const uint32_t w1 = *(const uint32_t *)(lds + addr + 4);
            const uint32_t w2 = *(const uint32_t *)(lds + addr + 8);
            const uint32_t xl = ~__builtin_amdgcn_alignbit(w1, w0, e[1]) & vl;
            const uint32_t xh = ~__builtin_amdgcn_alignbit(w2, w1, e[1]) & vh;
            if (xl | xh) {
                vl ^= xl;
                vh ^= xh;
                lastp = ptv[kk - 1];
                hl = xl;
                hh = xh;
            }
        }
        // A lane runs several blocks, not in ascending n (class by class, then
        // the second-pass queue), so an equal p keeps the smaller n, as every
        // later merge of the aggregates does.
        if (lastp != 0) {
            const uint32_t bit = hl ? (uint32_t)(__ffs(hl) - 1) : 32u + (uint32_t)(__ffs(hh) - 1);
            const uint64_t n = nbase + 6ull * bit;
            if (lastp > bestp || (lastp == bestp && n < bestn)) {
                bestp = lastp;
                bestn = n;
            }
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
            a.spill[idx].n = nbase + 6ull * bit;
            a.spill[idx].iv = ivx;
            a.spill[idx].p = 0;
        }
    }
}

// Second-pass queue entries per class of evens (a fifth of a class's blocks).
constexpr uint32_t gb_probe_queue(int log2e)
{
    return 1u << (log2e - 10);
}

// Number of primes in [37, x], counted at compile time (x <= 2^11 here).
constexpr uint32_t primes_from_37(uint32_t x)
{
    uint32_t c = 0;
    for (uint32_t n = 37; n <= x; n += 2) {
        bool pr = true;
        for (uint32_t d = 3; d * d <= n; d += 2)
            if (n % d == 0) {
                pr = false;
                break;
            }
        c += pr ? 1u : 0u;
    }
    return c;
}

// Primes up to this bound strike a window at least 1024 times: one wave each.
constexpr uint32_t wave_tier_max(int log2e)
{
    return 1u << (log2e - 9);
}

// Waves per SIMD that the LDS window allows (160 KB of LDS per CU, four SIMDs,
// at most eight waves each): the register budget is set to match it.
constexpr uint32_t lds_waves_per_simd(int log2e, int nt)
{
    const uint32_t wg_bytes = 2 * 4 * gb_class_words(log2e) + 30 * gb_probe_queue(log2e) +
                              8 * primes_from_37(wave_tier_max(log2e)) + 1024;
    const uint32_t wgs = (160u * 1024u) / wg_bytes;
    const uint32_t w = wgs * (uint32_t)(nt / 64) / 4;
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

template <int LOG2E, int NT>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(lds_waves_per_simd(LOG2E, NT)))) void sieve_probe_kernel(GbProbeArgs a)
{
    constexpr uint64_t E = 1ull << LOG2E;
    constexpr uint32_t WC = gb_class_words(LOG2E);  // words per class array
    constexpr uint32_t NWAVE = NT / 64;
    constexpr uint32_t kWaveTierMax = wave_tier_max(LOG2E);
    constexpr uint32_t kWaveN = primes_from_37(kWaveTierMax);
    __shared__ uint32_t bits[2 * WC];   // classes t3 + 1 and t3 + 2 (mod 3)
    // second-pass queues, one per class of evens: block index and open masks
    constexpr uint32_t kQueue = gb_probe_queue(LOG2E);
    __shared__ uint16_t qm[3][kQueue];
    __shared__ uint32_t ql[3][kQueue];
    __shared__ uint32_t qh[3][kQueue];
    __shared__ uint32_t qn[3];
    // first class index of each wave-tier prime in the two stored classes
    __shared__ uint32_t wt_i[2][kWaveN];
    __shared__ unsigned long long sh_seg;
    __shared__ uint32_t sh_nroot;
    __shared__ unsigned long long red_sum[NWAVE];
    __shared__ uint32_t red_cnt[NWAVE];
    __shared__ uint32_t red_p[NWAVE];
    __shared__ unsigned long long red_n[NWAVE];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    const uint32_t wave = tid >> 6;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(wave);
    const uint32_t H = a.H;        // multiple of 96
    const uint32_t H96 = H / 96;   // class-array words below a lane's first block word
    const uint32_t WCU = a.wcu;    // class-array words in use
    const uint32_t *__restrict__ primes = a.primes;
    const cprime_t cp = (cprime_t)primes;
    // primes[kFirstStrided .. nwave) are struck one prime per wave
    const uint32_t nwave = count_le(primes, a.nprimes, kWaveTierMax);
    const uint32_t tabbase = (uint32_t)(LOG2E - 18) * 9;

    if (tid == 0)
        sh_seg = atomicAdd(a.claim, 1ull);
    __syncthreads();
    for (;;) {
        const uint64_t claim = uniform64(sh_seg);  // published by the last barrier
        if (claim >= a.nsegs)
            break;
        const uint64_t seg = a.seg_base + claim;

        // ---- locate the interval and the segment geometry (uniform) ----
        // (descriptors read through the constant address space: scalar loads)
        const civ_t ivs = (civ_t)a.iv;
        uint32_t lo = 0, hi = a.k - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (ivs[mid].seg_first <= seg)
                lo = mid;
            else
                hi = mid - 1;
        }
        const uint32_t ivx = lo;
        const uint64_t iv_seg_first = ivs[ivx].seg_first;
        const uint64_t iv_A = ivs[ivx].A;
        const uint64_t iv_nE = ivs[ivx].nE;
        const uint64_t iv_nseg = ivs[ivx].nseg;
        const uint64_t js = seg - iv_seg_first;
        const uint64_t n0 = iv_A + 2 * E * js;
        const uint64_t rem = iv_nE - E * js;
        const uint32_t cnt = (uint32_t)(rem < E ? rem : E);
        const uint32_t weff = cnt - 1 + H;          // odd bits [0, weff) are read by the probe
        const bool neg = n0 <= 2ull * H;            // q_lo < 0
        const uint64_t qlo = n0 - 1 - 2ull * H;     // valid when !neg
        const uint64_t qneg = 2ull * H + 1 - n0;    // valid when neg
        const uint64_t qhi = n0 + 2ull * cnt - 5;   // largest q any n of the segment needs
        // class of the multiples of 3: q_lo + 2*t3 = 0 (mod 3)
        const uint32_t x3 = neg ? (uint32_t)(qneg % 3) : (uint32_t)((3 - qlo % 3) % 3);
        const uint32_t t3 = (2 * x3) % 3;
        const ClassGeo cg = class_geo(t3, weff);
        // windows starting in (0, 2^52) take the double-precision first-bit
        // path, later ones the double-double one (h = (q_lo - 1) / 2 = hh + hl)
        const bool small = !neg && qlo < (1ull << 52);
        const double qd = (double)qlo;
        const double hh = (double)(qlo >> 1);
        const double hl = (double)(int64_t)((qlo >> 1) - (uint64_t)hh);
        const uint32_t sq_lo = neg ? 0u : gb_isqrt64(qlo);
        if (wave == 0) {
            const uint32_t c = count_le_wave(primes, a.nprimes, gb_isqrt64(qhi), lane);
            if (lane == 0)
                sh_nroot = c;
        }

        // first class indices of the wave-tier primes, one prime per thread
        // (published, like qn, by the barrier after the presieve)
        {
            const uint32_t nw = nwave - kFirstStrided < kWaveN ? nwave - kFirstStrided : kWaveN;
            for (uint32_t t = tid; t < nw; t += NT) {
                const uint32_t p = primes[kFirstStrided + t];
                const uint32_t j0 = small ? first_bit_d(hh, qd, sq_lo, p)
                                    : neg ? first_bit(qlo, qneg, neg, p)
                                          : first_bit_h(hh, hl, qlo, sq_lo, p);
                uint32_t i0 = 0xFFFFFFFFu, i1 = 0xFFFFFFFFu;
                if (j0 < weff) {
                    // j0 < weff < 2^21 and p <= 2^11: j0 + 2p < 2^23
                    const uint32_t sh = 2 * mod3(j0, div3(j0)) + __umul24(mod3(p, div3(p)), 6u);
                    i0 = div3(j0 + __umul24((cg.ktab[0] >> sh) & 3u, p));
                    i1 = div3(j0 + __umul24((cg.ktab[1] >> sh) & 3u, p));
                }
                wt_i[0][t] = i0;
                wt_i[1][t] = i1;
            }
        }
        if (tid < 3)
            qn[tid] = 0;   // published by the barrier after the presieve
        // ---- presieve: periodic masks of 5..31 in the two stored classes ----
        {
            const uint32_t *__restrict__ bm =
                a.bitmap ? a.bitmap + (seg - a.seg_base) * (uint64_t)(3 * WCU) : nullptr;
            uint32_t xr[9];   // -q_lo mod p (qneg mod p when neg) for p = 5..31
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const uint32_t p = kPre[i + 1];
                xr[i] = neg ? (uint32_t)(qneg % p) : (uint32_t)((p - qlo % p) % p);
            }
            for (uint32_t sl = 0; sl < 2; ++sl) {
                const uint32_t t = (t3 + 1 + sl) % 3;
                uint32_t *cw = bits + sl * WC;
                // class index i is q = q_lo + 2t + 6i: a multiple of p when
                // i = (xr - 2t) / 6 (mod p)
                uint32_t ph[9];
                uint32_t dec[9];
                // (32 * tid) mod p is recomputed here rather than kept live
                // across the segment loop, where it would be spilled
                uint32_t tt = tid;
                asm volatile("" : "+v"(tt));
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const uint32_t p = kPre[i + 1];
                    const uint32_t phi = (((xr[i] + 2 * p - 2 * t) % p) * kInv6[i]) % p;
                    ph[i] = (phi + p - (32u * tt) % p) % p;   // (phi - 32w) mod p at w = tid
                    dec[i] = (32u * NT) % p;
                }
                const uint32_t *__restrict__ bmt = bm ? bm + t * WCU : nullptr;
                for (uint32_t w = tid; w < WCU; w += NT) {
                    uint32_t m = bmt ? bmt[w] : 0u;
#pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        m |= word_pattern(kPre[i + 1]) << ph[i];
                        ph[i] = ph[i] >= dec[i] ? ph[i] - dec[i] : ph[i] + kPre[i + 1] - dec[i];
                    }
                    cw[w] = m;
                }
            }
        }
        // unmark the primes 3..31 and mark q <= 1 where the window reaches them
        if (neg || qlo <= 35) {
            __syncthreads();
            const uint64_t bmax = neg ? (35 + qneg) >> 1 : (35 - qlo) >> 1;  // odd bits 0..bmax
            const uint32_t wmax = (uint32_t)((bmax / 3) >> 5);
            for (uint32_t sl = 0; sl < 2; ++sl) {
                const uint32_t t = (t3 + 1 + sl) % 3;
                for (uint32_t w = tid; w <= wmax; w += NT) {
                    uint32_t v = bits[sl * WC + w];
                    for (uint32_t k = 0; k < 32; ++k) {
                        const uint64_t b = 3ull * (32 * w + k) + t;
                        if (b > bmax)
                            break;
                        const int64_t q = neg ? (int64_t)(2 * b) - (int64_t)qneg : (int64_t)(qlo + 2 * b);
                        v = small_prime_35(q) ? (v & ~(1u << k)) : (v | (1u << k));
                    }
                    bits[sl * WC + w] = v;
                }
            }
        }
        __syncthreads();

        const uint32_t nroot = __builtin_amdgcn_readfirstlane(sh_nroot);  // published by the barrier above
        const uint32_t nsieve = nroot < a.lb_count ? nroot : a.lb_count;  // primes struck here

        // ---- strikes, one prime per wave: 37 <= p <= kWaveTierMax ----
        // The prime's odd multiples b = j0 + kp fall in the two stored
        // classes at class indices i_s + mp.  Lane l strikes i_s + l*p + m*64p;
        // 64p is a multiple of 32, so a lane's bit position and mask never change.
        {
            const uint32_t wave_end = nwave < nsieve ? nwave : nsieve;
            for (uint32_t i = kFirstStrided + wv; i < wave_end; i += NWAVE) {
                const uint32_t p = cp[i];
#pragma unroll
                for (uint32_t sl = 0; sl < 2; ++sl) {
                    const uint32_t i0 = __builtin_amdgcn_readfirstlane(wt_i[sl][i - kFirstStrided]);
                    if (i0 >= cg.lim[sl])
                        continue;
                    const uint32_t it = i0 + __umul24(lane, p);
                    if (it < cg.lim[sl]) {
                        const uint32_t mask = 1u << (it & 31);
                        const uint32_t wend = (cg.lim[sl] + 31) >> 5;
                        uint32_t *cw = bits + sl * WC;
                        for (uint32_t w = it >> 5; w < wend; w += 2 * p)
                            atomicOr(&cw[w], mask);
                    }
                }
            }
        }
        // ---- strikes, one prime per thread: kWaveTierMax < p <= min(isqrt(q_hi), bound) ----
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
                            strike_prime<WC>(bits, cg, weff, pv[t],
                                             first_bit_d(hh, qd, sq_lo, pv[t]));
                } else if (!neg) {
#pragma unroll
                    for (uint32_t t = 0; t < kPrimesInFlight; ++t)
                        if (pv[t])
                            strike_prime<WC>(bits, cg, weff, pv[t], first_bit_h(hh, hl, qlo, sq_lo, pv[t]));
                } else {
#pragma unroll
                    for (uint32_t t = 0; t < kPrimesInFlight; ++t)
                        if (pv[t])
                            strike_prime<WC>(bits, cg, weff, pv[t], first_bit(qlo, qneg, neg, pv[t]));
                }
            }
        }
        __syncthreads();

        // ---- probe ----
        // The evens of the segment fall in three classes r (n = n0 + 2r + 6i',
        // i' = 0, 1, ...).  A wave takes 64 blocks of one class; a lane owns a
        // block of 64 consecutive i' as two mask words (lo: the first 32).  For
        // an even of class r and candidate p, n - p lies in class
        // t = (r - (p-1)/2) mod 3 of the window; candidates with t = t3 give a
        // multiple of 3 and are absent from the class's table, so a block tests
        // only the candidates that can hit.  Table entry k (p = its p) holds the
        // byte offset of the LDS word with bit(n - p) below the lane's first
        // word, the funnel-shift amount and the gap to the previous entry's p;
        // four entries make one 48-byte group, read with two scalar loads.  Per
        // entry a lane reads three LDS words, funnel-shifts the 64 bits n - p of
        // its evens, counts its open evens and removes the hits.  The checksum
        // of a block is accumulated in gap form: the sum of p_min over the evens
        // resolved by entries 1..K equals the sum over k of gap_k * (evens open
        // before k), minus p_K per even still open after K.
        //
        // Two passes: a wave runs in lockstep until its slowest block is done,
        // and a 64-even block needs far fewer entries on average than the worst
        // of 64 blocks.  The first pass gives every block ka groups of entries
        // (0.31 groups per bit of n, the best of a sweep at [4, 10^12]);
        // blocks still open then go to a per-class queue in LDS, and the second
        // pass packs 64 of them per wave and continues from entry 4*ka + 1.  A
        // block that finds its queue full simply continues in the first pass.
        const char *lds = (const char *)bits;
        uint64_t sum = 0;
        uint32_t nres = 0;
        uint32_t bestp = 0;
        uint64_t bestn = 0;
        // 4 = 2 + 2 (the only even p_min) and 6 = 3 + 3 (n - p = 3 lies in
        // class t3) are set here; the probe skips them
        const bool has6 = a.ncand >= 1 && (n0 == 6 || (n0 == 4 && cnt > 1));
        if (tid == 0) {
            if (n0 == 4) {
                sum = 2;
                nres = 1;
                bestp = 2;
                bestn = 4;
            }
            if (has6) {
                sum += 3;
                nres += 1;
                bestp = 3;
                bestn = 6;
            }
        }
        const uint32_t ka = ((64u - (uint32_t)__builtin_clzll(n0)) * 310u + 999u) / 1000u;
        uint32_t cntc[3], nblkc[3], nwbc[3];
#pragma unroll
        for (uint32_t r = 0; r < 3; ++r) {
            cntc[r] = cnt > r ? (cnt - r + 2) / 3 : 0u;
            nblkc[r] = (cntc[r] + 63) >> 6;
            nwbc[r] = (nblkc[r] + 63) >> 6;
        }
        const uint32_t nwb = nwbc[0] + nwbc[1] + nwbc[2];
        for (uint32_t wb = wv; wb < nwb; wb += NWAVE) {
            const uint32_t r = wb < nwbc[0] ? 0u : (wb < nwbc[0] + nwbc[1] ? 1u : 2u);
            const uint32_t wb0 = r == 0 ? 0u : (r == 1 ? nwbc[0] : nwbc[0] + nwbc[1]);
            const uint32_t m = (wb - wb0) * 64 + lane;   // the lane's block in class r
            const bool act = m < nblkc[r];
            uint32_t ul = 0, uh = 0;
            if (act) {
                ul = 0xFFFFFFFFu;
                uh = 0xFFFFFFFFu;
                const uint32_t left = cntc[r] - 64 * m;
                if (left < 64) {
                    if (left < 32) {
                        ul = (1u << left) - 1;
                        uh = 0;
                    } else {
                        uh = left == 32 ? 0u : (1u << (left - 32)) - 1;
                    }
                }
                if (m == 0 && ((n0 == 4 && r == 0) || (has6 && r == (n0 == 4 ? 1u : 0u))))
                    ul &= ~1u;
            }
            const uint32_t open0 = (uint32_t)(__popc(ul) + __popc(uh));
            const uint32_t tab = tabbase + r * 3 + t3;
            const cgroup_t gt = (cgroup_t)(a.ctab + (uint64_t)tab * 3 * kCandStride);
            const uint32_t nv = a.nv[r * 3 + t3];
            const uint32_t ngrp = nv >> 2;
            const uint32_t base4 = ((act ? 2 * m : 0) + H96) * 4;  // byte address of the lane's first word
            uint32_t acc = 0;     // gap-form checksum, < 64 * 2^16 per block
            ProbeTrack T = {0, 0, 0, 0};
            uint32_t tl0 = 0, th0 = 0, pc0 = 0, tl1 = 0, th1 = 0, pc1 = 0;
            uint32_t qopen = 0;   // evens handed to the second pass
            uint32_t k = 1;       // next entry (1-based)
            // One group: settle the previous one (start state in set P), hand
            // the lane's block to the second pass at group ka, stop when no
            // lane is open, else keep this group's start state in set S and
            // run it.
#define GB_FIRST_PASS_GROUP(TLS, THS, PCS, TLP, THP, PCP)                      \
            {                                                                  \
                uint32_t c = open_count(ul, uh);                               \
                settle_group(T, c, TLP, THP, PCP);                             \
                if (g == ka) {                                                 \
                    if (c != 0) {                                              \
                        const uint32_t slot = atomicAdd(&qn[r], 1u);           \
                        if (slot < kQueue) {                                   \
                            qm[r][slot] = (uint16_t)m;                         \
                            ql[r][slot] = ul;                                  \
                            qh[r][slot] = uh;                                  \
                            qopen = c;                                         \
                            ul = 0;                                            \
                            uh = 0;                                            \
                            c = 0;                                             \
                        }                                                      \
                    }                                                          \
                }                                                              \
                if (__ballot(c != 0) == 0)                                     \
                    break;                                                     \
                TLS = ul;                                                      \
                THS = uh;                                                      \
                PCS = c;                                                       \
                T.pk = k;                                                      \
                probe_group(lds, base4, gt + g, c, ul, uh, acc);               \
                k += 4;                                                        \
                if (++g >= ngrp)                                               \
                    break;                                                     \
            }
            uint32_t g = 0;
            bool odd = false;   // the group just run keeps its state in set 1
            if (ngrp > 0) {
                for (;;) {
                    odd = false;
                    GB_FIRST_PASS_GROUP(tl0, th0, pc0, tl1, th1, pc1)
                    odd = true;
                    GB_FIRST_PASS_GROUP(tl1, th1, pc1, tl0, th0, pc0)
                }
            }
#undef GB_FIRST_PASS_GROUP
            settle_group(T, open_count(ul, uh), odd ? tl1 : tl0, odd ? th1 : th0, odd ? pc1 : pc0);
            finish_block(a, lds, base4, tab, nv, k, ul, uh, acc, T.lastk, T.gl, T.gh, open0 - qopen,
                         n0 + 2ull * r + 384ull * m, ivx, sum, nres, bestp, bestn);
        }
        // The next segment is claimed here by the last wave, which takes no
        // more first-pass blocks than wave 0 and so can wait on the round
        // trip; sh_seg was read by every thread before the barriers above and
        // is read again after the one that ends this pass of the loop.
        if (tid == NT - 64)
            sh_seg = atomicAdd(a.claim, 1ull);
        __syncthreads();
        // second pass over the queued blocks, 64 per wave, class by class
        {
            uint32_t nqc[3], nqwb[3];
#pragma unroll
            for (uint32_t r = 0; r < 3; ++r) {
                const uint32_t q = qn[r];
                nqc[r] = q < kQueue ? q : kQueue;
                nqwb[r] = (nqc[r] + 63) >> 6;
            }
            const uint32_t nwb2 = nqwb[0] + nqwb[1] + nqwb[2];
            for (uint32_t wb = wv; wb < nwb2; wb += NWAVE) {
                const uint32_t r = wb < nqwb[0] ? 0u : (wb < nqwb[0] + nqwb[1] ? 1u : 2u);
                const uint32_t wb0 = r == 0 ? 0u : (r == 1 ? nqwb[0] : nqwb[0] + nqwb[1]);
                const uint32_t e = (wb - wb0) * 64 + lane;
                const bool act = e < nqc[r];
                const uint32_t m = act ? (uint32_t)qm[r][e] : 0u;
                uint32_t ul = act ? ql[r][e] : 0u;
                uint32_t uh = act ? qh[r][e] : 0u;
                const uint32_t open0 = (uint32_t)(__popc(ul) + __popc(uh));
                const uint32_t tab = tabbase + r * 3 + t3;
                const cgroup_t gt = (cgroup_t)(a.ctab + (uint64_t)tab * 3 * kCandStride);
                const uint32_t nv = a.nv[r * 3 + t3];
                const uint32_t ngrp = nv >> 2;
                const uint32_t base4 = (2 * m + H96) * 4;
                uint32_t acc = 0;
                ProbeTrack T = {0, 0, 0, 0};
                uint32_t tl0 = 0, th0 = 0, pc0 = 0, tl1 = 0, th1 = 0, pc1 = 0;
                uint32_t k = 4 * ka + 1;
#define GB_SECOND_PASS_GROUP(TLS, THS, PCS, TLP, THP, PCP)                     \
                {                                                              \
                    const uint32_t c = open_count(ul, uh);                     \
                    settle_group(T, c, TLP, THP, PCP);                         \
                    if (__ballot(c != 0) == 0)                                 \
                        break;                                                 \
                    TLS = ul;                                                  \
                    THS = uh;                                                  \
                    PCS = c;                                                   \
                    T.pk = k;                                                  \
                    probe_group(lds, base4, gt + g, c, ul, uh, acc);           \
                    k += 4;                                                    \
                    if (++g >= ngrp)                                           \
                        break;                                                 \
                }
                uint32_t g = ka;
                bool odd = false;
                if (g < ngrp) {
                    for (;;) {
                        odd = false;
                        GB_SECOND_PASS_GROUP(tl0, th0, pc0, tl1, th1, pc1)
                        odd = true;
                        GB_SECOND_PASS_GROUP(tl1, th1, pc1, tl0, th0, pc0)
                    }
                }
#undef GB_SECOND_PASS_GROUP
                settle_group(T, open_count(ul, uh), odd ? tl1 : tl0, odd ? th1 : th0,
                             odd ? pc1 : pc0);
                finish_block(a, lds, base4, tab, nv, k, ul, uh, acc, T.lastk, T.gl, T.gh, open0,
                             n0 + 2ull * r + 384ull * m, ivx, sum, nres, bestp, bestn);
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
        // Thread 0 combines the waves' partials after the barrier that ends
        // this pass of the loop: the other waves start the next segment
        // meanwhile, and none writes red_* again before the presieve barrier
        // of that segment, which thread 0 reaches only after this.  The
        // interval is complete when its last segment record is written.
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
            GbSegRecord rec;
            rec.checksum = s;
            rec.verified = c;
            rec.max_p = bp;
            rec.max_n = bp ? bn : 0;
            rec.pad = 0;
            a.rec[seg] = rec;
            __threadfence();
            if (atomicAdd(&a.done[ivx].segs_done, 1ull) + 1 == iv_nseg)
                a.done[ivx].t_done = wall_clock64();
        }
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

// One interval descriptor written from a kernel argument (a launch with no
// host staging buffer).
__global__ void put_interval_kernel(GbInterval *dst, GbInterval v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *dst = v;
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

hipError_t gb_launch_put_interval(GbInterval *dst, const GbInterval &v, hipStream_t s)
{
    hipLaunchKernelGGL(put_interval_kernel, dim3(1), dim3(64), 0, s, dst, v);
    return hipGetLastError();
}

hipError_t gb_launch_pow2_counts(const uint32_t *primes, uint64_t nprimes, uint64_t *out33,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(pow2_counts_kernel, dim3(1), dim3(64), 0, s, primes, nprimes, out33);
    return hipGetLastError();
}
