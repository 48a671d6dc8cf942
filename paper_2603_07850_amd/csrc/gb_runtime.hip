// gb_runtime.hip -- host side of libgoldbach: the C ABI declared in
// include/goldbach.h, argument validation before any launch (Sec. 3.5),
// status codes instead of exit() (Sec. 3.4, graceful error handling), the
// resident prime table (Sec. 3.1) and the launch sequence of one verification:
//
//   reset counters -> persistent sieve+probe -> Phase 2 -> reduce -> emit list
//
// Every kernel of the sequence reads its sizes from device memory, so the
// sequence has no host round trip between kernels; the host waits once at the
// end and copies the result records out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/goldbach.h"
#include "gb_internal.h"

namespace {

thread_local std::string g_err;

void set_err(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

#define GB_HIP(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            set_err("%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
            return GB_EHIP;                                                            \
        }                                                                              \
    } while (0)

#define GB_TRY(expr)                   \
    do {                               \
        gb_status s_ = (expr);         \
        if (s_ != GB_OK)               \
            return s_;                 \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void release()
    {
        if (p)
            (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // grow-only device buffer; contents are not preserved
    gb_status reserve(size_t need)
    {
        if (need <= bytes)
            return GB_OK;
        release();
        size_t want = std::max(need, (size_t)4096);
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            set_err("hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
            return GB_ENOMEM;
        }
        bytes = want;
        return GB_OK;
    }
};

struct HostBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void release()
    {
        if (p)
            (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
    gb_status reserve(size_t need)
    {
        if (need <= bytes)
            return GB_OK;
        release();
        size_t want = std::max(need, (size_t)4096);
        hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            set_err("hipHostMalloc(%zu) failed: %s", want, hipGetErrorString(e));
            return GB_ENOMEM;
        }
        bytes = want;
        return GB_OK;
    }
};

struct Ctx {
    std::mutex mu;
    int device = -1;
    int num_cu = 0;
    uint64_t T = 0;
    uint64_t nprimes = 0;
    DevBuf primes;
    std::vector<uint32_t> small;  // host copy of the primes <= 65536 (launch planning)
    gb_params params = {18, 256, 4096, 0};
    // workspaces of the verification sequence
    DevBuf d_iv, d_rec, d_spill, d_res, d_unres, d_ctr;
    HostBuf h_iv, h_res, h_ctr;
    uint64_t spill_cap = 0;
};

Ctx &ctx()
{
    static Ctx c;
    return c;
}

uint64_t isqrt_u64(uint64_t x)
{
    uint64_t r = (uint64_t)std::sqrt((double)x);
    if (r > 0xFFFFFFFFull)
        r = 0xFFFFFFFFull;
    while (r * r > x)
        --r;
    while (r < 0xFFFFFFFFull && (r + 1) * (r + 1) <= x)
        ++r;
    return r;
}

// Inward rounding of [A, B] to even bounds with A >= 4; false if empty.
bool normalize(uint64_t A, uint64_t B, uint64_t *An, uint64_t *Bn)
{
    const uint64_t b = B & ~(uint64_t)1;
    uint64_t a;
    if (A & 1) {
        if (A == UINT64_MAX) {
            *An = UINT64_MAX;
            *Bn = b;
            return false;
        }
        a = A + 1;
    } else {
        a = A;
    }
    if (a < 4)
        a = 4;
    *An = a;
    *Bn = b;
    return a <= b;
}

gb_status use_device(Ctx &c)
{
    if (c.device < 0 || !c.primes.p) {
        set_err("no prime table: call gb_base_primes first");
        return GB_ENOTABLE;
    }
    GB_HIP(hipSetDevice(c.device));
    return GB_OK;
}

bool params_valid(const gb_params &p)
{
    if (!gb_probe_supported((int)p.seg_log2, (int)p.wg_size))
        return false;
    if (p.window != 0 && (p.window < 3 || p.window > 65536))
        return false;
    return p.wg_per_cu <= 64;
}

void release_all(Ctx &c)
{
    c.primes.release();
    c.d_iv.release();
    c.d_rec.release();
    c.d_spill.release();
    c.d_res.release();
    c.d_unres.release();
    c.d_ctr.release();
    c.h_iv.release();
    c.h_res.release();
    c.h_ctr.release();
    c.small.clear();
    c.T = 0;
    c.nprimes = 0;
    c.spill_cap = 0;
}

gb_status build_table(Ctx &c, uint64_t limit)
{
    int dev = 0;
    GB_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    GB_HIP(hipGetDeviceProperties(&prop, dev));
    release_all(c);
    c.device = dev;
    c.num_cu = prop.multiProcessorCount;
    const uint64_t T = std::max<uint64_t>(limit, 65536);
    const uint64_t nodd = (T + 1) / 2;  // odd numbers 1, 3, ..., <= T
    const uint32_t segbits = 1u << gb_table_seg_log2();
    const uint32_t nsegs = (uint32_t)((nodd + segbits - 1) / segbits);
    // pi(x) < 1.25506 x / ln x for x > 1 (Rosser and Schoenfeld 1962)
    const uint64_t cap = (uint64_t)(1.25506 * (double)T / std::log((double)T)) + 64;

    DevBuf seed, counts;
    gb_status st;
    if ((st = seed.reserve(8192 * 4 + 64)) != GB_OK)
        return st;
    if ((st = counts.reserve((size_t)nsegs * 4 + 64)) != GB_OK) {
        seed.release();
        return st;
    }
    if ((st = c.primes.reserve(cap * 4)) != GB_OK) {
        seed.release();
        counts.release();
        return st;
    }
    uint32_t *d_seed = (uint32_t *)seed.p;
    uint32_t *d_nseed = d_seed + 8192;
    uint64_t *d_total = (uint64_t *)((char *)counts.p + ((size_t)nsegs * 4 + 7) / 8 * 8);
    hipStream_t s = nullptr;
    hipError_t e = gb_launch_seed(d_seed, d_nseed, s);
    if (e == hipSuccess)
        e = gb_launch_table_count(d_seed, d_nseed, T, nsegs, (uint32_t *)counts.p, s);
    if (e == hipSuccess)
        e = gb_launch_table_scan((uint32_t *)counts.p, nsegs, d_total, s);
    if (e == hipSuccess)
        e = gb_launch_table_emit(d_seed, d_nseed, T, nsegs, (uint32_t *)counts.p,
                                 (uint32_t *)c.primes.p, s);
    uint64_t total = 0;
    if (e == hipSuccess)
        e = hipMemcpy(&total, d_total, 8, hipMemcpyDeviceToHost);
    seed.release();
    counts.release();
    if (e != hipSuccess) {
        set_err("prime table build failed: %s", hipGetErrorString(e));
        release_all(c);
        return GB_EHIP;
    }
    c.T = T;
    c.nprimes = total + 1;
    if (c.nprimes > cap) {
        set_err("prime table overflow (%llu > %llu)", (unsigned long long)c.nprimes,
                (unsigned long long)cap);
        release_all(c);
        return GB_EHIP;
    }
    const uint64_t nsmall = std::min<uint64_t>(c.nprimes, 6542);  // pi(65536)
    c.small.resize(nsmall);
    e = hipMemcpy(c.small.data(), c.primes.p, nsmall * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        set_err("prime table copy failed: %s", hipGetErrorString(e));
        release_all(c);
        return GB_EHIP;
    }
    return GB_OK;
}

// Number of table primes <= x for x <= 65536, from the host copy.
uint64_t small_count_le(const Ctx &c, uint64_t x)
{
    return (uint64_t)(std::upper_bound(c.small.begin(), c.small.end(), (uint32_t)std::min<uint64_t>(x, 0xFFFFFFFFu)) -
                      c.small.begin());
}

struct Plan {
    uint32_t H = 0;          // halo bits
    uint32_t ncand = 0;      // odd candidates probed in LDS
    uint64_t total_segs = 0;
    uint64_t total_evens = 0;
    std::vector<GbInterval> iv;
    std::vector<uint64_t> An, Bn;
};

gb_status make_plan(Ctx &c, const uint64_t *AB, uint64_t k, uint64_t P_max, const gb_params &pr,
                    Plan &pl)
{
    if (P_max < 2) {
        set_err("P_max must be >= 2 (got %llu)", (unsigned long long)P_max);
        return GB_EINVAL;
    }
    if (P_max > c.T) {
        set_err("P_max %llu exceeds the prime table limit %llu", (unsigned long long)P_max,
                (unsigned long long)c.T);
        return GB_ERANGE;
    }
    const uint64_t cap = pr.window ? pr.window : 65536;
    const uint64_t pwin = std::min<uint64_t>(P_max, cap);
    const uint64_t nc = small_count_le(c, pwin);  // includes 2
    pl.ncand = (uint32_t)(nc > 0 ? nc - 1 : 0);
    uint32_t hmax = pl.ncand ? (c.small[pl.ncand] - 1) / 2 : 0;
    pl.H = std::max<uint32_t>(32, (hmax + 31) & ~31u);
    const uint64_t W = 1ull << pr.seg_log2;
    const uint64_t E = W - pl.H;
    pl.iv.resize(k);
    pl.An.resize(k);
    pl.Bn.resize(k);
    uint64_t seg = 0, evens = 0;
    for (uint64_t i = 0; i < k; ++i) {
        uint64_t a, b;
        const bool ne = normalize(AB[2 * i], AB[2 * i + 1], &a, &b);
        pl.An[i] = a;
        pl.Bn[i] = b;
        GbInterval g = {};
        g.A = a;
        g.seg_first = seg;
        if (ne) {
            if (isqrt_u64(b) > c.T) {
                set_err("prime table limit %llu is below isqrt(B) = %llu for interval %llu",
                        (unsigned long long)c.T, (unsigned long long)isqrt_u64(b),
                        (unsigned long long)i);
                return GB_ERANGE;
            }
            g.nE = (b - a) / 2 + 1;
            g.nseg = (g.nE + E - 1) / E;
        }
        seg += g.nseg;
        evens += g.nE;
        pl.iv[i] = g;
    }
    pl.total_segs = seg;
    pl.total_evens = evens;
    return GB_OK;
}

// One pass of the launch sequence; the caller retries when spills overflow.
gb_status run_once(Ctx &c, const Plan &pl, uint64_t P_max, const gb_params &pr, hipStream_t s,
                   uint64_t *spills_out)
{
    const uint64_t k = pl.iv.size();
    GB_TRY(c.d_iv.reserve(k * sizeof(GbInterval)));
    GB_TRY(c.d_rec.reserve(std::max<uint64_t>(pl.total_segs, 1) * sizeof(GbSegRecord)));
    GB_TRY(c.d_res.reserve(k * sizeof(GbIvResult)));
    GB_TRY(c.d_ctr.reserve(sizeof(GbCounters)));
    GB_TRY(c.h_iv.reserve(k * sizeof(GbInterval)));
    GB_TRY(c.h_res.reserve(k * sizeof(GbIvResult)));
    GB_TRY(c.h_ctr.reserve(sizeof(GbCounters)));
    GB_TRY(c.d_spill.reserve(c.spill_cap * sizeof(GbSpill)));
    GB_TRY(c.d_unres.reserve(c.spill_cap * sizeof(uint64_t)));

    std::memcpy(c.h_iv.p, pl.iv.data(), k * sizeof(GbInterval));
    GB_HIP(hipMemcpyAsync(c.d_iv.p, c.h_iv.p, k * sizeof(GbInterval), hipMemcpyHostToDevice, s));
    GbCounters *ctr = (GbCounters *)c.d_ctr.p;
    GB_HIP(gb_launch_reset(ctr, s));

    if (pl.total_segs) {
        int occ = 0;
        GB_HIP(gb_probe_occupancy((int)pr.seg_log2, (int)pr.wg_size, &occ));
        if (occ < 1)
            occ = 1;
        if (pr.wg_per_cu)
            occ = std::min<int>(occ, (int)pr.wg_per_cu);
        const uint64_t grid = std::min<uint64_t>(pl.total_segs, (uint64_t)c.num_cu * occ);
        GbProbeArgs a = {};
        a.primes = (const uint32_t *)c.primes.p;
        a.nprimes = c.nprimes;
        a.iv = (const GbInterval *)c.d_iv.p;
        a.k = (uint32_t)k;
        a.H = pl.H;
        a.ncand = pl.ncand;
        a.total_segs = pl.total_segs;
        a.rec = (GbSegRecord *)c.d_rec.p;
        a.spill = (GbSpill *)c.d_spill.p;
        a.spill_cap = c.spill_cap;
        a.ctr = ctr;
        GB_HIP(gb_launch_probe((int)pr.seg_log2, (int)pr.wg_size, (uint32_t)grid, a, s));
    }
    GB_HIP(gb_launch_phase2((const uint32_t *)c.primes.p, c.nprimes, (uint64_t)pl.ncand + 1,
                            (GbSpill *)c.d_spill.p, c.spill_cap, ctr, (uint32_t)c.num_cu * 4, s));
    GB_HIP(gb_launch_reduce((const GbInterval *)c.d_iv.p, (uint32_t)k, (const GbSegRecord *)c.d_rec.p,
                            (const GbSpill *)c.d_spill.p, c.spill_cap, ctr, P_max,
                            (GbIvResult *)c.d_res.p, s));
    GB_HIP(gb_launch_unres_emit((const GbSpill *)c.d_spill.p, c.spill_cap, ctr, P_max,
                                (uint64_t *)c.d_unres.p, (uint32_t)c.num_cu * 2, s));
    GB_HIP(hipMemcpyAsync(c.h_res.p, c.d_res.p, k * sizeof(GbIvResult), hipMemcpyDeviceToHost, s));
    GB_HIP(hipMemcpyAsync(c.h_ctr.p, ctr, sizeof(GbCounters), hipMemcpyDeviceToHost, s));
    GB_HIP(hipStreamSynchronize(s));
    *spills_out = ((GbCounters *)c.h_ctr.p)->spills;
    return GB_OK;
}

gb_status verify_many(Ctx &c, const uint64_t *AB, uint64_t k, uint64_t P_max, hipStream_t s,
                      gb_result *outs)
{
    if (k == 0)
        return GB_OK;
    if (!AB || !outs) {
        set_err("null interval or result array");
        return GB_EINVAL;
    }
    if (k > (1ull << 32) - 1) {
        set_err("too many intervals in one batch");
        return GB_EINVAL;
    }
    GB_TRY(use_device(c));
    const gb_params pr = c.params;
    Plan pl;
    GB_TRY(make_plan(c, AB, k, P_max, pr, pl));
    if (c.spill_cap == 0)
        c.spill_cap = 1 << 16;
    uint64_t spills = 0;
    for (int attempt = 0;; ++attempt) {
        GB_TRY(run_once(c, pl, P_max, pr, s, &spills));
        if (spills <= c.spill_cap)
            break;
        if (attempt >= 3) {
            set_err("spill list kept overflowing (%llu entries)", (unsigned long long)spills);
            return GB_ENOMEM;
        }
        c.spill_cap = spills + spills / 4 + 1024;
    }
    const GbIvResult *res = (const GbIvResult *)c.h_res.p;
    gb_status status = GB_OK;
    for (uint64_t i = 0; i < k; ++i) {
        gb_result &o = outs[i];
        const GbIvResult &r = res[i];
        o.A = pl.An[i];
        o.B = pl.Bn[i];
        o.P_max = P_max;
        o.verified = r.verified;
        o.max_p = r.max_p;
        o.max_p_n = r.max_p_n;
        o.checksum = r.checksum;
        o.n_unresolved = r.n_unresolved;
        o.n_failed = r.n_failed;
        if (r.n_unresolved) {
            const uint64_t take = std::min<uint64_t>(r.n_unresolved, o.unresolved ? o.unresolved_cap : 0);
            if (take) {
                GB_HIP(hipMemcpy(o.unresolved, (const uint64_t *)c.d_unres.p + r.unres_first,
                                 take * 8, hipMemcpyDeviceToHost));
            }
            if (take < r.n_unresolved) {
                status = GB_ETRUNC;
                set_err("unresolved list truncated for interval %llu (%llu > %llu)",
                        (unsigned long long)i, (unsigned long long)r.n_unresolved,
                        (unsigned long long)take);
            }
        }
    }
    return status;
}

}  // namespace

extern "C" {

gb_status gb_base_primes(uint64_t limit)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if (limit > 0xFFFFFFFFull) {
        set_err("limit %llu exceeds 2^32 - 1", (unsigned long long)limit);
        return GB_EINVAL;
    }
    return build_table(c, limit);
}

uint64_t gb_table_limit(void)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    return c.primes.p ? c.T : 0;
}

uint64_t gb_table_count(void)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    return c.primes.p ? c.nprimes : 0;
}

gb_status gb_table_read(uint32_t *out, uint64_t first, uint64_t count)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    GB_TRY(use_device(c));
    if (!out || first > c.nprimes || count > c.nprimes - first) {
        set_err("table slice out of range");
        return GB_EINVAL;
    }
    if (count)
        GB_HIP(hipMemcpy(out, (const uint32_t *)c.primes.p + first, count * 4, hipMemcpyDeviceToHost));
    return GB_OK;
}

gb_status gb_verify_range(uint64_t A, uint64_t B, uint64_t P_max, void *stream, gb_result *out)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if (!out) {
        set_err("null result");
        return GB_EINVAL;
    }
    const uint64_t AB[2] = {A, B};
    return verify_many(c, AB, 1, P_max, (hipStream_t)stream, out);
}

gb_status gb_verify_batch(const uint64_t *AB, uint64_t k, uint64_t P_max, void *stream,
                          gb_result *outs)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    return verify_many(c, AB, k, P_max, (hipStream_t)stream, outs);
}

gb_status gb_set_params(const gb_params *p)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if (!p || !params_valid(*p)) {
        set_err("unsupported launch parameters");
        return GB_EINVAL;
    }
    c.params = *p;
    return GB_OK;
}

gb_status gb_get_params(gb_params *p)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if (!p) {
        set_err("null params");
        return GB_EINVAL;
    }
    *p = c.params;
    return GB_OK;
}

gb_status gb_autotune(uint64_t A, uint64_t B, uint64_t P_max, void *stream, gb_params *best)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    GB_TRY(use_device(c));
    uint64_t An, Bn;
    if (!normalize(A, B, &An, &Bn) || (Bn - An) / 2 + 1 > (1ull << 31)) {
        set_err("calibration range must be non-empty and hold at most 2^31 evens");
        return GB_EINVAL;
    }
    const gb_params saved = c.params;
    const uint32_t logs[3] = {18, 19, 20};
    const uint32_t wgs[3] = {256, 512, 1024};
    const uint32_t wins[2] = {4096, 16384};
    double best_t = 1e300;
    gb_params best_p = saved;
    const uint64_t AB[2] = {A, B};
    hipStream_t s = (hipStream_t)stream;
    for (uint32_t lg : logs)
        for (uint32_t wg : wgs)
            for (uint32_t win : wins) {
                gb_params p = {lg, wg, win, 0};
                int occ = 0;
                if (gb_probe_occupancy((int)lg, (int)wg, &occ) != hipSuccess || occ < 1) {
                    (void)hipGetLastError();
                    continue;
                }
                c.params = p;
                gb_result r = {};
                double tmin = 1e300;
                for (int rep = 0; rep < 2; ++rep) {
                    const auto t0 = std::chrono::steady_clock::now();
                    gb_status st = verify_many(c, AB, 1, P_max, s, &r);
                    const auto t1 = std::chrono::steady_clock::now();
                    if (st != GB_OK && st != GB_ETRUNC) {
                        c.params = saved;
                        return st;
                    }
                    tmin = std::min(tmin, std::chrono::duration<double>(t1 - t0).count());
                }
                if (tmin < best_t) {
                    best_t = tmin;
                    best_p = p;
                }
            }
    c.params = best_p;
    if (best)
        *best = best_p;
    return GB_OK;
}

gb_status gb_is_prime_u64(const uint64_t *q, uint64_t count, uint8_t *is_prime, void *stream)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if (count && (!q || !is_prime)) {
        set_err("null device pointer");
        return GB_EINVAL;
    }
    if (c.device >= 0)
        GB_HIP(hipSetDevice(c.device));
    GB_HIP(gb_launch_is_prime(q, count, is_prime, (hipStream_t)stream));
    GB_HIP(hipStreamSynchronize((hipStream_t)stream));
    return GB_OK;
}

gb_status gb_release(void)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if (c.device >= 0)
        (void)hipSetDevice(c.device);
    release_all(c);
    return GB_OK;
}

const char *gb_last_error(void) { return g_err.c_str(); }

}  // extern "C"
