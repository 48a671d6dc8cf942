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
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "goldbach.h"
#include "gb_internal.h"
#include "gb_wide_types.h"

// Scratch of gb_verify_range_noalloc: counters, the interval descriptor and
// result, the segment records, the spill list and the unresolved list of one
// call live in this file-scope device array, so that the call allocates
// nothing.  Each device holds its own copy at its own address until the
// process ends.  In host code the name `scratch` is a host-side stand-in, not
// a device address: host code uses only the address hipGetSymbolAddress gives
// for the current device (kept in g_scratch at gb_base_primes).
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices] = {};   // device address of `scratch` per device (context lock)


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

// Device memory of the library comes from the registered allocator
// (gb_set_allocator; hipMalloc / hipFree by default).  A buffer remembers the
// allocator that gave it its memory and returns the memory there.
struct Allocator {
    gb_alloc_fn alloc = nullptr;   // null: hipMalloc / hipFree
    gb_free_fn free_ = nullptr;
    void *user = nullptr;
};
Allocator g_alloc;   // guarded by the context lock

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    Allocator from;
    void release()
    {
        if (p) {
            if (from.alloc)
                from.free_(p, bytes, nullptr, from.user);
            else
                (void)hipFree(p);
        }
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
        if (g_alloc.alloc) {
            p = g_alloc.alloc(want, nullptr, g_alloc.user);
            if (!p) {
                set_err("registered allocator returned no memory for %zu bytes", want);
                return GB_ENOMEM;
            }
        } else {
            hipError_t e = hipMalloc(&p, want);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                p = nullptr;
                set_err("hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
                return GB_ENOMEM;
            }
        }
        from = g_alloc;
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
    DevBuf d_ctab, d_ptab;        // probe candidate tables and their p (gb_internal.h)
    std::vector<uint32_t> small;  // host copy of the primes <= 65536 (launch planning)
    gb_params params = {18, 256, 4096, 0, 0, 0};
    uint64_t pi2[33] = {};        // number of table primes <= 2^k
    // workspaces of the verification sequence
    DevBuf d_iv, d_rec, d_spill, d_res, d_unres, d_ctr;
    HostBuf h_iv, h_res, h_ctr;
    uint64_t spill_cap = 0;
    DevBuf d_done;
    HostBuf h_done;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    gb_stats stats = {};
    double wall_khz = 100000.0;      // device wall-clock rate
    uint64_t last_k = 0;
    unsigned long long last_t_start = 0;
    hipStream_t cap_stream = nullptr;   // capture stream of the batched graph
    hipGraphExec_t graph_exec = nullptr;
    std::vector<uint64_t> graph_key;    // every value the captured sequence bakes in
    // strike bitmaps of the large primes, their chunks and fill tasks
    DevBuf d_bitmap, d_chunk, d_claims, d_task;
    HostBuf h_chunk, h_task;
    // bitmap-and-scan emission of long unresolved lists
    DevBuf d_woff, d_ubits, d_ublock;
    HostBuf h_woff;
    std::vector<uint64_t> last_slot;    // last call: caller's index -> kernel slot
    // workspaces of the verification past 2^64
    DevBuf d_wrec, d_wspill, d_wres, d_wunres, d_wctr, d_wbits;
    HostBuf h_wres;
    uint32_t wide_chunk_log2 = kWideChunkLog2Default;   // evens per chunk past 2^64
    // stream-ordered calls: the gb_result image they copy out, and the event
    // that ends the last one's use of the shared workspaces
    DevBuf d_async;
    hipEvent_t ev_busy = nullptr;
    bool async_pending = false;
    // autotuner choices by (device, kind, P_max, size class of the calibration)
    std::map<std::vector<uint64_t>, gb_params> tuned;
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

// Wait on the host until the last stream-ordered call no longer uses the
// shared workspaces (before they are resized or released, or before a
// blocking call enqueues work that reuses them).
void quiesce(Ctx &c)
{
    if (c.async_pending && c.ev_busy)
        (void)hipEventSynchronize(c.ev_busy);
    c.async_pending = false;
}

bool params_valid(const gb_params &p)
{
    if (!gb_probe_supported((int)p.seg_log2, (int)p.wg_size))
        return false;
    if (p.window != 0 && (p.window < 3 || p.window > 65536))
        return false;
    if (p.bucket_log2 != 0 && (p.bucket_log2 < 17 || p.bucket_log2 > 32))
        return false;
    return p.wg_per_cu <= 64 && p.bucket_mib <= (1u << 20);
}

// Before a table is rebuilt on the same device: the captured graph (it holds
// the table's address) goes, and the table counts as absent until the build
// ends.  The buffers stay: the prime table's is reused when large enough, and
// the candidate tables (from the primes below 2^16, the same for every table)
// are kept as they are.  Nothing of the library may still be running.
void release_tables(Ctx &c)
{
    if (c.device >= 0 && c.primes.p)
        (void)hipDeviceSynchronize();
    c.async_pending = false;
    c.T = 0;
    c.nprimes = 0;
    c.graph_key.clear();
    if (c.graph_exec)
        (void)hipGraphExecDestroy(c.graph_exec);
    c.graph_exec = nullptr;
}

void release_all(Ctx &c)
{
    // memory may go back to a caching allocator that hands it out again at
    // once: nothing of the library may still be running on it
    if (c.device >= 0 && c.primes.p)
        (void)hipDeviceSynchronize();
    c.async_pending = false;
    if (c.ev_busy)
        (void)hipEventDestroy(c.ev_busy);
    c.ev_busy = nullptr;
    c.d_async.release();
    c.primes.release();
    c.d_ctab.release();
    c.d_ptab.release();
    c.d_iv.release();
    c.d_rec.release();
    c.d_spill.release();
    c.d_res.release();
    c.d_unres.release();
    c.d_ctr.release();
    c.d_done.release();
    c.h_done.release();
    c.d_bitmap.release();
    c.d_chunk.release();
    c.d_claims.release();
    c.d_task.release();
    c.d_woff.release();
    c.d_ubits.release();
    c.d_ublock.release();
    c.h_woff.release();
    c.h_chunk.release();
    c.h_task.release();
    c.graph_key.clear();
    if (c.graph_exec)
        (void)hipGraphExecDestroy(c.graph_exec);
    c.graph_exec = nullptr;
    if (c.cap_stream)
        (void)hipStreamDestroy(c.cap_stream);
    c.cap_stream = nullptr;
    c.h_iv.release();
    c.h_res.release();
    c.h_ctr.release();
    c.d_wrec.release();
    c.d_wspill.release();
    c.d_wres.release();
    c.d_wunres.release();
    c.d_wctr.release();
    c.d_wbits.release();
    c.h_wres.release();
    c.small.clear();
    for (auto &e : c.ev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    c.T = 0;
    c.nprimes = 0;
    c.spill_cap = 0;
}

gb_status build_table(Ctx &c, uint64_t limit)
{
    int dev = 0;
    GB_HIP(hipGetDevice(&dev));
    int ncu = 0;
    GB_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // a table on the same device keeps the verification workspaces (sized for
    // earlier calls, they stay valid); on another device everything goes
    if (c.device == dev)
        release_tables(c);
    else
        release_all(c);
    if (dev < 0 || dev >= kMaxDevices) {
        set_err("device index %d is outside the supported 0..%d", dev, kMaxDevices - 1);
        return GB_EINVAL;
    }
    if (!g_scratch[dev]) {
        // once per device, with that device current
        void *ptr = nullptr;
        const hipError_t se = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (se != hipSuccess || !ptr) {
            (void)hipGetLastError();
            set_err("hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                    hipGetErrorString(se));
            return GB_EHIP;
        }
        g_scratch[dev] = ptr;
    }
    c.device = dev;
    c.num_cu = ncu;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
        c.wall_khz = khz;
    const uint64_t T = std::max<uint64_t>(limit, 65536);
    const uint64_t nodd = (T + 1) / 2;  // odd numbers 1, 3, ..., <= T
    const uint32_t segbits = 1u << gb_table_seg_log2();
    const uint32_t nsegs = (uint32_t)((nodd + segbits - 1) / segbits);
    // pi(x) < 1.25506 x / ln x for x > 1 (Rosser and Schoenfeld 1962)
    const uint64_t cap = (uint64_t)(1.25506 * (double)T / std::log((double)T)) + 64;

    DevBuf seed, counts, stash;
    gb_status st;
    if ((st = seed.reserve(8192 * 4 + 64)) != GB_OK)
        return st;
    if ((st = counts.reserve((size_t)nsegs * 4 + 64)) != GB_OK) {
        seed.release();
        return st;
    }
    // each table block's sieved bits, written by the count pass and read by
    // the emit pass (T / 16 bytes: 256 MiB for T = 2^32 - 1)
    if ((st = stash.reserve((size_t)nsegs * gb_table_block_words() * 4)) != GB_OK) {
        seed.release();
        counts.release();
        return st;
    }
    if ((st = c.primes.reserve(cap * 4)) != GB_OK) {
        seed.release();
        counts.release();
        stash.release();
        return st;
    }
    uint32_t *d_seed = (uint32_t *)seed.p;
    uint32_t *d_nseed = d_seed + 8192;
    uint64_t *d_total = (uint64_t *)((char *)counts.p + ((size_t)nsegs * 4 + 7) / 8 * 8);
    hipStream_t s = nullptr;
    hipError_t e = gb_launch_seed(d_seed, d_nseed, s);
    if (e == hipSuccess)
        e = gb_launch_table_count(d_seed, d_nseed, T, nsegs, (uint32_t *)counts.p,
                                  (uint32_t *)stash.p, s);
    if (e == hipSuccess)
        e = gb_launch_table_scan((uint32_t *)counts.p, nsegs, d_total, s);
    if (e == hipSuccess)
        e = gb_launch_table_emit((const uint32_t *)stash.p, nsegs, (uint32_t *)counts.p,
                                 (uint32_t *)c.primes.p, s);
    uint64_t total = 0;
    if (e == hipSuccess)
        e = hipMemcpy(&total, d_total, 8, hipMemcpyDeviceToHost);
    seed.release();
    stash.release();
    if (e != hipSuccess) {
        counts.release();
        set_err("prime table build failed: %s", hipGetErrorString(e));
        release_all(c);
        return GB_EHIP;
    }
    c.T = T;
    c.nprimes = total + 1;
    if (c.nprimes > cap) {
        counts.release();
        set_err("prime table overflow (%llu > %llu)", (unsigned long long)c.nprimes,
                (unsigned long long)cap);
        release_all(c);
        return GB_EHIP;
    }
    if ((st = counts.reserve(sizeof c.pi2)) != GB_OK) {
        release_all(c);
        return st;
    }
    e = gb_launch_pow2_counts((const uint32_t *)c.primes.p, c.nprimes, (uint64_t *)counts.p, s);
    if (e == hipSuccess)
        e = hipMemcpy(c.pi2, counts.p, sizeof c.pi2, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        set_err("prime counts failed: %s", hipGetErrorString(e));
        release_all(c);
        return GB_EHIP;
    }
    const uint64_t nsmall = std::min<uint64_t>(c.nprimes, 6542);  // pi(65536)
    counts.release();
    // every table holds the primes below 2^16 (T >= 2^16): the host copy and
    // the candidate tables built from them are made once per device
    if (c.small.size() == nsmall && c.d_ctab.p && c.d_ptab.p)
        return GB_OK;
    c.small.resize(nsmall);
    e = hipMemcpy(c.small.data(), c.primes.p, nsmall * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        set_err("prime table copy failed: %s", hipGetErrorString(e));
        release_all(c);
        return GB_EHIP;
    }
    // probe candidate tables from the odd primes <= 65536, one per (segment
    // size, class r of the evens, class t3 of the multiples of 3)
    std::vector<uint32_t> tab((size_t)27 * kCandStride * 3, 0u), ptab((size_t)27 * kCandStride, 0u);
    for (int lg = 18; lg <= 20; ++lg) {
        const int64_t WC = gb_class_words(lg);
        for (int64_t r = 0; r < 3; ++r)
            for (int64_t t3 = 0; t3 < 3; ++t3) {
                const size_t base = ((size_t)(lg - 18) * 9 + (size_t)(r * 3 + t3)) * kCandStride;
                size_t e_ = 0;
                uint32_t prev = 0;
                for (size_t k = 1; k < nsmall; ++k) {
                    const uint32_t pk = c.small[k];
                    const int64_t h = pk >> 1;
                    const int64_t t = (((r - h) % 3) + 3) % 3;
                    if (t == t3)
                        continue;
                    const int64_t d = (r - h - t) / 3;                   // exact
                    const int64_t fw = d >= 0 ? d / 32 : -((-d + 31) / 32);  // floor(d / 32)
                    uint32_t *te = &tab[(base + e_) * 3];
                    const int64_t slot = (t + 2 - t3) % 3;          // stored class arrays
                    te[0] = (uint32_t)(-4 * (slot * WC + fw));
                    te[1] = (uint32_t)(d - 32 * fw);
                    te[2] = pk - prev;
                    ptab[base + e_] = pk;
                    prev = pk;
                    ++e_;
                }
            }
    }
    if ((st = c.d_ctab.reserve(tab.size() * 4)) != GB_OK ||
        (st = c.d_ptab.reserve(ptab.size() * 4)) != GB_OK) {
        release_all(c);
        return st;
    }
    e = hipMemcpy(c.d_ctab.p, tab.data(), tab.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(c.d_ptab.p, ptab.data(), ptab.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        set_err("candidate table upload failed: %s", hipGetErrorString(e));
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

struct Round {
    uint64_t seg_base = 0;    // global index of the round's first segment
    uint64_t nsegs = 0;
    uint32_t bm = 0;          // 1: primes above the bucket bound go through strike bitmaps
    uint64_t chunk_first = 0; // chunks of this round in Plan::chunks
    uint64_t nchunk = 0;
    uint64_t task_first = 0;  // fill tasks of this round in Plan::tasks
    uint64_t ntask = 0;
    uint64_t ntiles = 0;      // fill tiles (from upper bounds; extra items exit at once)
};

struct Plan {
    uint32_t H = 0;           // halo bits
    uint32_t ncand = 0;       // odd candidates probed in LDS
    uint32_t lb_count = 0;    // primes sieved inside the segment kernel
    uint64_t lb = 0;          // bucket bound: larger primes go through buckets
    uint64_t total_segs = 0;
    uint64_t total_evens = 0;
    std::vector<GbInterval> iv;       // in the caller's order
    std::vector<GbInterval> dev_iv;   // in segment order (what the kernels see)
    std::vector<uint64_t> slot;       // caller's index -> position in dev_iv
    std::vector<uint64_t> An, Bn;
    std::vector<Round> rounds;
    std::vector<GbChunk> chunks;
    std::vector<GbFillTask> tasks;
    uint64_t max_round_segs = 0;
    uint64_t max_bitmap_words = 0;
    uint32_t wcu = 0;         // class-array words per segment, (E + H)/96 + 1
    uint32_t words = 0;       // strike-bitmap words per segment, 3 * wcu
    uint32_t nv[9] = {};      // probe table entries per (r, t3) within the window
};

// pi(x) < 1.25506 x / ln x for x > 1 (Rosser and Schoenfeld 1962).
uint64_t pi_upper(uint64_t x) { return (uint64_t)(1.25506 * (double)x / std::log((double)x)) + 16; }

// Automatic strike-bitmap budget (bucket_mib = 0): a first round of
// kBucketMibFirst MiB, then rounds of kBucketMibDefault MiB.  Each round is one
// fill launch and one persistent sieve launch, each of which drains at its
// end, so few large rounds beat many small ones (a 4096-interval batch near
// 2^64: 0.218 s per launch in 512 MiB rounds, 0.188 s in one 4-16 GiB round);
// the small first round finishes the cheapest intervals of the batch early
// (median completion 24 ms instead of 141 ms, at 0.192 s per launch).  Memory
// is taken only for the segments a round holds.
// Unresolved lists of up to kRankEmitMax entries are ordered by pairwise
// ranking; longer ones by a bitmap of the evens and a scan, at most
// kEmitBitmapMaxBytes of bitmap.
constexpr uint64_t kRankEmitMax = 1ull << 16;
constexpr uint64_t kEmitBitmapMaxBytes = 8ull << 30;

constexpr uint32_t kBucketMibFirst = 512;
constexpr uint32_t kBucketMibDefault = 8192;

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
    // halo: a multiple of 96 (32-bit words of the three class arrays) reaching
    // two bits past the largest candidate's offset
    pl.H = std::max<uint32_t>(96, (hmax + 2 + 95) / 96 * 96);
    for (uint32_t k = 1; k <= pl.ncand; ++k) {
        const int64_t h = c.small[k] >> 1;
        for (int64_t r = 0; r < 3; ++r) {
            const int64_t t = (((r - h) % 3) + 3) % 3;
            for (int64_t t3 = 0; t3 < 3; ++t3)
                if (t != t3)
                    ++pl.nv[r * 3 + t3];
        }
    }
    const uint32_t lg = pr.seg_log2;
    const uint64_t E = 1ull << lg;
    const uint64_t Wbits = E + pl.H;
    // bucket bound: a prime above it strikes a window at most once or twice
    uint32_t blog = pr.bucket_log2 ? pr.bucket_log2 : lg + 4;
    if (blog > 32)
        blog = 32;
    pl.lb = blog >= 32 ? 0xFFFFFFFFull : (1ull << blog);
    pl.lb_count = (uint32_t)std::min<uint64_t>(blog >= 32 ? c.nprimes : c.pi2[blog], c.nprimes);
    const bool auto_budget = pr.bucket_mib == 0;
    const uint64_t budget = (uint64_t)(auto_budget ? kBucketMibDefault : pr.bucket_mib) << 20;
    // budget of the round being filled (the first one smaller when
    // automatic); a chunk is cut to fit the smallest round
    uint64_t round_budget = auto_budget ? std::min<uint64_t>(budget, (uint64_t)kBucketMibFirst << 20)
                                        : budget;
    const uint64_t chunk_budget = round_budget;
    pl.wcu = (uint32_t)((Wbits + 95) / 96 + 1);
    pl.words = 3 * pl.wcu;

    pl.iv.resize(k);
    pl.An.resize(k);
    pl.Bn.resize(k);
    std::vector<uint8_t> usebm(k, 0);   // the interval takes strike bitmaps
    std::vector<uint64_t> order;
    order.reserve(k);
    uint64_t evens = 0;
    for (uint64_t i = 0; i < k; ++i) {
        uint64_t a, b;
        const bool ne = normalize(AB[2 * i], AB[2 * i + 1], &a, &b);
        pl.An[i] = a;
        pl.Bn[i] = b;
        GbInterval g = {};
        g.A = a;
        if (ne) {
            const uint64_t root = isqrt_u64(b);
            if (root > c.T) {
                set_err("prime table limit %llu is below isqrt(B) = %llu for interval %llu",
                        (unsigned long long)c.T, (unsigned long long)root,
                        (unsigned long long)i);
                return GB_ERANGE;
            }
            g.nE = (b - a) / 2 + 1;
            g.nseg = (g.nE + E - 1) >> lg;
            // bitmaps only for intervals whose root is above the bound (the
            // automatic bound 2^(seg_log2+4) keeps all of [4, 10^12] in the
            // per-segment tiers)
            if (root > pl.lb && a > 2 * (uint64_t)pl.H + 2)
                usebm[i] = 1;
        }
        evens += g.nE;
        pl.iv[i] = g;
        order.push_back(i);
    }
    // segments are numbered interval by interval; intervals without bitmaps
    // come first, then the others by growing top (so that the chunks of a
    // round come by growing root, mostly, and a fill task's chunk group needs
    // about the same primes)
    std::stable_sort(order.begin(), order.end(), [&](uint64_t x, uint64_t y) {
        if (usebm[x] != usebm[y])
            return usebm[x] < usebm[y];
        return usebm[x] && pl.Bn[x] < pl.Bn[y];
    });
    uint64_t seg = 0;
    for (uint64_t i : order) {
        pl.iv[i].seg_first = seg;
        seg += pl.iv[i].nseg;
    }
    pl.total_segs = seg;
    pl.total_evens = evens;

    // rounds: first the segments without buckets, then bucketed chunks under
    // the memory budget
    uint64_t pos = 0;
    size_t oi = 0;
    {
        Round r;
        r.seg_base = 0;
        while (oi < order.size() && !usebm[order[oi]]) {
            r.nsegs += pl.iv[order[oi]].nseg;
            ++oi;
        }
        pos = r.nsegs;
        if (r.nsegs)
            pl.rounds.push_back(r);
    }
    Round cur;
    cur.seg_base = pos;
    std::vector<uint64_t> croot;   // isqrt of each chunk's top (host side)
    const uint64_t per_tile = (uint64_t)kFillThreads * kFillPerThread;
    auto close_round = [&]() {
        if (cur.nsegs) {
            // fill tasks: per prime band (2^b, 2^(b+1)] and group of
            // kFillChunks consecutive chunks of the round that reach the band
            for (uint32_t bb = blog; bb < 32; ++bb) {
                const uint64_t pf = c.pi2[bb];
                for (uint64_t g0 = 0; g0 < cur.nchunk; g0 += kFillChunks) {
                    const uint64_t g1 = std::min<uint64_t>(g0 + kFillChunks, cur.nchunk);
                    uint64_t rmax = 0;
                    for (uint64_t q = g0; q < g1; ++q)
                        rmax = std::max(rmax, croot[cur.chunk_first + q]);
                    if (rmax <= (1ull << bb))
                        continue;
                    const uint64_t pe = std::min<uint64_t>(
                        c.pi2[bb + 1], std::min<uint64_t>(pi_upper(rmax), c.nprimes));
                    if (pe <= pf)
                        continue;
                    GbFillTask t = {};
                    t.tile_first = cur.ntiles;
                    t.chunk_first = (uint32_t)g0;
                    t.nchunk = (uint32_t)(g1 - g0);
                    t.p_first = (uint32_t)pf;
                    t.np = (uint32_t)(pe - pf);
                    cur.ntiles += (t.np + per_tile - 1) / per_tile;
                    pl.tasks.push_back(t);
                    ++cur.ntask;
                }
            }
            pl.rounds.push_back(cur);
            pl.max_round_segs = std::max(pl.max_round_segs, cur.nsegs);
            pl.max_bitmap_words = std::max(pl.max_bitmap_words, cur.nsegs * (uint64_t)pl.words);
        }
        cur = Round();
        cur.seg_base = pos;
        cur.chunk_first = pl.chunks.size();
        cur.task_first = pl.tasks.size();
    };
    cur.chunk_first = pl.chunks.size();
    cur.task_first = pl.tasks.size();
    for (; oi < order.size(); ++oi) {
        const uint64_t i = order[oi];
        const GbInterval &I = pl.iv[i];
        // chunk length: a chunk's strike bitmaps fit one round within the budget
        uint64_t cmax = chunk_budget / ((uint64_t)pl.words * 4);
        if (cmax < 1) {
            set_err("bucket budget of %llu MiB is below one segment's strike bitmap",
                    (unsigned long long)(chunk_budget >> 20));
            return GB_ENOMEM;
        }
        cmax = std::min<uint64_t>(cmax, 1u << 16);
        for (uint64_t s0 = 0; s0 < I.nseg; s0 += cmax) {
            const uint64_t ns = std::min<uint64_t>(cmax, I.nseg - s0);
            GbChunk ch = {};
            ch.nseg = (uint32_t)ns;
            const uint64_t n0 = I.A + 2 * E * s0;                 // first even of the chunk
            const uint64_t last = s0 + ns - 1;
            const uint64_t nl = I.A + 2 * E * last;               // first even of its last segment
            const uint64_t cl = std::min<uint64_t>(E, I.nE - E * last);
            const uint64_t top = nl + 2 * cl - 5;                 // largest q read
            ch.Q0 = n0 - 1 - 2ull * pl.H;                         // n0 > 2H + 2 here
            ch.dmax = (top - ch.Q0) / 2;
            ch.p_root = 0;                                        // set on the device
            const uint64_t h = ch.Q0 >> 1;                        // Q0 = 2h + 1
            ch.hh = (double)h;
            ch.hl = (double)(int64_t)(h - (uint64_t)ch.hh);
            ch.sqrt_q0 = (uint32_t)isqrt_u64(ch.Q0);
            ch.q0m3 = (uint32_t)(ch.Q0 % 3);
            if (cur.nsegs && (cur.nsegs + ns) * (uint64_t)pl.words * 4 > round_budget) {
                close_round();
                if (auto_budget)
                    round_budget = budget;
            }
            cur.bm = 1;
            ch.seg_first = I.seg_first + s0;
            cur.nsegs += ns;
            pos += ns;
            ++cur.nchunk;
            pl.chunks.push_back(ch);
            croot.push_back(isqrt_u64(top));
        }
    }
    close_round();
    for (const Round &r : pl.rounds)
        pl.max_round_segs = std::max(pl.max_round_segs, r.nsegs);
    // the kernels locate a segment's interval by binary search over seg_first,
    // so they see the intervals in segment order
    pl.dev_iv.resize(k);
    pl.slot.resize(k);
    for (uint64_t j = 0; j < k; ++j) {
        pl.dev_iv[j] = pl.iv[order[j]];
        pl.slot[order[j]] = j;
    }
    return GB_OK;
}

// Device workspace of one launch sequence: where its kernels keep counters,
// descriptors, segment records, spills and results.  The library's own
// buffers fill it for gb_verify_range / gb_verify_batch; the static scratch
// array fills it for gb_verify_range_noalloc.
struct Ws {
    GbCounters *ctr = nullptr;
    unsigned long long *claims = nullptr;   // one queue head per round
    GbIvDone *done = nullptr;
    GbInterval *iv = nullptr;
    GbSegRecord *rec = nullptr;
    GbSpill *spill = nullptr;
    uint64_t spill_cap = 0;
    GbIvResult *res = nullptr;
    uint64_t *unres = nullptr;
    GbChunk *chunk = nullptr;
    GbFillTask *task = nullptr;
    uint32_t *bitmap = nullptr;
    // long unresolved lists: one bit per even, interval i from word woff[i]
    bool emit_by_bitmap = false;
    uint64_t *woff = nullptr;
    uint32_t *ubits = nullptr;
    uint64_t *ublock = nullptr;
    uint64_t ubits_words = 0;
};

Ws library_ws(const Ctx &c)
{
    Ws w;
    w.ctr = (GbCounters *)c.d_ctr.p;
    w.claims = (unsigned long long *)c.d_claims.p;
    w.done = (GbIvDone *)c.d_done.p;
    w.iv = (GbInterval *)c.d_iv.p;
    w.rec = (GbSegRecord *)c.d_rec.p;
    w.spill = (GbSpill *)c.d_spill.p;
    w.spill_cap = c.spill_cap;
    w.res = (GbIvResult *)c.d_res.p;
    w.unres = (uint64_t *)c.d_unres.p;
    w.chunk = (GbChunk *)c.d_chunk.p;
    w.task = (GbFillTask *)c.d_task.p;
    w.bitmap = (uint32_t *)c.d_bitmap.p;
    return w;
}

// The kernels of one verification, in stream order:
//   reset -> per round: [bucket reset -> bucket fill ->] persistent
//   sieve+probe -> Phase 2 -> reduce -> unresolved list.
// Every kernel reads its sizes from device memory (counters, descriptors), so
// the sequence needs no host round trip and can be captured as a graph.
gb_status enqueue_kernels(Ctx &c, const Plan &pl, uint64_t P_max, const gb_params &pr,
                          uint32_t grid, hipStream_t s, bool mark_probe, const Ws &w)
{
    const uint64_t k = pl.iv.size();
    GbCounters *ctr = w.ctr;
    unsigned long long *claims = w.claims;
    GB_HIP(gb_launch_reset(ctr, w.done, (uint32_t)k, claims, (uint32_t)pl.rounds.size(), s));
    GB_HIP(gb_launch_chunk_roots((const uint32_t *)c.primes.p, c.nprimes, w.chunk,
                                 pl.chunks.size(), s));
    if (mark_probe)
        GB_HIP(hipEventRecord(c.ev[1], s));
    for (size_t ri = 0; ri < pl.rounds.size(); ++ri) {
        const Round &r = pl.rounds[ri];
        if (r.bm) {
            GB_HIP(gb_launch_bucket_reset(w.bitmap, r.nsegs * (uint64_t)pl.words, s));
            GbBucketArgs b = {};
            b.primes = (const uint32_t *)c.primes.p;
            b.chunk = w.chunk + r.chunk_first;
            b.task = w.task + r.task_first;
            b.ntask = (uint32_t)r.ntask;
            b.log2e = pr.seg_log2;
            b.H = pl.H;
            b.words = pl.words;
            b.wcu = pl.wcu;
            b.ntiles = r.ntiles;
            b.seg_base = r.seg_base;
            b.bitmap = w.bitmap;
            if (r.ntask && r.ntiles)
                GB_HIP(gb_launch_bucket_fill(b, (uint32_t)std::min<uint64_t>(r.ntiles, 1u << 16), s));
        }
        GbProbeArgs a = {};
        a.primes = (const uint32_t *)c.primes.p;
        a.nprimes = c.nprimes;
        a.iv = w.iv;
        a.k = (uint32_t)k;
        a.H = pl.H;
        a.ncand = pl.ncand;
        a.lb_count = r.bm ? pl.lb_count : (uint32_t)c.nprimes;
        a.seg_base = r.seg_base;
        a.nsegs = r.nsegs;
        a.rec = w.rec;
        a.spill = w.spill;
        a.spill_cap = w.spill_cap;
        a.ctr = ctr;
        a.claim = claims + ri;
        a.done = w.done;
        a.bitmap = r.bm ? w.bitmap : nullptr;
        a.ctab = (const uint32_t *)c.d_ctab.p;
        a.ptab = (const uint32_t *)c.d_ptab.p;
        a.wcu = pl.wcu;
        for (int q = 0; q < 9; ++q)
            a.nv[q] = pl.nv[q];
        const uint32_t g = (uint32_t)std::min<uint64_t>(grid, r.nsegs);
        GB_HIP(gb_launch_probe((int)pr.seg_log2, (int)pr.wg_size, g, a, s));
    }
    if (mark_probe)
        GB_HIP(hipEventRecord(c.ev[2], s));
    GB_HIP(gb_launch_phase2((const uint32_t *)c.primes.p, c.nprimes, (uint64_t)pl.ncand + 1,
                            w.spill, w.spill_cap, ctr, (uint32_t)c.num_cu * 4, s));
    GB_HIP(gb_launch_reduce(w.iv, (uint32_t)k, w.rec, w.spill, w.spill_cap, ctr, P_max, w.res, s));
    if (w.emit_by_bitmap)
        GB_HIP(gb_launch_unres_bitmap(w.spill, w.spill_cap, ctr, P_max, w.iv, (uint32_t)k, w.woff,
                                      w.ubits_words, w.ubits, w.ublock, w.unres,
                                      (uint32_t)c.num_cu * 4, s));
    else
        GB_HIP(gb_launch_unres_emit(w.spill, w.spill_cap, ctr, P_max, w.unres,
                                    (uint32_t)c.num_cu * 2, s));
    return GB_OK;
}

void drop_graph(Ctx &c)
{
    if (c.graph_exec)
        (void)hipGraphExecDestroy(c.graph_exec);
    c.graph_exec = nullptr;
    c.graph_key.clear();
}

// Every value the captured sequence bakes into kernel arguments.
std::vector<uint64_t> graph_key(const Ctx &c, const Plan &pl, uint64_t P_max, const gb_params &pr,
                                uint32_t grid)
{
    std::vector<uint64_t> key = {
        (uint64_t)c.primes.p, (uint64_t)c.d_ctab.p, (uint64_t)c.d_ptab.p, (uint64_t)c.d_iv.p, (uint64_t)c.d_rec.p, (uint64_t)c.d_spill.p,
        (uint64_t)c.d_unres.p, (uint64_t)c.d_res.p, (uint64_t)c.d_ctr.p, (uint64_t)c.d_done.p,
        (uint64_t)c.d_bitmap.p, (uint64_t)pl.words, (uint64_t)c.d_chunk.p,
        (uint64_t)c.d_claims.p, (uint64_t)c.d_task.p, pl.chunks.size(), c.nprimes, pl.iv.size(),
        c.spill_cap, P_max, pl.H, pl.ncand,
        pl.lb_count, pr.seg_log2, pr.wg_size, grid, (uint64_t)c.num_cu};
    for (const Round &r : pl.rounds) {
        key.push_back(r.seg_base);
        key.push_back(r.nsegs);
        key.push_back(r.bm);
        key.push_back(r.chunk_first);
        key.push_back(r.nchunk);
        key.push_back(r.task_first);
        key.push_back(r.ntask);
        key.push_back(r.ntiles);
    }
    return key;
}

// Capture the launch sequence on the library's own stream (the legacy default
// stream cannot be captured) and instantiate it; reused while the key holds.
gb_status capture_graph(Ctx &c, const Plan &pl, uint64_t P_max, const gb_params &pr,
                        uint32_t grid, const std::vector<uint64_t> &key, const Ws &w)
{
    if (c.graph_exec && c.graph_key == key)
        return GB_OK;
    drop_graph(c);
    if (!c.cap_stream)
        GB_HIP(hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking));
    GB_HIP(hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeThreadLocal));
    gb_status st = enqueue_kernels(c, pl, P_max, pr, grid, c.cap_stream, false, w);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c.cap_stream, &graph);
    if (st != GB_OK) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) {
        set_err("graph capture failed: %s", hipGetErrorString(e));
        return GB_EHIP;
    }
    e = hipGraphInstantiate(&c.graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        c.graph_exec = nullptr;
        set_err("graph instantiation failed: %s", hipGetErrorString(e));
        return GB_EHIP;
    }
    c.graph_key = key;
    return GB_OK;
}

// Persistent grid of the sieve+probe kernel: the workgroups that fit on the
// device at once (or wg_per_cu per CU), never more than there are segments.
gb_status probe_grid(const Ctx &c, const Plan &pl, const gb_params &pr, uint32_t *grid)
{
    *grid = 0;
    if (pl.total_segs) {
        int occ = 0;
        GB_HIP(gb_probe_occupancy((int)pr.seg_log2, (int)pr.wg_size, &occ));
        if (occ < 1)
            occ = 1;
        if (pr.wg_per_cu)
            occ = std::min<int>(occ, (int)pr.wg_per_cu);
        *grid = (uint32_t)std::min<uint64_t>(pl.total_segs, (uint64_t)c.num_cu * occ);
    }
    return GB_OK;
}

// Failure injected by gb_debug_fail_next() into the next run: 1 before
// anything is enqueued, 2 after the kernels are enqueued.
std::atomic<uint32_t> g_fail_next{0};

// One pass of the launch sequence; the caller retries when a capacity
// (spill list, bucket) overflowed.  `enqueued` is set once work is on s.
gb_status run_once_impl(Ctx &c, const Plan &pl, uint64_t P_max, const gb_params &pr,
                        hipStream_t s, bool use_graph, uint64_t *spills_out, bool &enqueued)
{
    const uint32_t inject = g_fail_next.exchange(0, std::memory_order_relaxed);
    if (inject == 1) {
        set_err("failure injected before anything was enqueued (test hook)");
        return GB_EHIP;
    }
    const uint64_t k = pl.iv.size();
    const uint64_t nr = std::max<size_t>(pl.rounds.size(), 1);
    GB_TRY(c.d_iv.reserve(k * sizeof(GbInterval)));
    GB_TRY(c.d_rec.reserve(std::max<uint64_t>(pl.total_segs, 1) * sizeof(GbSegRecord)));
    GB_TRY(c.d_res.reserve(k * sizeof(GbIvResult)));
    GB_TRY(c.d_ctr.reserve(sizeof(GbCounters)));
    GB_TRY(c.d_done.reserve(k * sizeof(GbIvDone)));
    GB_TRY(c.d_claims.reserve(nr * 8));
    GB_TRY(c.d_chunk.reserve(std::max<size_t>(pl.chunks.size(), 1) * sizeof(GbChunk)));
    GB_TRY(c.h_chunk.reserve(std::max<size_t>(pl.chunks.size(), 1) * sizeof(GbChunk)));
    GB_TRY(c.d_task.reserve(std::max<size_t>(pl.tasks.size(), 1) * sizeof(GbFillTask)));
    GB_TRY(c.h_task.reserve(std::max<size_t>(pl.tasks.size(), 1) * sizeof(GbFillTask)));
    GB_TRY(c.d_bitmap.reserve(std::max<uint64_t>(pl.max_bitmap_words, 1) * 4));
    GB_TRY(c.h_iv.reserve(k * sizeof(GbInterval)));
    GB_TRY(c.h_res.reserve(k * sizeof(GbIvResult)));
    GB_TRY(c.h_ctr.reserve(sizeof(GbCounters)));
    GB_TRY(c.h_done.reserve(k * sizeof(GbIvDone)));
    GB_TRY(c.d_spill.reserve(c.spill_cap * sizeof(GbSpill)));
    GB_TRY(c.d_unres.reserve(c.spill_cap * sizeof(uint64_t)));
    Ws w = library_ws(c);
    // unresolved lists longer than the pairwise ranking handles: one bit per
    // even of each interval, then a scan
    std::vector<uint64_t> woff;
    if (c.spill_cap > kRankEmitMax) {
        woff.resize(k);
        uint64_t words = 0;
        for (uint64_t j = 0; j < k; ++j) {
            woff[j] = words;
            words += (pl.dev_iv[j].nE + 31) / 32;
        }
        if (words * 4 > kEmitBitmapMaxBytes) {
            set_err("%llu evens were left open by P_max; listing them in order needs %llu MiB "
                    "(at most %llu MiB): raise P_max or split the range",
                    (unsigned long long)c.spill_cap, (unsigned long long)(words * 4 >> 20),
                    (unsigned long long)(kEmitBitmapMaxBytes >> 20));
            return GB_ENOMEM;
        }
        GB_TRY(c.d_woff.reserve(k * 8));
        GB_TRY(c.h_woff.reserve(k * 8));
        GB_TRY(c.d_ubits.reserve(std::max<uint64_t>(words, 1) * 4));
        GB_TRY(c.d_ublock.reserve(std::max<uint64_t>(gb_unres_bitmap_blocks(words), 1) * 8));
        w.emit_by_bitmap = true;
        w.woff = (uint64_t *)c.d_woff.p;
        w.ubits = (uint32_t *)c.d_ubits.p;
        w.ublock = (uint64_t *)c.d_ublock.p;
        w.ubits_words = words;
    }
    for (auto &e : c.ev)
        if (!e)
            GB_HIP(hipEventCreate(&e));

    uint32_t grid = 0;
    GB_TRY(probe_grid(c, pl, pr, &grid));
    std::memcpy(c.h_iv.p, pl.dev_iv.data(), k * sizeof(GbInterval));
    enqueued = true;
    GB_HIP(hipMemcpyAsync(c.d_iv.p, c.h_iv.p, k * sizeof(GbInterval), hipMemcpyHostToDevice, s));
    if (w.emit_by_bitmap) {
        std::memcpy(c.h_woff.p, woff.data(), k * 8);
        GB_HIP(hipMemcpyAsync(c.d_woff.p, c.h_woff.p, k * 8, hipMemcpyHostToDevice, s));
    }
    if (!pl.chunks.empty()) {
        std::memcpy(c.h_chunk.p, pl.chunks.data(), pl.chunks.size() * sizeof(GbChunk));
        GB_HIP(hipMemcpyAsync(c.d_chunk.p, c.h_chunk.p, pl.chunks.size() * sizeof(GbChunk),
                              hipMemcpyHostToDevice, s));
    }
    if (!pl.tasks.empty()) {
        std::memcpy(c.h_task.p, pl.tasks.data(), pl.tasks.size() * sizeof(GbFillTask));
        GB_HIP(hipMemcpyAsync(c.d_task.p, c.h_task.p, pl.tasks.size() * sizeof(GbFillTask),
                              hipMemcpyHostToDevice, s));
    }
    GB_HIP(hipEventRecord(c.ev[0], s));
    if (use_graph) {
        std::vector<uint64_t> key = graph_key(c, pl, P_max, pr, grid);
        key.push_back(w.emit_by_bitmap);
        key.push_back((uint64_t)w.woff);
        key.push_back((uint64_t)w.ubits);
        key.push_back((uint64_t)w.ublock);
        key.push_back(w.ubits_words);
        GB_TRY(capture_graph(c, pl, P_max, pr, grid, key, w));
        GB_HIP(hipGraphLaunch(c.graph_exec, s));
    } else {
        GB_TRY(enqueue_kernels(c, pl, P_max, pr, grid, s, true, w));
    }
    if (inject == 2) {
        set_err("failure injected after the kernels were enqueued (test hook)");
        return GB_EHIP;
    }
    GB_HIP(hipMemcpyAsync(c.h_res.p, c.d_res.p, k * sizeof(GbIvResult), hipMemcpyDeviceToHost, s));
    GB_HIP(hipMemcpyAsync(c.h_ctr.p, c.d_ctr.p, sizeof(GbCounters), hipMemcpyDeviceToHost, s));
    GB_HIP(hipMemcpyAsync(c.h_done.p, c.d_done.p, k * sizeof(GbIvDone), hipMemcpyDeviceToHost, s));
    GB_HIP(hipEventRecord(c.ev[3], s));
    GB_HIP(hipStreamSynchronize(s));
    const GbCounters *hc = (const GbCounters *)c.h_ctr.p;
    *spills_out = hc->spills;
    float total = 0;
    GB_HIP(hipEventElapsedTime(&total, c.ev[0], c.ev[3]));
    const GbIvDone *hd = (const GbIvDone *)c.h_done.p;
    unsigned long long tmax = hc->t_start;
    for (uint64_t i = 0; i < k; ++i)
        tmax = std::max(tmax, hd[i].t_done);
    double probe = (double)(tmax - hc->t_start) / c.wall_khz;
    if (!use_graph) {
        float pm = 0;
        GB_HIP(hipEventElapsedTime(&pm, c.ev[1], c.ev[2]));
        probe = pm;
    }
    c.last_k = k;
    c.last_t_start = hc->t_start;
    gb_stats &st = c.stats;
    st.probe_ms = probe;
    st.total_ms = total;
    st.segments = pl.total_segs;
    st.evens = pl.total_evens;
    st.spills = *spills_out;
    st.grid = grid;
    st.wg_size = pr.wg_size;
    st.seg_log2 = pr.seg_log2;
    st.halo_bits = pl.H;
    st.ncand = pl.ncand;
    st.intervals = k;
    return GB_OK;
}

gb_status run_once(Ctx &c, const Plan &pl, uint64_t P_max, const gb_params &pr, hipStream_t s,
                   bool use_graph, uint64_t *spills_out)
{
    bool enqueued = false;
    const gb_status st = run_once_impl(c, pl, P_max, pr, s, use_graph, spills_out, enqueued);
    if (st != GB_OK && enqueued) {
        // a failed call returns only when none of its work is still in flight,
        // so the next call may reuse every buffer, pinned staging included
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
    }
    return st;
}

gb_status verify_many(Ctx &c, const uint64_t *AB, uint64_t k, uint64_t P_max, hipStream_t s,
                      gb_result *outs, bool use_graph)
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
    quiesce(c);
    const gb_params pr = c.params;
    if (c.spill_cap == 0)
        c.spill_cap = 1 << 16;
    Plan pl;
    uint64_t spills = 0;
    GB_TRY(make_plan(c, AB, k, P_max, pr, pl));
    // A spill list grown by an earlier call (tiny P_max) is kept, but its
    // ordered listing needs one bit per even of the batch; where that bitmap
    // would exceed its limit, this call starts from the pairwise ranking's
    // 2^16 entries and grows only if its own spills need it.
    const uint64_t grown = c.spill_cap;
    if (c.spill_cap > kRankEmitMax) {
        uint64_t words = 0;
        for (const GbInterval &g : pl.dev_iv)
            words += (g.nE + 31) / 32;
        if (words * 4 > kEmitBitmapMaxBytes)
            c.spill_cap = kRankEmitMax;
    }
    GB_TRY(run_once(c, pl, P_max, pr, s, use_graph, &spills));
    if (spills <= c.spill_cap)
        c.spill_cap = std::max(c.spill_cap, grown);
    if (spills > c.spill_cap) {
        // the count is exact (every append counts, stored or not), so one
        // rerun with room for all of them completes the call
        c.spill_cap = spills + spills / 8 + 1024;
        GB_TRY(run_once(c, pl, P_max, pr, s, use_graph, &spills));
        if (spills > c.spill_cap) {
            set_err("spill list overflowed twice (%llu entries)", (unsigned long long)spills);
            return GB_ENOMEM;
        }
    }
    const GbIvResult *res = (const GbIvResult *)c.h_res.p;
    c.last_slot = pl.slot;
    gb_status status = GB_OK;
    for (uint64_t i = 0; i < k; ++i) {
        gb_result &o = outs[i];
        const GbIvResult &r = res[pl.slot[i]];
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

// Layout of the scratch array for one call: fixed records at the start, then
// the segment records, then the spill list and the unresolved list, which
// share what the records leave.
constexpr size_t kScrCtr = 0, kScrClaim = 64, kScrDone = 128, kScrIv = 256, kScrRes = 320;
constexpr size_t kScrRec = 4096;
constexpr uint64_t kScrMinSpill = 1024;

gb_status verify_noalloc(Ctx &c, uint64_t A, uint64_t B, uint64_t P_max, hipStream_t s,
                         gb_result *out)
{
    GB_TRY(use_device(c));
    if (c.async_pending && c.ev_busy)   // order after a stream-ordered call, without waiting
        GB_HIP(hipStreamWaitEvent(s, c.ev_busy, 0));
    char *base = (char *)g_scratch[c.device];
    if (!base) {
        set_err("the no-alloc scratch of device %d was not set up", c.device);
        return GB_ENOTABLE;
    }
    gb_params pr = c.params;
    pr.bucket_log2 = 32;   // every prime is sieved inside the segment: no strike bitmaps
    Plan pl;
    const uint64_t AB[2] = {A, B};
    GB_TRY(make_plan(c, AB, 1, P_max, pr, pl));
    const uint64_t rec_bytes = (pl.total_segs * sizeof(GbSegRecord) + 255) / 256 * 256;
    const uint64_t left = kScratchBytes - kScrRec >= rec_bytes ? kScratchBytes - kScrRec - rec_bytes : 0;
    // (lists are ordered by pairwise ranking here, so at most kRankEmitMax)
    const uint64_t spill_cap =
        std::min<uint64_t>(left / (sizeof(GbSpill) + sizeof(uint64_t)), kRankEmitMax);
    if (spill_cap < kScrMinSpill) {
        set_err("range of %llu segments needs %llu bytes of segment records; the no-alloc "
                "scratch holds %llu bytes (at most %llu segments of 2^%u evens)",
                (unsigned long long)pl.total_segs, (unsigned long long)rec_bytes,
                (unsigned long long)kScratchBytes,
                (unsigned long long)((kScratchBytes - kScrRec - kScrMinSpill * 24) / sizeof(GbSegRecord)),
                pr.seg_log2);
        return GB_ENOMEM;
    }
    Ws w;
    w.ctr = (GbCounters *)(base + kScrCtr);
    w.claims = (unsigned long long *)(base + kScrClaim);
    w.done = (GbIvDone *)(base + kScrDone);
    w.iv = (GbInterval *)(base + kScrIv);
    w.res = (GbIvResult *)(base + kScrRes);
    w.rec = (GbSegRecord *)(base + kScrRec);
    w.spill = (GbSpill *)(base + kScrRec + rec_bytes);
    w.spill_cap = spill_cap;
    w.unres = (uint64_t *)(base + kScrRec + rec_bytes + spill_cap * sizeof(GbSpill));
    uint32_t grid = 0;
    GB_TRY(probe_grid(c, pl, pr, &grid));
    // the descriptor goes in as a kernel argument: no host staging buffer
    hipError_t e = gb_launch_put_interval(w.iv, pl.dev_iv[0], s);
    gb_status st = GB_OK;
    if (e != hipSuccess) {
        set_err("descriptor upload failed: %s", hipGetErrorString(e));
        st = GB_EHIP;
    }
    if (st == GB_OK)
        st = enqueue_kernels(c, pl, P_max, pr, grid, s, false, w);
    GbIvResult r = {};
    GbCounters hc = {};
    if (st == GB_OK) {
        e = hipMemcpyAsync(&r, w.res, sizeof r, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&hc, w.ctr, sizeof hc, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) {
            set_err("result copy failed: %s", hipGetErrorString(e));
            st = GB_EHIP;
        }
    }
    // nothing of this call may still run when it returns
    e = hipStreamSynchronize(s);
    if (st != GB_OK)
        return st;
    if (e != hipSuccess) {
        set_err("stream synchronization failed: %s", hipGetErrorString(e));
        return GB_EHIP;
    }
    if (hc.spills > spill_cap) {
        set_err("%llu evens left open by the probe window exceed the %llu spill entries the "
                "no-alloc scratch holds for this range (gb_verify_range has no such limit)",
                (unsigned long long)hc.spills, (unsigned long long)spill_cap);
        return GB_ENOMEM;
    }
    out->A = pl.An[0];
    out->B = pl.Bn[0];
    out->P_max = P_max;
    out->verified = r.verified;
    out->max_p = r.max_p;
    out->max_p_n = r.max_p_n;
    out->checksum = r.checksum;
    out->n_unresolved = r.n_unresolved;
    out->n_failed = r.n_failed;
    if (r.n_unresolved) {
        const uint64_t take = std::min<uint64_t>(r.n_unresolved, out->unresolved ? out->unresolved_cap : 0);
        if (take)
            GB_HIP(hipMemcpy(out->unresolved, w.unres + r.unres_first, take * 8, hipMemcpyDeviceToHost));
        if (take < r.n_unresolved) {
            set_err("unresolved list truncated (%llu > %llu)", (unsigned long long)r.n_unresolved,
                    (unsigned long long)take);
            return GB_ETRUNC;
        }
    }
    return GB_OK;
}

// Host memory the device copies can reach without staging (hipHostMalloc or
// registered memory).
bool is_pinned(const void *p)
{
    hipPointerAttribute_t at;
    const hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeHost;
}

// gb_verify_range_async: the launch sequence of gb_verify_range, enqueued on
// the caller's stream after the last call's use of the workspaces, ending in
// copies of the result image, the status word and the unresolved list to the
// caller's pinned memory.  Nothing waits on the host unless a workspace must
// grow (or staging for strike-bitmap descriptors is in use by the last call).
gb_status verify_async(Ctx &c, uint64_t A, uint64_t B, uint64_t P_max, hipStream_t s,
                       gb_result *out, int32_t *status)
{
    GB_TRY(use_device(c));
    const uint64_t cap = out->unresolved ? out->unresolved_cap : 0;
    if (!is_pinned(out) || !is_pinned(status) || (cap && !is_pinned(out->unresolved))) {
        set_err("gb_verify_range_async needs pinned host memory for out, status and "
                "out->unresolved (hipHostMalloc)");
        return GB_EINVAL;
    }
    const gb_params pr = c.params;
    if (c.spill_cap == 0)
        c.spill_cap = 1 << 16;
    Plan pl;
    const uint64_t AB[2] = {A, B};
    GB_TRY(make_plan(c, AB, 1, P_max, pr, pl));
    const size_t need_rec = std::max<uint64_t>(pl.total_segs, 1) * sizeof(GbSegRecord);
    const size_t need_bm = std::max<uint64_t>(pl.max_bitmap_words, 1) * 4;
    const size_t need_chunk = std::max<size_t>(pl.chunks.size(), 1) * sizeof(GbChunk);
    const size_t need_task = std::max<size_t>(pl.tasks.size(), 1) * sizeof(GbFillTask);
    const bool grows = need_rec > c.d_rec.bytes || need_bm > c.d_bitmap.bytes ||
                       need_chunk > c.d_chunk.bytes || need_task > c.d_task.bytes ||
                       !c.d_iv.p || !c.d_spill.p || !c.d_async.p;
    if (grows || !pl.chunks.empty())
        quiesce(c);
    GB_TRY(c.d_iv.reserve(sizeof(GbInterval)));
    GB_TRY(c.d_rec.reserve(need_rec));
    GB_TRY(c.d_res.reserve(sizeof(GbIvResult)));
    GB_TRY(c.d_ctr.reserve(sizeof(GbCounters)));
    GB_TRY(c.d_done.reserve(sizeof(GbIvDone)));
    GB_TRY(c.d_claims.reserve(std::max<size_t>(pl.rounds.size(), 1) * 8));
    GB_TRY(c.d_chunk.reserve(need_chunk));
    GB_TRY(c.h_chunk.reserve(need_chunk));
    GB_TRY(c.d_task.reserve(need_task));
    GB_TRY(c.h_task.reserve(need_task));
    GB_TRY(c.d_bitmap.reserve(need_bm));
    GB_TRY(c.d_spill.reserve(c.spill_cap * sizeof(GbSpill)));
    GB_TRY(c.d_unres.reserve(c.spill_cap * sizeof(uint64_t)));
    GB_TRY(c.d_async.reserve(128));
    if (!c.ev_busy)
        GB_HIP(hipEventCreateWithFlags(&c.ev_busy, hipEventDisableTiming));
    uint32_t grid = 0;
    GB_TRY(probe_grid(c, pl, pr, &grid));
    if (c.async_pending)
        GB_HIP(hipStreamWaitEvent(s, c.ev_busy, 0));
    GB_HIP(gb_launch_put_interval((GbInterval *)c.d_iv.p, pl.dev_iv[0], s));
    if (!pl.chunks.empty()) {
        std::memcpy(c.h_chunk.p, pl.chunks.data(), pl.chunks.size() * sizeof(GbChunk));
        GB_HIP(hipMemcpyAsync(c.d_chunk.p, c.h_chunk.p, pl.chunks.size() * sizeof(GbChunk),
                              hipMemcpyHostToDevice, s));
        std::memcpy(c.h_task.p, pl.tasks.data(), pl.tasks.size() * sizeof(GbFillTask));
        GB_HIP(hipMemcpyAsync(c.d_task.p, c.h_task.p, pl.tasks.size() * sizeof(GbFillTask),
                              hipMemcpyHostToDevice, s));
    }
    // unresolved lists are ordered by pairwise ranking on this path, so the
    // spill list used is at most kRankEmitMax entries long
    Ws w = library_ws(c);
    w.spill_cap = std::min<uint64_t>(c.spill_cap, kRankEmitMax);
    GB_TRY(enqueue_kernels(c, pl, P_max, pr, grid, s, false, w));
    GB_HIP(gb_launch_finalize((const GbIvResult *)c.d_res.p, (const GbCounters *)c.d_ctr.p,
                              w.spill_cap, pl.An[0], pl.Bn[0], P_max, out->unresolved,
                              out->unresolved_cap, c.d_async.p, s));
    GB_HIP(hipMemcpyAsync(out, c.d_async.p, sizeof(gb_result), hipMemcpyDeviceToHost, s));
    GB_HIP(hipMemcpyAsync(status, (const char *)c.d_async.p + kFinalizeStatusOffset, 4,
                          hipMemcpyDeviceToHost, s));
    const uint64_t take = std::min<uint64_t>(cap, w.spill_cap);
    if (take)
        GB_HIP(hipMemcpyAsync(out->unresolved, c.d_unres.p, take * 8, hipMemcpyDeviceToHost, s));
    GB_HIP(hipEventRecord(c.ev_busy, s));
    c.async_pending = true;
    return GB_OK;
}

// ---- verification past 2^64 ----

typedef unsigned __int128 u128h;   // host-side 128-bit integers

u128h to_u128(uint64_t lo, uint64_t hi) { return ((u128h)hi << 64) | lo; }

constexpr uint64_t kWideSpillCap = 1ull << 16;   // the reduce ranks spills pairwise
constexpr uint64_t kWideMaxEvens = 1ull << 40;
constexpr uint32_t kWideSieveLog2 = 28;           // sieve bound S = min(T, 2^28)

// Every even of [A, B] with A >= 2^64 (normalized, A <= B), by the wide
// kernels; fields of *out other than the unresolved buffer are written.
gb_status verify_wide_part(Ctx &c, u128h A, u128h B, uint64_t P_max, hipStream_t s,
                           gb_result128 *out, std::vector<u128h> &unres)
{
    const u128h nE128 = (B - A) / 2 + 1;
    if (nE128 > kWideMaxEvens) {
        set_err("a range past 2^64 may hold at most 2^40 evens per call");
        return GB_EINVAL;
    }
    const uint64_t nE = (uint64_t)nE128;
    const uint64_t pc = std::min<uint64_t>(P_max, 65536);
    const uint64_t nc = small_count_le(c, pc);
    const uint32_t ncand = (uint32_t)(nc > 0 ? nc - 1 : 0);
    const uint32_t hmax = ncand ? (c.small[ncand] - 1) / 2 : 0;
    // the probe reads 32 strikes below bit(n - p) at once: 32 bits of halo more
    const uint32_t H = (hmax + 32 + 31) / 32 * 32;
    const uint64_t nsieve = c.T >= (1ull << kWideSieveLog2) ? c.pi2[kWideSieveLog2] : c.nprimes;
    const uint64_t chunk = 1ull << c.wide_chunk_log2;
    const uint64_t nchunks = (nE + chunk - 1) / chunk;
    uint32_t occ[6] = {0, 0, 0, 0, 0, 0};   // probe blocks per CU by limb count
    for (int l = 3; l <= 5; ++l)
        occ[l] = (uint32_t)gb_wide_occupancy(l);
    const uint32_t nrec = (uint32_t)c.num_cu * std::max(occ[3], std::max(occ[4], occ[5]));
    const uint64_t max_words = (std::min<uint64_t>(nE, chunk) + H + 31) / 32 + 1;   // + a spare
    GB_TRY(c.d_wrec.reserve((uint64_t)nrec * sizeof(GbWideRecord)));
    GB_TRY(c.d_wspill.reserve(kWideSpillCap * sizeof(GbWideSpill)));
    GB_TRY(c.d_wunres.reserve(kWideSpillCap * sizeof(u128w)));
    GB_TRY(c.d_wres.reserve(sizeof(GbWideResult)));
    GB_TRY(c.d_wctr.reserve(64));
    GB_TRY(c.d_wbits.reserve(max_words * 4));
    GB_TRY(c.h_wres.reserve(sizeof(GbWideResult)));
    for (auto &e : c.ev)
        if (!e)
            GB_HIP(hipEventCreate(&e));
    GbWideArgs a = {};
    a.primes = (const uint32_t *)c.primes.p;
    a.nprimes = c.nprimes;
    a.nsieve = (uint32_t)nsieve;
    a.ncand = ncand;
    a.H = H;
    a.hmax = hmax;
    // primes[1 ..) below 2^16 and below 2^12 (every table holds the primes below 2^16)
    a.nsmall = (uint32_t)std::min<uint64_t>(nsieve, small_count_le(c, 65535));
    a.ncoop = (uint32_t)std::min<uint64_t>(a.nsmall, small_count_le(c, 4095));
    a.nrec = nrec;
    a.A.lo = (uint64_t)A;
    a.A.hi = (uint64_t)(A >> 64);
    a.nE = nE;
    a.rec = (GbWideRecord *)c.d_wrec.p;
    a.spill = (GbWideSpill *)c.d_wspill.p;
    a.spill_cap = kWideSpillCap;
    a.ctr = (unsigned long long *)c.d_wctr.p;
    const uint32_t fill_grid =
        nsieve > a.nsmall ? (uint32_t)std::min<uint64_t>((nsieve - a.nsmall + 255) / 256,
                                                         (uint64_t)c.num_cu * 8)
                          : 0;
    uint32_t grid_max = 0;
    gb_status st = GB_OK;
    auto launch = [&]() -> gb_status {
        GB_HIP(hipEventRecord(c.ev[0], s));
        GB_HIP(gb_launch_wide_reset(a, s));
        GB_HIP(hipEventRecord(c.ev[1], s));
        for (uint64_t ci = 0; ci < nchunks; ++ci) {
            GbWideChunk ch = {};
            const uint64_t i0 = ci * chunk;
            ch.cnt = (uint32_t)std::min<uint64_t>(chunk, nE - i0);
            ch.nbits = ch.cnt + H;
            const u128h n0 = A + 2 * (u128h)i0;
            const u128h q0 = n0 - 1 - 2 * (u128h)H;   // n0 >= 2^64: no wrap
            ch.n0.lo = (uint64_t)n0;
            ch.n0.hi = (uint64_t)(n0 >> 64);
            ch.qlo.lo = (uint64_t)q0;
            ch.qlo.hi = (uint64_t)(q0 >> 64);
            ch.bits = (uint32_t *)c.d_wbits.p;
            // lanes to gather before a Lucas round: the more of the survivors
            // are composite (larger n), the sooner (a model of the rounds)
            ch.lucas_at = (n0 >> 80) ? 56 : 60;
            const uint64_t words = (ch.nbits + 31) / 32;
            const uint32_t sieve_grid = (uint32_t)std::min<uint64_t>(
                (words + kWideSieveWords - 1) / kWideSieveWords, (uint64_t)c.num_cu * 8);
            // the fewest 28-bit limbs that keep every q of the chunk (q < the
            // chunk's last n) 12 bits below R = 2^(28 limbs)
            const u128h nlast = n0 + 2 * (u128h)(ch.cnt - 1);
            const int nbits_last = (nlast >> 64) ? 128 - __builtin_clzll((uint64_t)(nlast >> 64))
                                                 : 64 - __builtin_clzll((uint64_t)nlast);
            const int limbs = nbits_last <= 72 ? 3 : (nbits_last <= 100 ? 4 : 5);
            // a block takes 512 evens at once (two per lane): no more blocks
            // than that fills, so that a short chunk launches no idle ones
            const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)c.num_cu * occ[limbs],
                                                               (ch.cnt + 511) / 512);
            grid_max = std::max(grid_max, grid);
            GB_HIP(gb_launch_wide_chunk(a, ch, sieve_grid, fill_grid, limbs, grid, s));
        }
        GB_HIP(hipEventRecord(c.ev[2], s));
        GB_HIP(gb_launch_wide_phase2(a, (uint32_t)c.num_cu * 4, s));
        GB_HIP(gb_launch_wide_reduce(a, P_max, (GbWideResult *)c.d_wres.p, (u128w *)c.d_wunres.p, s));
        GB_HIP(hipMemcpyAsync(c.h_wres.p, c.d_wres.p, sizeof(GbWideResult), hipMemcpyDeviceToHost, s));
        GB_HIP(hipEventRecord(c.ev[3], s));
        return GB_OK;
    };
    st = launch();
    const hipError_t se = hipStreamSynchronize(s);
    if (st != GB_OK)
        return st;
    GB_HIP(se);
    const GbWideResult &r = *(const GbWideResult *)c.h_wres.p;
    if (r.spills > kWideSpillCap) {
        set_err("%llu evens past 2^64 were left open by the candidates p <= %llu; at most %llu "
                "are supported per call (raise P_max or split the range)",
                (unsigned long long)r.spills, (unsigned long long)P_max,
                (unsigned long long)kWideSpillCap);
        return GB_ENOMEM;
    }
    float tot = 0, pm = 0;
    GB_HIP(hipEventElapsedTime(&tot, c.ev[0], c.ev[3]));
    GB_HIP(hipEventElapsedTime(&pm, c.ev[1], c.ev[2]));
    gb_stats &stt = c.stats;
    stt = gb_stats{};
    stt.probe_ms = pm;
    stt.total_ms = tot;
    stt.segments = nchunks;
    stt.evens = nE;
    stt.spills = r.spills;
    stt.grid = grid_max;
    stt.wg_size = kWideThreads;
    stt.seg_log2 = c.wide_chunk_log2;
    stt.halo_bits = H;
    stt.ncand = ncand;
    stt.intervals = 1;
    c.last_k = 0;
    out->verified = r.verified;
    out->checksum = r.checksum;
    out->max_p = r.max_p;
    out->max_p_n_lo = r.max_n_lo;
    out->max_p_n_hi = r.max_n_hi;
    out->n_unresolved = r.n_unresolved;
    out->n_failed = r.n_failed;
    unres.clear();
    if (r.n_unresolved) {
        std::vector<u128w> tmp(r.n_unresolved);
        GB_HIP(hipMemcpy(tmp.data(), c.d_wunres.p, r.n_unresolved * sizeof(u128w),
                         hipMemcpyDeviceToHost));
        for (const u128w &v : tmp)
            unres.push_back(to_u128(v.lo, v.hi));
    }
    return GB_OK;
}

gb_status verify_u128(Ctx &c, u128h A, u128h B, uint64_t P_max, hipStream_t s, gb_result128 *out)
{
    GB_TRY(use_device(c));
    quiesce(c);
    if (P_max < 2) {
        set_err("P_max must be >= 2 (got %llu)", (unsigned long long)P_max);
        return GB_EINVAL;
    }
    if (P_max > c.T) {
        set_err("P_max %llu exceeds the prime table limit %llu", (unsigned long long)P_max,
                (unsigned long long)c.T);
        return GB_ERANGE;
    }
    const u128h top = ~(u128h)0;
    gb_result128 r = {};
    r.P_max = P_max;
    bool empty = false;
    if (A & 1) {
        if (A == top)
            empty = true;
        else
            A += 1;
    }
    if (A < 4)
        A = 4;
    B &= ~(u128h)1;
    r.A_lo = empty ? ~0ull : (uint64_t)A;
    r.A_hi = empty ? ~0ull : (uint64_t)(A >> 64);
    r.B_lo = (uint64_t)B;
    r.B_hi = (uint64_t)(B >> 64);
    std::vector<u128h> list;
    gb_status status = GB_OK;
    if (!empty && A <= B) {
        const u128h two64 = (u128h)1 << 64;
        if (A < two64) {
            // the part below 2^64 goes through the 64-bit path
            const uint64_t b64 = B < two64 ? (uint64_t)B : ~1ull;   // 2^64 - 2
            std::vector<uint64_t> lo_list(1 << 16);
            gb_result lr = {};
            lr.unresolved = lo_list.data();
            lr.unresolved_cap = lo_list.size();
            const uint64_t AB[2] = {(uint64_t)A, b64};
            gb_status ls = verify_many(c, AB, 1, P_max, s, &lr, false);
            if (ls == GB_ETRUNC) {
                lo_list.resize(lr.n_unresolved);
                lr.unresolved = lo_list.data();
                lr.unresolved_cap = lo_list.size();
                ls = verify_many(c, AB, 1, P_max, s, &lr, false);
            }
            GB_TRY(ls);
            r.verified = lr.verified;
            r.checksum = lr.checksum;
            r.max_p = lr.max_p;
            r.max_p_n_lo = lr.max_p_n;
            r.max_p_n_hi = 0;
            r.n_unresolved = lr.n_unresolved;
            r.n_failed = lr.n_failed;
            for (uint64_t i = 0; i < lr.n_unresolved; ++i)
                list.push_back(lo_list[i]);
        }
        if (B >= two64) {
            const u128h a2 = A < two64 ? two64 : A;
            gb_result128 hr = {};
            std::vector<u128h> hl;
            GB_TRY(verify_wide_part(c, a2, B, P_max, s, &hr, hl));
            // merge: the high part's evens all lie above the low part's
            r.verified += hr.verified;
            r.checksum += hr.checksum;
            if (hr.max_p > r.max_p) {
                r.max_p = hr.max_p;
                r.max_p_n_lo = hr.max_p_n_lo;
                r.max_p_n_hi = hr.max_p_n_hi;
            }
            r.n_unresolved += hr.n_unresolved;
            r.n_failed += hr.n_failed;
            list.insert(list.end(), hl.begin(), hl.end());
        }
    }
    const uint64_t take = std::min<uint64_t>(list.size(), out->unresolved ? out->unresolved_cap : 0);
    for (uint64_t i = 0; i < take; ++i) {
        out->unresolved[2 * i] = (uint64_t)list[i];
        out->unresolved[2 * i + 1] = (uint64_t)(list[i] >> 64);
    }
    if (take < list.size()) {
        status = GB_ETRUNC;
        set_err("unresolved list truncated (%llu > %llu)", (unsigned long long)list.size(),
                (unsigned long long)take);
    }
    r.unresolved = out->unresolved;
    r.unresolved_cap = out->unresolved_cap;
    *out = r;
    return status;
}

}  // namespace

void gb_internal_set_error(const char *msg) { g_err = msg ? msg : ""; }

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
    return verify_many(c, AB, 1, P_max, (hipStream_t)stream, out, false);
}

gb_status gb_verify_batch(const uint64_t *AB, uint64_t k, uint64_t P_max, void *stream,
                          gb_result *outs)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    return verify_many(c, AB, k, P_max, (hipStream_t)stream, outs, true);
}

gb_status gb_verify_range_noalloc(uint64_t A, uint64_t B, uint64_t P_max, void *stream,
                                  gb_result *out)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if (!out) {
        set_err("null result");
        return GB_EINVAL;
    }
    return verify_noalloc(c, A, B, P_max, (hipStream_t)stream, out);
}

gb_status gb_verify_range_async(uint64_t A, uint64_t B, uint64_t P_max, void *stream,
                                gb_result *out, int32_t *status)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if (!out || !status) {
        set_err("null result or status");
        return GB_EINVAL;
    }
    return verify_async(c, A, B, P_max, (hipStream_t)stream, out, status);
}

gb_status gb_verify_range_u128(uint64_t A_lo, uint64_t A_hi, uint64_t B_lo, uint64_t B_hi,
                               uint64_t P_max, void *stream, gb_result128 *out)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if (!out) {
        set_err("null result");
        return GB_EINVAL;
    }
    return verify_u128(c, to_u128(A_lo, A_hi), to_u128(B_lo, B_hi), P_max, (hipStream_t)stream, out);
}

gb_status gb_is_prime_u128(const uint64_t *q, uint64_t count, uint8_t *is_prime, void *stream)
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
    GB_HIP(gb_launch_bpsw((const u128w *)q, count, is_prime, (hipStream_t)stream));
    GB_HIP(hipStreamSynchronize((hipStream_t)stream));
    return GB_OK;
}

gb_status gb_set_allocator(gb_alloc_fn alloc, gb_free_fn free_, void *user)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if ((alloc == nullptr) != (free_ == nullptr)) {
        set_err("gb_set_allocator needs both functions, or neither (hipMalloc / hipFree)");
        return GB_EINVAL;
    }
    if (c.device >= 0)
        (void)hipSetDevice(c.device);
    // every buffer goes back to the allocator that gave it
    release_all(c);
    g_alloc.alloc = alloc;
    g_alloc.free_ = free_;
    g_alloc.user = alloc ? user : nullptr;
    return GB_OK;
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

gb_status gb_set_wide_chunk_log2(uint32_t log2)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if (log2 < kWideChunkLog2Min || log2 > kWideChunkLog2Max) {
        set_err("the chunk size past 2^64 must be 2^%u .. 2^%u evens (got 2^%u)",
                kWideChunkLog2Min, kWideChunkLog2Max, log2);
        return GB_EINVAL;
    }
    c.wide_chunk_log2 = log2;
    return GB_OK;
}

gb_status gb_get_wide_chunk_log2(uint32_t *log2)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if (!log2) {
        set_err("null output");
        return GB_EINVAL;
    }
    *log2 = c.wide_chunk_log2;
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

namespace {

// Time verify_many over the given intervals under each launch shape (and
// strike-bitmap bound when `bounds` holds more than one) and keep the fastest.
gb_status tune(Ctx &c, const uint64_t *AB, uint64_t k, uint64_t P_max, hipStream_t s,
               const std::vector<uint32_t> &bounds, bool rel_bounds, gb_params *best)
{
    const gb_params saved = c.params;
    const uint32_t logs[3] = {18, 19, 20};
    const uint32_t wgs[3] = {256, 512, 1024};
    const uint32_t wins[3] = {4096, 16384, 65536};   // the probe windows 2^12, 2^14, 2^16
    double best_t = 1e300;
    gb_params best_p = saved;
    std::vector<gb_result> out(k);
    for (uint32_t lg : logs)
        for (uint32_t wg : wgs)
            for (uint32_t win : wins)
                for (uint32_t bd : bounds) {
                    const uint32_t blog = rel_bounds && bd ? lg + bd : bd;
                    gb_params p = {lg, wg, win, 0, blog, saved.bucket_mib};
                    int occ = 0;
                    if (gb_probe_occupancy((int)lg, (int)wg, &occ) != hipSuccess || occ < 1) {
                        (void)hipGetLastError();
                        continue;
                    }
                    c.params = p;
                    double tmin = 1e300;
                    for (int rep = 0; rep < 3; ++rep) {   // the fastest of three runs
                        const auto t0 = std::chrono::steady_clock::now();
                        gb_status st = verify_many(c, AB, k, P_max, s, out.data(), false);
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

}  // namespace

// floor(log2(x)) for x >= 1 (0 for 0): the size classes of the tuner cache.
uint64_t log2_floor(uint64_t x) { return x ? 63 - (uint64_t)__builtin_clzll(x) : 0; }

// A cached choice for `key`, applied as the current parameters.
bool tune_cached(Ctx &c, const std::vector<uint64_t> &key, gb_params *best)
{
    const auto it = c.tuned.find(key);
    if (it == c.tuned.end())
        return false;
    c.params = it->second;
    if (best)
        *best = it->second;
    return true;
}

gb_status gb_autotune(uint64_t A, uint64_t B, uint64_t P_max, void *stream, gb_params *best)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    GB_TRY(use_device(c));
    uint64_t An, Bn;
    if (!normalize(A, B, &An, &Bn) || (Bn - An) / 2 + 1 > (1ull << 36)) {
        set_err("calibration range must be non-empty and hold at most 2^36 evens");
        return GB_EINVAL;
    }
    const std::vector<uint64_t> key = {(uint64_t)c.device, 0, P_max, log2_floor(Bn),
                                       log2_floor((Bn - An) / 2 + 1)};
    if (tune_cached(c, key, best))
        return GB_OK;
    // the bucket bound matters only when the range reaches primes above the
    // smallest automatic bound, 2^22
    std::vector<uint32_t> bounds = {c.params.bucket_log2};
    if (isqrt_u64(Bn) > (1ull << 22))
        bounds = {0, 32};
    const uint64_t AB[2] = {A, B};
    gb_params chosen;
    GB_TRY(tune(c, AB, 1, P_max, (hipStream_t)stream, bounds, false, &chosen));
    c.tuned[key] = chosen;
    if (best)
        *best = chosen;
    return GB_OK;
}

gb_status gb_autotune_cache_clear(void)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    c.tuned.clear();
    return GB_OK;
}

gb_status gb_autotune_batch(const uint64_t *AB, uint64_t k, uint64_t P_max, void *stream,
                            gb_params *best)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    GB_TRY(use_device(c));
    if (k == 0 || !AB) {
        set_err("calibration batch must hold at least one interval");
        return GB_EINVAL;
    }
    uint64_t evens = 0, top = 0;
    for (uint64_t i = 0; i < k; ++i) {
        uint64_t An, Bn;
        if (normalize(AB[2 * i], AB[2 * i + 1], &An, &Bn)) {
            evens += (Bn - An) / 2 + 1;
            top = std::max(top, Bn);
        }
    }
    if (evens == 0 || evens > (1ull << 36)) {
        set_err("calibration batch must hold between 1 and 2^36 evens");
        return GB_EINVAL;
    }
    const std::vector<uint64_t> key = {(uint64_t)c.device, 1, P_max, log2_floor(k),
                                       log2_floor(evens), log2_floor(top)};
    if (tune_cached(c, key, best))
        return GB_OK;
    // automatic bound, and bounds 2^(seg_log2 + 3) and 2^(seg_log2 + 5)
    const std::vector<uint32_t> bounds = {0, 3, 5};
    gb_params chosen;
    GB_TRY(tune(c, AB, k, P_max, (hipStream_t)stream, bounds, true, &chosen));
    c.tuned[key] = chosen;
    if (best)
        *best = chosen;
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

gb_status gb_debug_fail_next(uint32_t where)
{
    if (where > 2) {
        set_err("gb_debug_fail_next: where must be 0, 1 or 2 (got %u)", where);
        return GB_EINVAL;
    }
    g_fail_next.store(where, std::memory_order_relaxed);
    g_err.clear();
    return GB_OK;
}

gb_status gb_last_stats(gb_stats *out)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if (!out) {
        set_err("null stats");
        return GB_EINVAL;
    }
    *out = c.stats;
    return GB_OK;
}

gb_status gb_last_latencies(double *ms, uint64_t k)
{
    Ctx &c = ctx();
    std::lock_guard<std::mutex> lk(c.mu);
    g_err.clear();
    if (!ms || k != c.last_k || !c.h_done.p) {
        set_err("latency buffer must hold exactly the last call's %llu intervals",
                (unsigned long long)c.last_k);
        return GB_EINVAL;
    }
    const GbIvDone *hd = (const GbIvDone *)c.h_done.p;
    for (uint64_t i = 0; i < k; ++i) {
        const uint64_t j = i < c.last_slot.size() ? c.last_slot[i] : i;
        ms[i] = hd[j].t_done ? (double)(hd[j].t_done - c.last_t_start) / c.wall_khz : 0.0;
    }
    return GB_OK;
}

const char *gb_last_error(void) { return g_err.c_str(); }

}  // extern "C"
