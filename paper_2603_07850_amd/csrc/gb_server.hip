// gb_server.hip -- the served form: a request loop with continuous batching.
//
// Requests (verification intervals) are submitted at any time from any
// thread.  A server thread admits them into a bounded set of active requests
// while their HBM reservations fit the budget, and runs ticks: every tick cuts
// the next piece (a run of segments) off each active request and verifies all
// pieces in one batched launch (gb_verify_batch: one persistent kernel over
// every piece, captured as a graph).  Requests that arrive while a tick is on
// the GPU join the next tick, so work of many requests overlaps on the device.
// A request's pieces are taken in ascending n and their aggregates merge
// associatively (wrapping sums, max with the smallest-n tie, concatenated
// unresolved lists), so the result is the same as verifying the request
// alone; the tests check exactly that.  Latency is measured from submission
// to the moment the result is visible to gb_server_poll.
//
// Host code only: the computation is the library's own batched path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "goldbach.h"
#include "gb_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    uint64_t id = 0;
    uint64_t A = 0, B = 0;       // as submitted
    uint64_t An = 0, Bn = 0;     // normalized
    uint64_t nE = 0;             // evens in the request
    uint64_t done_evens = 0;     // evens already handed to ticks
    uint64_t reserve = 0;        // HBM bytes reserved while active
    Clock::time_point t_submit;
    double latency_ms = 0;
    gb_status status = GB_OK;
    // merged aggregates
    uint64_t verified = 0, max_p = 0, max_p_n = 0, checksum = 0, n_unres = 0, n_failed = 0;
    std::vector<uint64_t> unres;
};

bool normalize_range(uint64_t A, uint64_t B, uint64_t *An, uint64_t *Bn)
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

}  // namespace

struct gb_server {
    gb_server_config cfg;
    uint64_t seg_evens = 1ull << 18;
    uint32_t lb_log2 = 19;      // bucket bound of the library's parameters
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> pending;
    std::vector<Req *> active;
    std::deque<Req *> finished;
    uint64_t next_id = 1;
    uint64_t reserved = 0;
    bool stop = false;
    std::thread th;
    hipStream_t stream = nullptr;
    gb_server_stats stats = {};
    std::string err;
    Clock::time_point t_open;
};

namespace {

// HBM reserved by a request while it is active: the strike bitmaps of one of
// its pieces when its range reaches primes above the bucket bound (a window
// of E + H <= E + 32832 bits per segment, in three class arrays), plus its
// segment records.
uint64_t reservation(const gb_server *s, const Req *r)
{
    const uint64_t segs = std::min<uint64_t>((r->nE + s->seg_evens - 1) / s->seg_evens,
                                             s->cfg.piece_segments);
    const bool big = std::sqrt((double)r->Bn) > std::ldexp(1.0, (int)s->lb_log2);
    return (big ? segs * ((s->seg_evens + 32832) / 8 + 32) : 0) + segs * 64 + 4096;
}

void finish(gb_server *s, Req *r, Clock::time_point now)
{
    r->latency_ms = std::chrono::duration<double, std::milli>(now - r->t_submit).count();
    s->reserved -= r->reserve;
    s->finished.push_back(r);
    s->stats.completed++;
    s->stats.completed_evens += r->nE;
}

void server_loop(gb_server *s)
{
    std::vector<uint64_t> AB;
    std::vector<gb_result> outs;
    std::vector<std::vector<uint64_t>> bufs;
    std::vector<Req *> owners;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                // admission: free slots and HBM budget
                while (!s->stop && !s->pending.empty() && s->active.size() < s->cfg.max_active) {
                    Req *r = s->pending.front();
                    if (!s->active.empty() && s->reserved + r->reserve > s->cfg.hbm_budget_bytes)
                        break;
                    s->pending.pop_front();
                    s->reserved += r->reserve;
                    s->active.push_back(r);
                    s->stats.admitted++;
                }
                if (!s->active.empty() || s->stop)
                    break;
                s->cv_work.wait(lk);
            }
            if (s->stop && s->active.empty())
                return;
            // one piece per active request, oldest first
            AB.clear();
            owners.clear();
            for (Req *r : s->active) {
                const uint64_t left = r->nE - r->done_evens;
                const uint64_t take = std::min<uint64_t>(left, s->cfg.piece_segments * s->seg_evens);
                const uint64_t a = r->An + 2 * r->done_evens;
                AB.push_back(a);
                AB.push_back(a + 2 * (take - 1));
                r->done_evens += take;
                owners.push_back(r);
            }
        }
        const size_t k = owners.size();
        outs.assign(k, gb_result{});
        bufs.resize(k);
        for (size_t i = 0; i < k; ++i) {
            bufs[i].resize(1024);
            outs[i].unresolved = bufs[i].data();
            outs[i].unresolved_cap = bufs[i].size();
        }
        const auto t0 = Clock::now();
        gb_status st = gb_verify_batch(AB.data(), k, s->cfg.P_max, s->stream, outs.data());
        if (st == GB_ETRUNC) {
            // a piece had more unresolved n than its buffer: verify it alone again
            st = GB_OK;
            for (size_t i = 0; i < k && st == GB_OK; ++i)
                if (outs[i].n_unresolved > outs[i].unresolved_cap) {
                    bufs[i].resize(outs[i].n_unresolved);
                    outs[i].unresolved = bufs[i].data();
                    outs[i].unresolved_cap = bufs[i].size();
                    st = gb_verify_range(AB[2 * i], AB[2 * i + 1], s->cfg.P_max, s->stream, &outs[i]);
                }
        }
        const auto t1 = Clock::now();
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.ticks++;
        s->stats.busy_ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
        if (st != GB_OK)
            s->err = gb_last_error();
        for (size_t i = 0; i < k; ++i) {
            Req *r = owners[i];
            const gb_result &o = outs[i];
            if (st != GB_OK) {
                r->status = st;
            } else {
                r->verified += o.verified;
                r->checksum += o.checksum;
                r->n_failed += o.n_failed;
                if (o.max_p > r->max_p || (o.max_p == r->max_p && o.max_p && o.max_p_n < r->max_p_n)) {
                    r->max_p = o.max_p;
                    r->max_p_n = o.max_p_n;
                }
                r->unres.insert(r->unres.end(), bufs[i].begin(),
                                bufs[i].begin() + std::min<uint64_t>(o.n_unresolved, o.unresolved_cap));
                r->n_unres += o.n_unresolved;
            }
        }
        // retire complete (or failed) requests
        auto it = s->active.begin();
        while (it != s->active.end()) {
            Req *r = *it;
            if (r->done_evens >= r->nE || r->status != GB_OK) {
                finish(s, r, t1);
                it = s->active.erase(it);
            } else {
                ++it;
            }
        }
        s->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

gb_status gb_server_open(const gb_server_config *cfg, gb_server **out)
{
    if (!cfg || !out || cfg->max_active == 0 || cfg->piece_segments == 0 || cfg->P_max < 2) {
        gb_internal_set_error("server: null argument, zero slots or piece size, or P_max < 2");
        return GB_EINVAL;
    }
    if (gb_table_limit() == 0) {
        gb_internal_set_error("server: no prime table (call gb_base_primes first)");
        return GB_ENOTABLE;
    }
    if (cfg->P_max > gb_table_limit()) {
        gb_internal_set_error("server: P_max exceeds the prime table limit");
        return GB_ERANGE;
    }
    gb_params p;
    gb_get_params(&p);
    gb_server *s = new gb_server();
    s->cfg = *cfg;
    s->seg_evens = 1ull << p.seg_log2;
    s->lb_log2 = p.bucket_log2 ? p.bucket_log2 : p.seg_log2 + 4;
    s->t_open = Clock::now();
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        gb_internal_set_error("server: stream creation failed");
        return GB_EHIP;
    }
    s->th = std::thread(server_loop, s);
    *out = s;
    return GB_OK;
}

gb_status gb_server_submit(gb_server *s, uint64_t A, uint64_t B, uint64_t *id)
{
    if (!s)
        return GB_EINVAL;
    Req *r = new Req();
    r->A = A;
    r->B = B;
    r->t_submit = Clock::now();
    if (normalize_range(A, B, &r->An, &r->Bn))
        r->nE = (r->Bn - r->An) / 2 + 1;
    r->reserve = reservation(s, r);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        delete r;
        gb_internal_set_error("server: closing");
        return GB_EINVAL;
    }
    if (r->reserve > s->cfg.hbm_budget_bytes) {
        delete r;
        gb_internal_set_error("server: the request's reservation exceeds the HBM budget");
        return GB_ENOMEM;
    }
    if (s->cfg.max_pending && s->pending.size() >= s->cfg.max_pending) {
        delete r;
        gb_internal_set_error("server: queue full");
        return GB_EBUSY;
    }
    r->id = s->next_id++;
    if (id)
        *id = r->id;
    s->stats.submitted++;
    if (r->nE == 0) {   // an empty range completes at once
        s->reserved += r->reserve;
        finish(s, r, Clock::now());
        s->cv_done.notify_all();
        return GB_OK;
    }
    s->pending.push_back(r);
    s->cv_work.notify_one();
    return GB_OK;
}

gb_status gb_server_poll(gb_server *s, int32_t wait_ms, uint64_t *id, gb_result *out,
                         double *latency_ms)
{
    if (!s || !out)
        return GB_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->finished.empty() && wait_ms != 0) {
        auto pred = [&] { return !s->finished.empty(); };
        if (wait_ms < 0)
            s->cv_done.wait(lk, pred);
        else
            s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), pred);
    }
    if (s->finished.empty())
        return GB_EBUSY;
    Req *r = s->finished.front();
    s->finished.pop_front();
    lk.unlock();
    if (id)
        *id = r->id;
    if (latency_ms)
        *latency_ms = r->latency_ms;
    out->A = r->An;
    out->B = r->Bn;
    out->P_max = s->cfg.P_max;
    out->verified = r->verified;
    out->max_p = r->max_p;
    out->max_p_n = r->max_p ? r->max_p_n : 0;
    out->checksum = r->checksum;
    out->n_unresolved = r->n_unres;
    out->n_failed = r->n_failed;
    gb_status st = r->status;
    const uint64_t take = std::min<uint64_t>(r->unres.size(), out->unresolved ? out->unresolved_cap : 0);
    for (uint64_t i = 0; i < take; ++i)
        out->unresolved[i] = r->unres[i];
    if (st == GB_OK && take < r->n_unres)
        st = GB_ETRUNC;
    delete r;
    return st;
}

gb_status gb_server_get_stats(gb_server *s, gb_server_stats *out)
{
    if (!s || !out)
        return GB_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->active = s->active.size();
    out->pending = s->pending.size();
    out->reserved_bytes = s->reserved;
    out->wall_ms = std::chrono::duration<double, std::milli>(Clock::now() - s->t_open).count();
    return GB_OK;
}

gb_status gb_server_close(gb_server *s)
{
    if (!s)
        return GB_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->th.joinable())
        s->th.join();
    for (Req *r : s->pending)
        delete r;
    for (Req *r : s->finished)
        delete r;
    (void)hipStreamDestroy(s->stream);
    delete s;
    return GB_OK;
}

}  // extern "C"
