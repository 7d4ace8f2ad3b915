// gb_server.hip -- the serving loop behind gb_server_*: continuous batching
// of single-n and range requests over several device streams, admission by
// device memory, completion timestamps for latency.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "gb_runtime.h"

using namespace gbrt;

namespace {

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Req {
    gb_request r;
    uint64_t id = 0;
    uint64_t bytes = 0;
    uint64_t submit_ns = 0;
};

struct Lane {
    hipStream_t stream = nullptr;
    Workspace ws;
    bool busy = false;
    std::vector<Req> batch;
    std::vector<size_t> range_idx, one_idx;  // positions in batch
    std::vector<uint64_t> out_off;           // per range: offset in the staging output
    uint64_t bytes = 0;
    uint64_t launch_ns = 0;
    bool want_pmin = false;
};

}  // namespace

struct gb_server {
    gb_ctx *ctx = nullptr;
    uint32_t max_batch = 4096;
    std::vector<Lane> lanes;
    std::thread thr;
    std::mutex mu;                      // guards pending, done, stats, stop
    std::condition_variable cv_work, cv_done;
    std::deque<Req> pending;
    std::deque<gb_completion> done;
    gb_server_stats st{};
    bool stop = false;
    uint64_t next_id = 1;
    std::string err;
    uint64_t tile_n = 0;
};

namespace {

uint64_t request_bytes(const gb_server *s, const gb_request &r)
{
    if (r.kind == GB_REQ_ONE) return 48;
    const uint64_t tiles = (r.len + s->tile_n - 1) / s->tile_n;
    return 64 + 40 + 16 * tiles + (r.pmin ? 2 * r.len : 0);
}

gb_completion base_completion(const Req &q, const Lane &L, uint32_t lane_idx)
{
    gb_completion c{};
    c.id = q.id;
    c.tag = q.r.tag;
    c.kind = q.r.kind;
    c.submit_ns = q.submit_ns;
    c.launch_ns = L.launch_ns;
    c.batch_requests = (uint32_t)L.batch.size();
    c.stream = lane_idx;
    return c;
}

// Enqueue one batch on lane L (all requests already admitted).
gb_status launch_batch(gb_server *s, Lane &L)
{
    gb_ctx *c = s->ctx;
    Workspace &ws = L.ws;
    L.range_idx.clear();
    L.one_idx.clear();
    L.out_off.clear();
    L.want_pmin = false;
    for (size_t i = 0; i < L.batch.size(); ++i)
        (L.batch[i].r.kind == GB_REQ_RANGE ? L.range_idx : L.one_idx).push_back(i);
    if (!L.range_idx.empty()) {
        Plan pl;
        pl.w.resize(L.range_idx.size());
        for (size_t j = 0; j < L.range_idx.size(); ++j) {
            const gb_request &r = L.batch[L.range_idx[j]].r;
            pl.w[j].first_n = r.n;
            pl.w[j].count = r.len;
            pl.w[j].slot = (uint32_t)j;
            if (r.pmin) L.want_pmin = true;
        }
        gb_status stt = plan_windows(c, pl);
        if (stt != GB_OK) return stt;
        for (auto &w : pl.w) L.out_off.push_back(w.out_off);
        stt = ensure_workspace(c, ws, pl, pl.w.size(), 1);
        if (stt != GB_OK) return stt;
        void *pmin_dev = nullptr;
        if (L.want_pmin) {
            GB_HIP(c, ws.pmin.ensure(pl.total_n * 2));
            pmin_dev = ws.pmin.p;
        }
        GB_HIP(c, hipMemcpyAsync(ws.win.p, pl.w.data(), pl.w.size() * sizeof(GbWindow), hipMemcpyHostToDevice,
                                 L.stream));
        Job j;
        j.pl = &pl;
        j.nslots = pl.w.size();
        j.hist_rows = 1;
        j.pmin_dev = pmin_dev;
        j.pmin_bits = pmin_dev ? 16 : 0;
        j.persistent = true;
        stt = run_job(c, ws, j, GraphKey{}, false, L.stream);
        if (stt != GB_OK) return stt;
    }
    if (!L.one_idx.empty()) {
        const uint64_t k = L.one_idx.size();
        GB_HIP(c, ws.q.ensure(2 * k));
        GB_HIP(c, ws.h_q.ensure(2 * k));
        for (uint64_t i = 0; i < k; ++i) ws.h_q.p[i] = L.batch[L.one_idx[i]].r.n;
        GB_HIP(c, hipMemcpyAsync(ws.q.p, ws.h_q.p, k * 8, hipMemcpyHostToDevice, L.stream));
        gb_status stt = enqueue_queries(c, ws, k, ws.q.p, ws.q.p + k, L.stream);
        if (stt != GB_OK) return stt;
        GB_HIP(c, hipMemcpyAsync(ws.h_q.p + k, ws.q.p + k, k * 8, hipMemcpyDeviceToHost, L.stream));
    }
    GB_HIP(c, hipEventRecord(ws.done, L.stream));
    return GB_OK;
}

// Turn a finished launch into completions.
void finish_batch(gb_server *s, Lane &L, uint32_t lane_idx, gb_status launch_status, std::vector<gb_completion> &out)
{
    gb_ctx *c = s->ctx;
    Workspace &ws = L.ws;
    const uint64_t t = now_ns();
    bool list_overflow = false;
    if (launch_status == GB_OK && !L.range_idx.empty() && ws.h_counters.p[0] > c->prm.max_unresolved)
        list_overflow = true;
    for (size_t j = 0; j < L.range_idx.size(); ++j) {
        const Req &q = L.batch[L.range_idx[j]];
        gb_completion comp = base_completion(q, L, lane_idx);
        comp.status = launch_status;
        if (launch_status == GB_OK) {
            merge_slot(comp.summary, ws.h_slots.p[j]);
            if (list_overflow) comp.status = GB_ENOMEM;
            else if (comp.summary.n_failed) comp.status = GB_EUNRESOLVED;
            if (q.r.pmin) {
                if (hipMemcpy(q.r.pmin, ws.pmin.p + 2 * L.out_off[j], q.r.len * 2, hipMemcpyDeviceToHost) !=
                    hipSuccess)
                    comp.status = GB_EDEVICE;
            }
        }
        comp.done_ns = now_ns();
        out.push_back(comp);
    }
    const uint64_t k = L.one_idx.size();
    for (size_t i = 0; i < k; ++i) {
        const Req &q = L.batch[L.one_idx[i]];
        gb_completion comp = base_completion(q, L, lane_idx);
        comp.status = launch_status;
        if (launch_status == GB_OK) {
            comp.p = ws.h_q.p[k + i];
            if (comp.p == 0) comp.status = GB_EUNRESOLVED;
        }
        comp.done_ns = t;
        out.push_back(comp);
    }
    L.batch.clear();
    L.busy = false;
}

void scheduler(gb_server *s)
{
    (void)hipSetDevice(s->ctx->prm.device);
    std::vector<gb_completion> fresh;
    for (;;) {
        bool any_busy = false;
        fresh.clear();
        uint64_t freed = 0;
        // 1. collect finished launches
        for (uint32_t i = 0; i < s->lanes.size(); ++i) {
            Lane &L = s->lanes[i];
            if (!L.busy) continue;
            const hipError_t e = hipEventQuery(L.ws.done);
            if (e == hipErrorNotReady) {
                any_busy = true;
                continue;
            }
            freed += L.bytes;
            finish_batch(s, L, i, e == hipSuccess ? GB_OK : GB_EDEVICE, fresh);
        }
        // 2. admit queued requests onto idle lanes
        std::unique_lock<std::mutex> lk(s->mu);
        s->st.bytes_inflight -= freed;
        if (!fresh.empty()) {
            s->st.completed += fresh.size();
            s->st.inflight -= fresh.size();
            for (auto &cpl : fresh) s->done.push_back(cpl);
            s->cv_done.notify_all();
        }
        for (uint32_t i = 0; i < s->lanes.size() && !s->pending.empty(); ++i) {
            Lane &L = s->lanes[i];
            if (L.busy) continue;
            L.batch.clear();
            L.bytes = 0;
            while (!s->pending.empty() && L.batch.size() < s->max_batch &&
                   s->st.bytes_inflight + L.bytes + s->pending.front().bytes <= s->ctx->prm.mem_budget) {
                L.bytes += s->pending.front().bytes;
                L.batch.push_back(s->pending.front());
                s->pending.pop_front();
            }
            if (L.batch.empty()) break;  // memory is full: wait for a launch to finish
            s->st.bytes_inflight += L.bytes;
            s->st.peak_bytes_inflight = std::max(s->st.peak_bytes_inflight, s->st.bytes_inflight);
            s->st.queued -= L.batch.size();
            s->st.inflight += L.batch.size();
            s->st.launches += 1;
            lk.unlock();
            L.launch_ns = now_ns();
            const gb_status ls = launch_batch(s, L);
            L.busy = true;
            if (ls != GB_OK) {
                // nothing (more) was enqueued: report the failure on every request
                (void)hipStreamSynchronize(L.stream);
                std::vector<gb_completion> bad;
                finish_batch(s, L, i, ls, bad);
                lk.lock();
                s->err = s->ctx->err;
                s->st.bytes_inflight -= L.bytes;
                s->st.completed += bad.size();
                s->st.inflight -= bad.size();
                for (auto &cpl : bad) s->done.push_back(cpl);
                s->cv_done.notify_all();
                continue;
            }
            any_busy = true;
            lk.lock();
        }
        uint64_t nbusy = 0;
        for (auto &L : s->lanes) nbusy += L.busy ? 1 : 0;
        s->st.peak_concurrent_launches = std::max(s->st.peak_concurrent_launches, nbusy);
        if (!any_busy && nbusy == 0) {
            if (s->stop && s->pending.empty()) break;
            s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        lk.unlock();
        std::this_thread::yield();
    }
}

}  // namespace

extern "C" {

gb_status gb_server_start(gb_server **out, const gb_params *prm, uint32_t streams, uint32_t max_batch)
{
    if (!out) return GB_EINVAL;
    *out = nullptr;
    if (streams == 0) streams = 2;
    if (streams > 8) return GB_EINVAL;
    gb_server *s = new (std::nothrow) gb_server();
    if (!s) return GB_ENOMEM;
    s->max_batch = max_batch ? max_batch : 4096;
    gb_status st = gb_create(&s->ctx, prm);
    if (st != GB_OK) {
        delete s;
        return st;
    }
    if (s->max_batch > s->ctx->prm.max_unresolved) s->max_batch = (uint32_t)s->ctx->prm.max_unresolved;
    s->tile_n = s->ctx->tile_n;
    s->lanes.resize(streams);
    for (auto &L : s->lanes) {
        if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
            L.ws.init(s->ctx->prm.max_unresolved) != hipSuccess || L.ws.h_counters.ensure(kCounters) != hipSuccess) {
            for (auto &M : s->lanes) {
                M.ws.release();
                if (M.stream) (void)hipStreamDestroy(M.stream);
            }
            gb_destroy(s->ctx);
            delete s;
            return GB_EDEVICE;
        }
    }
    s->thr = std::thread(scheduler, s);
    *out = s;
    return GB_OK;
}

gb_status gb_server_submit(gb_server *s, const gb_request *req, uint64_t *id)
{
    if (!s || !req) return GB_EINVAL;
    const gb_request &r = *req;
    if (r.flags != 0 || (r.kind != GB_REQ_ONE && r.kind != GB_REQ_RANGE)) return GB_EINVAL;
    if (r.n < 4 || (r.n & 1) || r.n > GB_MAX_N) return GB_EINVAL;
    if (r.kind == GB_REQ_RANGE) {
        if (r.len == 0 || r.len > (GB_MAX_N - r.n) / 2 + 1) return GB_EINVAL;
        if (r.n + 2 * (r.len - 1) > s->ctx->prm.max_hi) return GB_ERANGE;
    }
    Req q;
    q.r = r;
    q.bytes = request_bytes(s, r);
    q.submit_ns = now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    if (q.bytes > s->ctx->prm.mem_budget) {
        s->st.rejected += 1;
        return GB_ENOMEM;
    }
    q.id = s->next_id++;
    if (id) *id = q.id;
    s->pending.push_back(q);
    s->st.submitted += 1;
    s->st.queued += 1;
    s->cv_work.notify_one();
    return GB_OK;
}

gb_status gb_server_poll(gb_server *s, gb_completion *out, size_t cap, size_t *count, int32_t wait_ms)
{
    if (!s || !count || (cap && !out)) return GB_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
    size_t n = 0;
    while (n < cap && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    *count = n;
    return GB_OK;
}

gb_status gb_server_stats_get(gb_server *s, gb_server_stats *stats)
{
    if (!s || !stats) return GB_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *stats = s->st;
    return GB_OK;
}

gb_status gb_server_stop(gb_server *s)
{
    if (!s) return GB_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->thr.joinable()) s->thr.join();
    (void)hipSetDevice(s->ctx->prm.device);
    for (auto &L : s->lanes) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        L.ws.release();
        if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    gb_destroy(s->ctx);
    delete s;
    return GB_OK;
}

const char *gb_server_last_error(const gb_server *s) { return s ? s->err.c_str() : "null server"; }

}  // extern "C"
