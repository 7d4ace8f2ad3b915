// gb_server.hip -- the serving loop behind gb_server_*: continuous batching
// of single-n and range requests over several device streams, admission by
// device memory, completion timestamps for latency, and a trace replay that
// submits requests at given arrival times.
//
// A launch on one stream runs its single n first (one wavefront each, the
// exhaustive-phase kernel from p = 3) and records an event, then its ranges
// (one persistent tile launch over all their windows, the exhaustive phase,
// the summaries), then the per-n output copies, and records a second event.
// The single n of a launch are reported as soon as the first event has
// fired, so they never wait for the ranges they were launched with.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
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

// One range's per-n output moved from the launch's staging buffer to the
// caller's device buffer.
struct GbScatter {
    uint16_t *dst;
    unsigned long long src_off;  // index into the staging buffer
    unsigned long long len;
};

constexpr uint32_t kScatterChunk = 1u << 12;   // entries per workgroup (16 per thread)

// blockIdx.y: the range; blockIdx.x: its chunk of kScatterChunk entries
__global__ __launch_bounds__(256) void k_scatter16(const GbScatter *e, const uint16_t *src)
{
    const GbScatter s = e[blockIdx.y];
    const unsigned long long b = (unsigned long long)blockIdx.x * kScatterChunk;
    if (b >= s.len) return;
    const unsigned long long end = min(s.len, b + kScatterChunk);
    for (unsigned long long i = b + threadIdx.x; i < end; i += 256) s.dst[i] = src[s.src_off + i];
}

struct Req {
    gb_request r;
    uint64_t id = 0;
    uint64_t bytes = 0;
    uint64_t submit_ns = 0;
};

constexpr uint64_t kStageN = 1ull << 24;       // per-n staging entries set up at start
constexpr uint64_t kStageTiles = 1ull << 16;   // tile records set up at start
constexpr uint32_t kServeTileLog2 = 16;         // server tiles when the caller sets none
constexpr uint32_t kServeThreads = 1024;        // and their workgroup size

struct Lane {
    hipStream_t stream = nullptr;
    Workspace ws;
    hipEvent_t ev_one = nullptr;                 // after the single n of the launch
    bool busy = false, ones_open = false, ranges_open = false;
    std::vector<Req> batch;
    std::vector<size_t> range_idx, one_idx;     // positions in batch
    std::vector<uint64_t> out_off;              // per range: offset in the staging output
    uint64_t bytes = 0;
    uint64_t launch_ns = 0;
    bool host_pmin = false;
    PinBuf<GbWindow> h_win;
    PinBuf<uint16_t> h_pmin;                    // host copy of the staging output
    PinBuf<GbScatter> h_scat;
    DevBuf<GbScatter> scat;
};

}  // namespace

struct gb_server {
    gb_ctx *ctx = nullptr;
    uint32_t max_batch = 4096;
    std::vector<Lane> lanes;
    std::thread thr;
    std::mutex mu;                      // guards pending, done, stats, stop
    std::condition_variable cv_work, cv_done;
    std::deque<Req> pending_one, pending_rng;   // queued single n and ranges, each in arrival order
    std::deque<gb_completion> done;
    gb_server_stats st{};
    bool stop = false;
    uint64_t next_id = 1;
    std::string err;
    uint64_t tile_n = 0;
};

namespace {

uint64_t pow2_at_least(uint64_t x)
{
    uint64_t v = 1;
    while (v < x) v <<= 1;
    return v;
}

uint64_t request_bytes(const gb_server *s, const gb_request &r)
{
    if (r.kind == GB_REQ_ONE) return 48;
    // the planner moves a range's first n down to a multiple of 384 (up to
    // 191 n in front)
    const uint64_t tiles = (r.len + 191 + s->tile_n - 1) / s->tile_n;
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

// Enqueue one batch on lane L (all requests already admitted): single n
// first, their event, then the ranges, their output copies and the final
// event.
gb_status launch_batch(gb_server *s, Lane &L)
{
    gb_ctx *c = s->ctx;
    Workspace &ws = L.ws;
    L.range_idx.clear();
    L.one_idx.clear();
    L.out_off.clear();
    L.host_pmin = false;
    for (size_t i = 0; i < L.batch.size(); ++i)
        (L.batch[i].r.kind == GB_REQ_RANGE ? L.range_idx : L.one_idx).push_back(i);
    if (!L.one_idx.empty()) {
        const uint64_t k = L.one_idx.size();
        GB_HIP(c, ws.q.ensure(2 * k));
        GB_HIP(c, ws.h_q.ensure(2 * k));
        for (uint64_t i = 0; i < k; ++i) ws.h_q.p[i] = L.batch[L.one_idx[i]].r.n;
        GB_HIP(c, hipMemcpyAsync(ws.q.p, ws.h_q.p, k * 8, hipMemcpyHostToDevice, L.stream));
        gb_status stt = enqueue_queries(c, ws, k, ws.q.p, ws.q.p + k, L.stream);
        if (stt != GB_OK) return stt;
        GB_HIP(c, hipMemcpyAsync(ws.h_q.p + k, ws.q.p + k, k * 8, hipMemcpyDeviceToHost, L.stream));
        GB_HIP(c, hipEventRecord(L.ev_one, L.stream));
    }
    if (!L.range_idx.empty()) {
        Plan pl;
        pl.w.resize(L.range_idx.size());
        bool want_pmin = false;
        for (size_t j = 0; j < L.range_idx.size(); ++j) {
            const gb_request &r = L.batch[L.range_idx[j]].r;
            pl.w[j].first_n = r.n;
            pl.w[j].count = r.len;
            pl.w[j].slot = (uint32_t)j;
            if (r.pmin) want_pmin = true;
        }
        gb_status stt = plan_windows(c, pl);
        if (stt != GB_OK) return stt;
        for (auto &w : pl.w) L.out_off.push_back(w.out_off);
        stt = ensure_workspace(c, ws, pl, pl.w.size(), 1);
        if (stt != GB_OK) return stt;
        void *pmin_dev = nullptr;
        if (want_pmin) {
            // grown in powers of two: a reallocation waits for the device
            GB_HIP(c, ws.pmin.ensure(pow2_at_least(pl.total_n * 2)));
            pmin_dev = ws.pmin.p;
        }
        GB_HIP(c, L.h_win.ensure(pl.w.size()));
        std::memcpy(L.h_win.p, pl.w.data(), pl.w.size() * sizeof(GbWindow));
        GB_HIP(c, hipMemcpyAsync(ws.win.p, L.h_win.p, pl.w.size() * sizeof(GbWindow), hipMemcpyHostToDevice,
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
        if (want_pmin) {
            // device destinations: one scatter launch; host destinations: one
            // copy of the whole staging output into pinned memory
            std::vector<GbScatter> sc;
            uint64_t maxlen = 0;
            for (size_t j2 = 0; j2 < L.range_idx.size(); ++j2) {
                const gb_request &r = L.batch[L.range_idx[j2]].r;
                if (!r.pmin) continue;
                if (r.flags & GB_REQ_PMIN_DEVICE) {
                    sc.push_back({r.pmin, (unsigned long long)L.out_off[j2], (unsigned long long)r.len});
                    maxlen = std::max<uint64_t>(maxlen, r.len);
                } else {
                    L.host_pmin = true;
                }
            }
            if (!sc.empty()) {
                GB_HIP(c, L.scat.ensure(sc.size()));
                GB_HIP(c, L.h_scat.ensure(sc.size()));
                std::memcpy(L.h_scat.p, sc.data(), sc.size() * sizeof(GbScatter));
                GB_HIP(c, hipMemcpyAsync(L.scat.p, L.h_scat.p, sc.size() * sizeof(GbScatter), hipMemcpyHostToDevice,
                                         L.stream));
                const dim3 grid((uint32_t)((maxlen + kScatterChunk - 1) / kScatterChunk), (uint32_t)sc.size());
                hipLaunchKernelGGL(k_scatter16, grid, dim3(256), 0, L.stream, L.scat.p,
                                   reinterpret_cast<const uint16_t *>(ws.pmin.p));
                GB_HIP(c, hipGetLastError());
            }
            if (L.host_pmin) {
                GB_HIP(c, L.h_pmin.ensure(pow2_at_least(pl.total_n)));
                GB_HIP(c, hipMemcpyAsync(L.h_pmin.p, ws.pmin.p, pl.total_n * 2, hipMemcpyDeviceToHost, L.stream));
            }
        }
    }
    GB_HIP(c, hipEventRecord(ws.done, L.stream));
    L.ones_open = !L.one_idx.empty();
    L.ranges_open = !L.range_idx.empty();
    return GB_OK;
}

void finish_ones(Lane &L, uint32_t lane_idx, gb_status launch_status, std::vector<gb_completion> &out)
{
    const uint64_t t = now_ns();
    const uint64_t k = L.one_idx.size();
    for (size_t i = 0; i < k; ++i) {
        const Req &q = L.batch[L.one_idx[i]];
        gb_completion comp = base_completion(q, L, lane_idx);
        comp.status = launch_status;
        if (launch_status == GB_OK) {
            comp.p = L.ws.h_q.p[k + i];
            if (comp.p == 0) comp.status = GB_EUNRESOLVED;
        }
        comp.done_ns = t;
        out.push_back(comp);
    }
    L.ones_open = false;
}

void finish_ranges(gb_server *s, Lane &L, uint32_t lane_idx, gb_status launch_status, std::vector<gb_completion> &out)
{
    gb_ctx *c = s->ctx;
    Workspace &ws = L.ws;
    bool list_overflow = false;
    if (launch_status == GB_OK && ws.h_counters.p[0] > c->prm.max_unresolved) list_overflow = true;
    for (size_t j = 0; j < L.range_idx.size(); ++j) {
        const Req &q = L.batch[L.range_idx[j]];
        gb_completion comp = base_completion(q, L, lane_idx);
        comp.status = launch_status;
        if (launch_status == GB_OK) {
            merge_slot(comp.summary, ws.h_slots.p[j]);
            if (list_overflow) comp.status = GB_ENOMEM;
            else if (comp.summary.n_failed) comp.status = GB_EUNRESOLVED;
            if (q.r.pmin && !(q.r.flags & GB_REQ_PMIN_DEVICE))
                std::memcpy(q.r.pmin, L.h_pmin.p + L.out_off[j], q.r.len * 2);
        }
        comp.done_ns = now_ns();
        out.push_back(comp);
    }
    L.ranges_open = false;
}

void scheduler(gb_server *s)
{
    (void)hipSetDevice(s->ctx->prm.device);
    std::vector<gb_completion> fresh;
    for (;;) {
        bool any_busy = false;
        fresh.clear();
        uint64_t freed = 0;
        // 1. collect finished parts of launches
        for (uint32_t i = 0; i < s->lanes.size(); ++i) {
            Lane &L = s->lanes[i];
            if (!L.busy) continue;
            if (L.ones_open) {
                const hipError_t e = hipEventQuery(L.ev_one);
                if (e != hipErrorNotReady) finish_ones(L, i, e == hipSuccess ? GB_OK : GB_EDEVICE, fresh);
            }
            if (!L.ones_open && L.ranges_open) {
                const hipError_t e = hipEventQuery(L.ws.done);
                if (e != hipErrorNotReady) finish_ranges(s, L, i, e == hipSuccess ? GB_OK : GB_EDEVICE, fresh);
            }
            if (L.ones_open || L.ranges_open) {
                any_busy = true;
                continue;
            }
            freed += L.bytes;
            L.batch.clear();
            L.busy = false;
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
        for (uint32_t i = 0; i < s->lanes.size() && (!s->pending_one.empty() || !s->pending_rng.empty()); ++i) {
            Lane &L = s->lanes[i];
            if (L.busy) continue;
            L.batch.clear();
            L.bytes = 0;
            // With two or more streams, stream 0 takes single n only, so that a
            // single n never waits for a stream busy with ranges; the other
            // streams take both kinds in arrival (id) order.
            const bool ones_only = i == 0 && s->lanes.size() > 1;
            for (;;) {
                if (L.batch.size() >= s->max_batch) break;
                std::deque<Req> *from = nullptr;
                if (!s->pending_one.empty()) from = &s->pending_one;
                if (!ones_only && !s->pending_rng.empty() &&
                    (!from || s->pending_rng.front().id < from->front().id))
                    from = &s->pending_rng;
                if (!from || s->st.bytes_inflight + L.bytes + from->front().bytes > s->ctx->prm.mem_budget) break;
                L.bytes += from->front().bytes;
                L.batch.push_back(from->front());
                from->pop_front();
            }
            if (L.batch.empty()) {
                if (ones_only) continue;
                break;  // memory is full: wait for a launch to finish
            }
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
                finish_ones(L, i, ls, bad);
                finish_ranges(s, L, i, ls, bad);
                L.batch.clear();
                L.busy = false;
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
            if (s->stop && s->pending_one.empty() && s->pending_rng.empty()) break;
            s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        lk.unlock();
        std::this_thread::yield();
    }
}

gb_status check_request(const gb_server *s, const gb_request &r)
{
    if (r.kind != GB_REQ_ONE && r.kind != GB_REQ_RANGE) return GB_EINVAL;
    if (r.flags & ~GB_REQ_PMIN_DEVICE) return GB_EINVAL;
    if ((r.flags & GB_REQ_PMIN_DEVICE) && (r.kind != GB_REQ_RANGE || !r.pmin)) return GB_EINVAL;
    if (r.n < 4 || (r.n & 1) || r.n > GB_MAX_N) return GB_EINVAL;
    if (r.kind == GB_REQ_RANGE) {
        if (r.len == 0 || r.len > (GB_MAX_N - r.n) / 2 + 1) return GB_EINVAL;
        if (r.n + 2 * (r.len - 1) > s->ctx->prm.max_hi) return GB_ERANGE;
    }
    return GB_OK;
}

// queue one request stamped with submit_ns
gb_status submit_at(gb_server *s, const gb_request &r, uint64_t submit_ns, uint64_t *id)
{
    const gb_status chk = check_request(s, r);
    if (chk != GB_OK) return chk;
    Req q;
    q.r = r;
    q.bytes = request_bytes(s, r);
    q.submit_ns = submit_ns;
    std::lock_guard<std::mutex> lk(s->mu);
    if (q.bytes > s->ctx->prm.mem_budget) {
        s->st.rejected += 1;
        return GB_ENOMEM;
    }
    q.id = s->next_id++;
    if (id) *id = q.id;
    (r.kind == GB_REQ_ONE ? s->pending_one : s->pending_rng).push_back(q);
    s->st.submitted += 1;
    s->st.queued += 1;
    s->cv_work.notify_one();
    return GB_OK;
}

// Run one small range (with and without per-n output) and one single n on
// every lane, so that code objects are loaded and the lanes' buffers are
// sized before the first request.
gb_status warm_lanes(gb_server *s)
{
    gb_ctx *c = s->ctx;
    // every launch path once per lane: a single n beside a range with no
    // per-n output, with it in host memory, and with it in device memory,
    // so that no request pays a first launch of a kernel
    std::vector<uint16_t> out(256);
    uint16_t *dout = nullptr;
    GB_HIP(c, hipMalloc(&dout, 256 * sizeof(uint16_t)));
    gb_status st = GB_OK;
    for (uint32_t i = 0; i < s->lanes.size() && st == GB_OK; ++i) {
        Lane &L = s->lanes[i];
        for (int form = 0; form < 3 && st == GB_OK; ++form) {
            L.batch.clear();
            Req a, b;
            a.r = gb_request{GB_REQ_ONE, 0, 1000000000000ull, 1, nullptr, 0};
            b.r = gb_request{GB_REQ_RANGE, form == 2 ? GB_REQ_PMIN_DEVICE : 0u, 1000000000000ull, 256,
                             form == 0 ? nullptr : form == 1 ? out.data() : dout, 0};
            L.batch.push_back(a);
            L.batch.push_back(b);
            st = launch_batch(s, L);
            if (hipStreamSynchronize(L.stream) != hipSuccess && st == GB_OK) st = GB_EDEVICE;
            L.batch.clear();
            L.ones_open = L.ranges_open = false;
        }
    }
    (void)hipFree(dout);
    return st;
}

void release_lanes(gb_server *s)
{
    for (auto &L : s->lanes) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        L.ws.release();
        L.h_win.release();
        L.h_pmin.release();
        L.h_scat.release();
        L.scat.release();
        if (L.ev_one) (void)hipEventDestroy(L.ev_one);
        if (L.stream) (void)hipStreamDestroy(L.stream);
        L.ev_one = nullptr;
        L.stream = nullptr;
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
    // latency first: tiles of 2^16 n with 1024 threads unless the caller
    // sets them, so that a range spreads over many workgroups
    gb_params p{};
    if (prm) p = *prm;
    if (p.tile_log2 == 0) p.tile_log2 = kServeTileLog2;
    if (p.wg_threads == 0) p.wg_threads = kServeThreads;
    gb_status st = gb_create(&s->ctx, &p);
    if (st != GB_OK) {
        delete s;
        return st;
    }
    if (s->max_batch > s->ctx->prm.max_unresolved) s->max_batch = (uint32_t)s->ctx->prm.max_unresolved;
    s->tile_n = s->ctx->tile_n;
    s->lanes.resize(streams);
    bool ok = true;
    for (auto &L : s->lanes) {
        const uint64_t mb = s->max_batch;
        ok = ok && hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&L.ev_one, hipEventDisableTiming) == hipSuccess &&
             L.ws.init(s->ctx->prm.max_unresolved) == hipSuccess && L.ws.h_counters.ensure(kCounters) == hipSuccess &&
             L.ws.win.ensure(mb) == hipSuccess && L.ws.slots.ensure(mb) == hipSuccess &&
             L.ws.h_slots.ensure(mb) == hipSuccess && L.ws.recs.ensure(kStageTiles) == hipSuccess &&
             L.ws.hist.ensure(GB_HIST_BINS_I) == hipSuccess && L.ws.h_hist.ensure(GB_HIST_BINS_I) == hipSuccess &&
             L.ws.q.ensure(2 * mb) == hipSuccess && L.ws.h_q.ensure(2 * mb) == hipSuccess &&
             L.ws.pmin.ensure(2 * kStageN) == hipSuccess && L.h_pmin.ensure(kStageN) == hipSuccess &&
             L.h_win.ensure(mb) == hipSuccess && L.scat.ensure(mb) == hipSuccess && L.h_scat.ensure(mb) == hipSuccess;
        if (!ok) break;
    }
    if (ok) ok = warm_lanes(s) == GB_OK;
    if (!ok) {
        release_lanes(s);
        gb_destroy(s->ctx);
        delete s;
        return GB_EDEVICE;
    }
    s->thr = std::thread(scheduler, s);
    *out = s;
    return GB_OK;
}

gb_status gb_server_submit(gb_server *s, const gb_request *req, uint64_t *id)
{
    if (!s || !req) return GB_EINVAL;
    return submit_at(s, *req, now_ns(), id);
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

gb_status gb_server_replay(gb_server *s, const gb_request *req, const uint64_t *arrival_ns, size_t k,
                           gb_completion *out, uint32_t timeout_ms)
{
    if (!s || (k && (!req || !arrival_ns || !out))) return GB_EINVAL;
    for (size_t i = 0; i < k; ++i) {
        if (check_request(s, req[i]) != GB_OK) return GB_EINVAL;
        if (i && arrival_ns[i] < arrival_ns[i - 1]) return GB_EINVAL;
    }
    std::unordered_map<uint64_t, size_t> where;
    std::unordered_map<uint64_t, gb_completion> early;
    where.reserve(k * 2 + 1);
    const uint64_t t0 = now_ns() + 200000;        // a small lead before the first arrival
    const uint64_t deadline = t0 + (arrival_ns && k ? arrival_ns[k - 1] : 0) + (uint64_t)timeout_ms * 1000000ull;
    size_t next = 0, got = 0;
    while (got < k) {
        uint64_t now = now_ns();
        while (next < k && t0 + arrival_ns[next] <= now) {
            uint64_t id = 0;
            const gb_status st = submit_at(s, req[next], t0 + arrival_ns[next], &id);
            if (st != GB_OK) {
                // already checked: only an oversized request gets here
                gb_completion c{};
                c.tag = req[next].tag;
                c.kind = req[next].kind;
                c.status = st;
                c.submit_ns = c.launch_ns = c.done_ns = t0 + arrival_ns[next];
                out[next] = c;
                ++got;
            } else {
                // the scheduler may finish it before this thread records the id
                auto u = early.find(id);
                if (u != early.end()) {
                    out[next] = u->second;
                    early.erase(u);
                    ++got;
                } else {
                    where[id] = next;
                }
            }
            ++next;
        }
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->done.empty() && next == k)
                s->cv_done.wait_for(lk, std::chrono::microseconds(500), [&] { return !s->done.empty(); });
            while (!s->done.empty()) {
                const gb_completion c = s->done.front();
                s->done.pop_front();
                auto it = where.find(c.id);
                if (it == where.end()) {
                    early[c.id] = c;
                    continue;
                }
                out[it->second] = c;
                where.erase(it);
                ++got;
            }
        }
        now = now_ns();
        if (now > deadline) return GB_EDEVICE;
        if (next < k) {
            const uint64_t at = t0 + arrival_ns[next];
            if (at > now + 300000)
                std::this_thread::sleep_for(std::chrono::nanoseconds(at - now - 200000));
            else if (at > now)
                std::this_thread::yield();
        }
    }
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
    release_lanes(s);
    gb_destroy(s->ctx);
    delete s;
    return GB_OK;
}

const char *gb_server_last_error(const gb_server *s) { return s ? s->err.c_str() : "null server"; }

}  // extern "C"
