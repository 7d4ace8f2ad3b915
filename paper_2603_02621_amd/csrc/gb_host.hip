// gb_host.hip -- host runtime behind the C ABI in include/goldbach.h:
// context and resident tables, segment/tile planning, launches, the HIP
// graphs of the batched forms, and the summary merge.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "gb_runtime.h"

namespace gbrt {

std::atomic<uint64_t> g_buffer_generation{1};

gb_status fail(gb_ctx *c, gb_status st, const std::string &msg)
{
    if (c) c->err = msg;
    return st;
}

uint64_t isqrt64(uint64_t x)
{
    uint64_t lo = 0, hi = 4294967295ull;
    if (hi > x) hi = x;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        if ((unsigned __int128)mid * mid <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

namespace {

// Odd primes up to `limit` by a segmented odd-only sieve (host, once per context).
std::vector<uint32_t> host_odd_primes(uint64_t limit)
{
    std::vector<uint32_t> out;
    if (limit < 3) return out;
    const uint64_t r = isqrt64(limit);
    std::vector<uint8_t> small(r + 1, 1);
    std::vector<uint32_t> base;
    for (uint64_t i = 3; i <= r; i += 2)
        if (small[i]) {
            base.push_back((uint32_t)i);
            for (uint64_t j = i * i; j <= r; j += 2 * i) small[j] = 0;
        }
    const uint64_t SEG = 1ull << 22;  // odd numbers per segment
    std::vector<uint8_t> seg(SEG);
    for (uint64_t lo = 3; lo <= limit; lo += 2 * SEG) {
        uint64_t hi = std::min<uint64_t>(lo + 2 * (SEG - 1), limit | 1ull);
        if (hi > limit) hi -= 2;
        const uint64_t n = (hi - lo) / 2 + 1;
        std::fill(seg.begin(), seg.begin() + n, 1);
        for (uint32_t p : base) {
            uint64_t m = (uint64_t)p * p;
            if (m > hi) break;
            if (m < lo) {
                m = (lo + p - 1) / p * p;
                if (!(m & 1)) m += p;
            }
            for (; m <= hi; m += 2ull * p) seg[(m - lo) / 2] = 0;
        }
        for (uint64_t i = 0; i < n; ++i)
            if (seg[i]) out.push_back((uint32_t)(lo + 2 * i));
    }
    return out;
}

uint32_t count_le(const std::vector<uint32_t> &v, uint64_t x)
{
    return (uint32_t)(std::upper_bound(v.begin(), v.end(), x,
                                       [](uint64_t a, uint32_t b) { return a < (uint64_t)b; }) -
                      v.begin());
}

GbTileArgs base_args(gb_ctx *c, Workspace &ws)
{
    GbTileArgs a{};
    a.tile_n = c->tile_n_odd;
    a.halo_bits = c->halo_bits;
    a.primes = c->d_primes;
    a.magic = c->d_magic;
    a.k_first = c->k_first;
    a.k_wg_end = c->k_wg_end;
    a.k_wave_end = c->k_wave_end;
    a.wheel = c->d_wheel;
    a.wheel_len = c->wheel_len;
    a.wheel_max = c->prm.wheel_max;
    a.list = ws.list.p;
    a.list_count = ws.counters.p;
    a.list_cap = c->prm.max_unresolved;
    a.queue = ws.counters.p + 1;
    a.cls = c->d_cls;
    a.cls_words = c->cls_words;
    a.np_cls = c->np_cls;
    a.hk = c->hk;
    a.sb_per_tile = c->sb_per_tile;
    a.wheel6 = c->d_wheel6;
    a.wheel6_len = c->wheel6_len;
    a.wheel6_stride = c->wheel6_stride;
    a.k6_first = c->k6_first;
    a.k6_wave_end = c->k6_wave_end;
    a.k6_single = c->k6_single;
    a.pmax_fast = c->prm.pmax;
    a.prime6 = c->d_prime6;
    a.n_prime6 = c->n_prime6;
    return a;
}

GbMrArgs mr_args(gb_ctx *c, Workspace &ws)
{
    GbMrArgs m{};
    m.list = ws.list.p;
    m.list_count = ws.counters.p;
    m.list_cap = c->prm.max_unresolved;
    m.primes = c->d_primes;
    m.ntab = c->ntab;
    m.budget = c->prm.exhaustive_budget_p;
    return m;
}

uint32_t mr_grid(gb_ctx *c) { return (uint32_t)std::max(64, c->num_cu * 8); }

gb_status enqueue_init(gb_ctx *c, Workspace &ws, const Job &j, hipStream_t st)
{
    GB_HIP(c, gb_launch_init(ws.slots.p, j.nslots, ws.hist.p, j.hist_rows * GB_HIST_BINS_I, ws.counters.p,
                             kCounters, st));
    return GB_OK;
}

hipError_t ensure_plain_streams(gb_ctx *c)
{
    if (c->plain_fork) return hipSuccess;
    hipError_t e;
    for (int l = 0; l < gb_ctx::kPlainLanes - 1; ++l) {
        if ((e = hipStreamCreateWithFlags(&c->plain_st[l], hipStreamNonBlocking)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&c->plain_join[l], hipEventDisableTiming)) != hipSuccess) return e;
    }
    return hipEventCreateWithFlags(&c->plain_fork, hipEventDisableTiming);
}

// Workgroups of a persistent launch of the class kernel.
uint64_t cls_grid(const gb_ctx *c, const Plan &pl)
{
    return std::min<uint64_t>(pl.ntiles, (uint64_t)c->num_cu * c->occ6);
}

gb_status enqueue_tiles(gb_ctx *c, Workspace &ws, const Job &j, hipStream_t st)
{
    GbTileArgs a = base_args(c, ws);
    a.slots = ws.slots.p;
    a.hist = ws.hist.p;
    a.hist_per_slot = j.hist_rows > 1 ? 1u : 0u;
    a.recs = ws.recs.p;
    a.rec_count = ws.counters.p + 2;
    a.rec_cap = ws.recs.cap;
    a.pmin = j.pmin_dev;
    const Plan &pl = *j.pl;
    // minimal p and bulk verification both run the residue-class layout
    // (pmin_bits 1: bulk, no per-n output, hit counts or checksum)
    const bool bulk = j.pmin_bits == 1;
    size_t lds6 = c->lds6;
    a.tile_n = c->tile_n;
    if (!j.persistent) {
        // the plain form's geometry (its plan was cut with kPlanClassPlain)
        a.tile_n = c->tile_np;
        a.sb_per_tile = c->sbp;
        a.k6_wave_end = c->k6p_wave_end;
        a.k6_single = c->k6p_single;
        lds6 = c->lds6p;
    }
    auto launch = [&](const GbTileArgs &b, uint32_t grid, bool pers, hipStream_t ls) -> hipError_t {
        return gb_launch_cls(b, grid, c->threads, lds6, j.pmin_bits, pers, false, ls);
    };
    if (j.persistent) {
        a.win = ws.win.p;
        a.nwin = (uint32_t)pl.w.size();
        a.ntiles = pl.ntiles;
        const uint64_t g = cls_grid(c, pl);
        // the first 7/8 of the tiles round-robin, the rest from the queue
        a.static_tiles = g * ((pl.ntiles - pl.ntiles / 8) / g);
        if (!bulk) {
            a.wg_hist = ws.wgh.p;   // num_cu * occ6 rows, at least g
            a.wg_hist_stride = c->wgh_stride;
        }
        GB_HIP(c, launch(a, (uint32_t)g, true, st));
    } else {
        // One launch per segment.  A segment of S even n is S/T tiles, fewer
        // than the device holds at S = 2^24, so consecutive segments go to
        // the caller's stream and up to three more in turn and run side by
        // side; each segment writes only its own slot, histogram row, tile
        // records and per-n output.
        const int lanes = (int)std::min<size_t>((size_t)c->plain_lanes, pl.w.size());
        if (lanes > 1) {
            GB_HIP(c, ensure_plain_streams(c));
            GB_HIP(c, hipEventRecord(c->plain_fork, st));
            for (int l = 1; l < lanes; ++l) GB_HIP(c, hipStreamWaitEvent(c->plain_st[l - 1], c->plain_fork, 0));
        }
        for (size_t i = 0; i < pl.w.size(); ++i) {
            GbTileArgs b = a;
            b.win = ws.win.p + i;
            b.nwin = 1;
            b.tile0 = pl.w[i].tile_base;
            const uint64_t nt = (pl.w[i].count + a.tile_n - 1) / a.tile_n;
            const int l = (int)(i % (size_t)lanes);
            hipStream_t ls = l == 0 ? st : c->plain_st[l - 1];
            GB_HIP(c, launch(b, (uint32_t)nt, false, ls));
        }
        for (int l = 1; l < lanes; ++l) {
            GB_HIP(c, hipEventRecord(c->plain_join[l - 1], c->plain_st[l - 1]));
            GB_HIP(c, hipStreamWaitEvent(st, c->plain_join[l - 1], 0));
        }
    }
    return GB_OK;
}

gb_status enqueue_rest(gb_ctx *c, Workspace &ws, const Job &j, hipStream_t st)
{
    GbMrArgs m = mr_args(c, ws);
    m.pmin = j.pmin_dev;
    m.pmin_bits = (uint32_t)j.pmin_bits;
    m.slots = ws.slots.p;
    m.hist = ws.hist.p;
    m.hist_per_slot = j.hist_rows > 1 ? 1u : 0u;
    // the class search leaves n_exhaustive to this phase: an n counts when
    // no prime up to P_max gives it a partition (the class lists may stop
    // below P_max when they do not fit the LDS)
    m.count_exh = 1u;
    m.pmax_fast = c->prm.pmax;
    if (j.persistent && j.pmin_bits != 1)
        GB_HIP(c, gb_launch_hist_reduce(ws.wgh.p, (uint32_t)cls_grid(c, *j.pl), c->wgh_stride, c->cls_recs,
                                        c->d_rec_bin, ws.hist.p, st));
    GB_HIP(c, gb_launch_mr(m, mr_grid(c), st));
    GB_HIP(c, gb_launch_argmax(ws.slots.p, ws.recs.p, ws.counters.p + 2, ws.recs.cap, ws.list.p,
                               ws.counters.p, c->prm.max_unresolved, st));
    GB_HIP(c, hipMemcpyAsync(ws.h_slots.p, ws.slots.p, j.nslots * sizeof(GbSlot), hipMemcpyDeviceToHost, st));
    GB_HIP(c, hipMemcpyAsync(ws.h_hist.p, ws.hist.p, j.hist_rows * GB_HIST_BINS_I * 8, hipMemcpyDeviceToHost,
                             st));
    GB_HIP(c, hipMemcpyAsync(ws.h_counters.p, ws.counters.p, kCounters * 8, hipMemcpyDeviceToHost, st));
    return GB_OK;
}

using PhaseFn = gb_status (*)(gb_ctx *, Workspace &, const Job &, hipStream_t);

gb_status capture(gb_ctx *c, Workspace &ws, PhaseFn fn, const Job &j, hipGraphExec_t *out)
{
    hipStream_t cap = nullptr;
    GB_HIP(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return fail(c, GB_EDEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    const gb_status s = fn(c, ws, j, cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap, &g);
    (void)hipStreamDestroy(cap);
    if (s != GB_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    GB_HIP(c, e);
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    GB_HIP(c, e);
    return GB_OK;
}

}  // namespace

hipError_t Workspace::init(uint64_t list_cap)
{
    hipError_t e;
    if ((e = list.ensure(list_cap)) != hipSuccess) return e;
    if ((e = counters.ensure(kCounters)) != hipSuccess) return e;
    if ((e = h_counters.ensure(kCounters)) != hipSuccess) return e;
    for (hipEvent_t *ev : {&ev0, &ev1, &evt0, &evt1})
        if ((e = hipEventCreate(ev)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&done, hipEventDisableTiming)) != hipSuccess) return e;
    return hipSuccess;
}

void Workspace::drop_graphs()
{
    for (auto &g : gexec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

void Workspace::release()
{
    drop_graphs();
    win.release();
    slots.release();
    hist.release();
    recs.release();
    wgh.release();
    list.release();
    counters.release();
    pmin.release();
    q.release();
    pc_bits.release();
    pc_counts.release();
    pc_red.release();
    h_pc_red.release();
    big_n.release();
    big_state.release();
    big_list.release();
    h_big.release();
    big_p.release();
    h_slots.release();
    h_hist.release();
    h_counters.release();
    h_q.release();
    for (hipEvent_t *ev : {&ev0, &ev1, &evt0, &evt1, &done}) {
        if (*ev) (void)hipEventDestroy(*ev);
        *ev = nullptr;
    }
}

gb_status apply_params(gb_ctx *c, const gb_params *in)
{
    gb_params p{};
    if (in) p = *in;
    if (p.pmax == 0) p.pmax = 8192;
    if (p.seg_log2 == 0) p.seg_log2 = 24;
    if (p.tile_log2 == 0) p.tile_log2 = 19;
    if (p.wg_threads == 0) p.wg_threads = 512;
    if (p.wheel_max == 0) p.wheel_max = 19;
    if (p.search_mode == 0) p.search_mode = 1;
    if (p.max_hi == 0) p.max_hi = kDefaultMaxHi;
    if (p.max_unresolved == 0) p.max_unresolved = 1ull << 20;
    if (p.mem_budget == 0) p.mem_budget = 4ull << 30;
    if (p.pmax > 65535) return fail(c, GB_EINVAL, "pmax must be at most 65535");
    if (p.seg_log2 < 16 || p.seg_log2 > 30) return fail(c, GB_EINVAL, "seg_log2 must be in 16..30");
    if (p.tile_log2 < 12 || p.tile_log2 > 20) return fail(c, GB_EINVAL, "tile_log2 must be in 12..20");
    if (p.tile_log2 > p.seg_log2) return fail(c, GB_EINVAL, "tile_log2 must not exceed seg_log2");
    if (p.wg_threads != 256 && p.wg_threads != 512 && p.wg_threads != 1024)
        return fail(c, GB_EINVAL, "wg_threads must be 256, 512 or 1024");
    if (p.wheel_max != 7 && p.wheel_max != 11 && p.wheel_max != 13 && p.wheel_max != 17 && p.wheel_max != 19)
        return fail(c, GB_EINVAL, "wheel_max must be 7, 11, 13, 17 or 19");
    if (p.search_mode != 1) return fail(c, GB_EINVAL, "search_mode must be 1 (or 0 for the default)");
    if (p.reserved != 0) return fail(c, GB_EINVAL, "reserved must be 0");
    if (p.max_hi > GB_MAX_N) return fail(c, GB_EINVAL, "max_hi must be at most 2^63");
    if (p.max_hi < 1024) p.max_hi = 1024;
    c->prm = p;
    return GB_OK;
}

gb_status build_tables(gb_ctx *c)
{
    // odd primes up to sqrt(max_hi + slack), and at least past 2^16
    uint64_t lim = isqrt64(c->prm.max_hi + (1ull << 30)) + 2;
    lim = std::max<uint64_t>(lim, 70000);
    c->h_primes = host_odd_primes(lim);
    c->table_limit = lim;
    c->ntab = c->h_primes.size();
    std::vector<unsigned long long> magic(c->ntab);
    for (uint64_t i = 0; i < c->ntab; ++i) magic[i] = ~0ull / c->h_primes[i];
    GB_HIP(c, hipMalloc(&c->d_primes, c->ntab * 4));
    GB_HIP(c, hipMalloc(&c->d_magic, c->ntab * 8));
    GB_HIP(c, hipMemcpy(c->d_primes, c->h_primes.data(), c->ntab * 4, hipMemcpyHostToDevice));
    GB_HIP(c, hipMemcpy(c->d_magic, magic.data(), c->ntab * 8, hipMemcpyHostToDevice));
    // plane-sieve entries: p, the first k of plane 6k+1 that p divides, 1/p
    c->n_prime6 = (uint32_t)count_le(c->h_primes, (1u << 27) - 1u);
    std::vector<uint32_t> e6(4ull * c->n_prime6);
    for (uint32_t i = 0; i < c->n_prime6; ++i) {
        const uint32_t p = c->h_primes[i];
        const double r = 1.0 / (double)p;
        uint64_t rb;
        std::memcpy(&rb, &r, 8);
        e6[4ull * i] = p;
        e6[4ull * i + 1] = (uint32_t)(((uint64_t)(p % 6u) * p - 1u) / 6u);   // 6 k + 1 = (p mod 6) p
        e6[4ull * i + 2] = (uint32_t)rb;
        e6[4ull * i + 3] = (uint32_t)(rb >> 32);
    }
    GB_HIP(c, hipMalloc(&c->d_prime6, e6.size() * 4 + 16));
    GB_HIP(c, hipMemcpy(c->d_prime6, e6.data(), e6.size() * 4, hipMemcpyHostToDevice));
    return GB_OK;
}

void free_tables(gb_ctx *c)
{
    for (void *q : {(void *)c->d_primes, (void *)c->d_magic, (void *)c->d_prime6, (void *)c->d_wheel,
                    (void *)c->d_cls, (void *)c->d_wheel6, (void *)c->d_rec_bin})
        if (q) (void)hipFree(q);
    c->d_rec_bin = nullptr;
    c->d_primes = nullptr;
    c->d_magic = nullptr;
    c->d_prime6 = nullptr;
    c->d_wheel = nullptr;
    c->d_cls = nullptr;
    c->d_wheel6 = nullptr;
}

namespace {

// The class table of the search split by residue mod 6 for the first np
// odd primes of the table (layout: GB_CLS_* in gb_internal.h), and its
// plane halo hk.  Class h = a/2 lists the primes p with a - p not a
// multiple of 3, in groups of four whose probes start within two rows of
// the group's lowest start; a group that would be wider is closed early and
// padded with copies of its last entry (a copy cannot hit an n twice).
std::vector<uint32_t> class_table(const gb_ctx *c, uint32_t np, uint32_t &hk)
{
    std::vector<uint32_t> T(GB_CLS_HDR, 0u);
    // q = n - p lies d stretches of 6 below n, in the plane of c = (a - p) mod 6
    uint32_t dmax = 0;
    for (uint32_t h = 0; h < 3; ++h)
        for (uint32_t e = 0; e < np; ++e) {
            const uint32_t p = c->h_primes[e], a = 2 * h, cc = (a + 6 - p % 6) % 6;
            if (cc == 1 || cc == 5) dmax = std::max(dmax, (p + cc - a) / 6);
        }
    hk = std::max<uint32_t>(64, (dmax + 63) / 64 * 64);
    std::vector<uint32_t> rec;
    for (uint32_t h = 0; h < 3; ++h) {
        struct Ent { uint32_t sb, plane, g; };
        std::vector<Ent> ent;
        for (uint32_t e = 0; e < np; ++e) {
            const uint32_t p = c->h_primes[e], a = 2 * h, cc = (a + 6 - p % 6) % 6;
            if (cc != 1 && cc != 5) continue;
            ent.push_back({hk - (p + cc - a) / 6, cc == 5 ? 1u : 0u, 65536u - (p + 1) / 2});
        }
        std::vector<std::vector<Ent>> groups;
        for (size_t e = 0; e < ent.size();) {
            std::vector<Ent> gr{ent[e]};
            size_t f = e + 1;
            // start bits fall with p: the first entry has the highest row
            while (f < ent.size() && gr.size() < 4 && ent[e].sb / 32 - ent[f].sb / 32 <= 1) gr.push_back(ent[f++]);
            while (gr.size() < 4) gr.push_back(gr.back());
            groups.push_back(gr);
            e = f;
        }
        const uint32_t real = (uint32_t)groups.size();
        for (int k = 0; k < 2 && real; ++k) groups.push_back(std::vector<Ent>(4, groups[real - 1][3]));
        T[3 * h] = (uint32_t)rec.size() * 4u;
        T[3 * h + 1] = real;
        T[3 * h + 2] = T[3 * h] + 48u * real;
        for (const auto &gr : groups) {
            const uint32_t R = gr[3].sb / 32;   // the group's lowest row
            uint32_t grp[12] = {};
            for (uint32_t u = 0; u < 4; ++u) {
                const Ent &en = gr[u];
                grp[u] = ((8u * R) << 16) | (en.plane << 6) | ((en.sb / 32 - R) << 5) | (en.sb & 31u);
                grp[4 + u] = en.g;
            }
            rec.insert(rec.end(), grp, grp + 12);
        }
    }
    rec.resize(rec.size() + 3 * 12, 0u);   // what a lane of an empty last list reads past the end
    T.insert(T.end(), rec.begin(), rec.end());
    return T;
}

}  // namespace

// Launch geometry and wheel pattern for the current parameters.
gb_status setup_geometry(gb_ctx *c)
{
    const gb_params &p = c->prm;
    c->tile_n_odd = 1u << p.tile_log2;
    c->threads = p.wg_threads;
    c->np_search = count_le(c->h_primes, p.pmax);
    const uint32_t need = (p.pmax + 1) / 2;
    c->halo_bits = std::max<uint32_t>(64, (need + 63) / 64 * 64);
    c->k_first = count_le(c->h_primes, p.wheel_max);
    const uint32_t nbits = c->tile_n_odd + c->halo_bits;
    // Marking classes by hits per tile, H = nbits/p.  A class pays a fixed
    // cost per prime (first strike, loop set-up) in every thread it uses:
    // - whole workgroup for p < nbits/(32 threads): H/threads >= 32 strides
    //   per thread, the only primes that would unbalance the waves;
    // - one wave per prime while H >= 256: 64 lanes x set-up plus 2 VALU
    //   per clear beats one lane's 6 VALU per clear (measured flat between
    //   H >= 96 and H >= 384, and for 4 to 64 strides per thread);
    // - one lane per prime above.
    c->k_wg_end = std::max(c->k_first, count_le(c->h_primes, nbits / (32 * c->threads)));
    c->k_wave_end = std::max(c->k_wg_end, count_le(c->h_primes, nbits / 256));
    c->lds = gb_tile_lds_bytes(c->tile_n_odd, c->halo_bits, c->k_wave_end - c->k_first);
    if (c->lds > 160 * 1024)
        return fail(c, GB_EINVAL, "tile does not fit in LDS (" + std::to_string(c->lds) +
                                      " bytes); lower tile_log2, wg_threads or pmax");
    hipDeviceProp_t prop;
    GB_HIP(c, hipGetDeviceProperties(&prop, p.device));
    c->num_cu = prop.multiProcessorCount;
    {
        const char *q = std::getenv("GPU_MAX_HW_QUEUES");
        const long hw = q ? std::strtol(q, nullptr, 10) : 4;
        c->plain_hwq = (int)std::max<long>(1, std::min<long>(gb_ctx::kPlainLanes, hw > 0 ? hw : 4));
    }
    GB_HIP(c, gb_prepare_tiles(c->threads, c->lds));
    // wheel pattern over (v-1)/2 for odd v: bit g set iff 2g+1 is coprime to the wheel
    static const uint32_t wp[] = {3, 5, 7, 11, 13, 17, 19};
    uint32_t L = 1;
    for (uint32_t q : wp)
        if (q <= p.wheel_max) L *= q;
    std::vector<uint32_t> pat((L + 64 + 31) / 32 + 1, 0u);
    for (uint32_t g = 0; g < L + 64; ++g) {
        const uint32_t v = 2 * (g % L) + 1;
        bool ok = true;
        for (uint32_t q : wp)
            if (q <= p.wheel_max && v % q == 0) ok = false;
        if (ok) pat[g >> 5] |= 1u << (g & 31);
    }
    if (c->d_wheel) (void)hipFree(c->d_wheel);
    c->d_wheel = nullptr;
    GB_HIP(c, hipMalloc(&c->d_wheel, pat.size() * 4));
    GB_HIP(c, hipMemcpy(c->d_wheel, pat.data(), pat.size() * 4, hipMemcpyHostToDevice));
    c->wheel_len = L;

    // ---- search split by residue mod 6: stretches, class lists, planes ----
    // A class tile spends 2/3 of a plane bit per n.  It is the largest that
    // fits the LDS beside the lists, from 2^tile_log2 / 96 stretches (twice
    // the n of an odd-number tile of 2^tile_log2 bits) down in steps of
    // 1/64, and at least 2^tile_log2 / 192 stretches (the n of that tile):
    // per-tile costs (first strikes of every sieving prime, the search's
    // tail, barriers) then spread over more n.
    const uint32_t sb_max = std::max<uint32_t>(1, (1u << p.tile_log2) / 96u);
    const uint32_t sb_min = std::max<uint32_t>(1, (1u << p.tile_log2) / 192u);
    c->sb_per_tile = sb_max;
    c->k6_first = count_le(c->h_primes, std::max<uint32_t>(3, p.wheel_max));
    // the class lists hold every odd prime <= P_max when they fit the LDS
    // beside the planes, else the longest prefix that does; the exhaustive
    // phase takes the n they leave from the next prime on
    uint32_t np = c->np_search;
    std::vector<uint32_t> T;
    for (;;) {
        T = class_table(c, np, c->hk);
        const uint32_t Lk = c->hk + 64 * c->sb_per_tile;
        // one wave per prime up to Lk/64 (at least two strikes per lane and
        // plane); no whole-workgroup class: at 10^12 striding a workgroup over
        // each prime up to Lk/threads took 28.15 ms a launch, up to
        // Lk/(8 threads) 27.58 ms, and none 27.28 ms (same box)
        c->k6_wave_end = std::max(c->k6_first, count_le(c->h_primes, Lk / 64));
        c->k6_single = std::max(c->k6_wave_end, count_le(c->h_primes, Lk - 1));
        c->lds6 = gb_cls_lds_bytes(c->sb_per_tile, c->hk, (uint32_t)T.size());
        if (c->lds6 <= 160 * 1024 || np == 0) break;
        if (c->sb_per_tile > sb_min)
            c->sb_per_tile = std::max(sb_min, c->sb_per_tile - std::max<uint32_t>(1, c->sb_per_tile / 64));
        else
            np -= std::max<uint32_t>(1, np / 16);
    }
    c->tile_n = 192u * c->sb_per_tile;
    // The plain form launches one grid per segment of S even n, with up to
    // plain_hwq segments in flight: its tiles are cut so that a segment
    // makes num_cu / plain_hwq of them (never more n than a batched tile);
    // then the segments in flight are cut to the number whose tiles exceed
    // the CUs by at most 1/8 (a larger backlog delays each segment's last
    // tiles, and with them the next launch of its stream).
    {
        const uint64_t S = 1ull << p.seg_log2;
        const uint64_t want = std::max<uint64_t>(1, ((uint64_t)c->num_cu + c->plain_hwq - 1) / (uint64_t)c->plain_hwq);
        // a segment with its lead (< 192 n) in `want` tiles, or in as many
        // more as batched-size tiles need, all of one size (no sliver tile:
        // it would pay every sieving prime's first strikes for a few n)
        const uint64_t span = S + 191;
        const uint64_t k = std::max<uint64_t>(want, (span + 192ull * c->sb_per_tile - 1) / (192ull * c->sb_per_tile));
        c->sbp = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(c->sb_per_tile, (span + 192 * k - 1) / (192 * k)));
        const uint64_t fit = ((uint64_t)c->num_cu + c->num_cu / 8) / k;
        c->plain_lanes = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)c->plain_hwq, fit));
        c->tile_np = 192u * c->sbp;
        const uint32_t Lk = c->hk + 64 * c->sbp;
        c->k6p_wave_end = std::max(c->k6_first, count_le(c->h_primes, Lk / 64));
        c->k6p_single = std::max(c->k6p_wave_end, count_le(c->h_primes, Lk - 1));
        c->lds6p = gb_cls_lds_bytes(c->sbp, c->hk, (uint32_t)T.size());
    }
    if (c->lds6 > 160 * 1024)
        return fail(c, GB_EINVAL, "tile does not fit in LDS (" + std::to_string(c->lds6) + " bytes); lower tile_log2");
    c->np_cls = np;
    c->cls_words = (uint32_t)T.size();
    // the histogram bin of every probe record of the real groups, in the
    // order in which a workgroup stores its counts
    {
        std::vector<uint32_t> bins;
        for (uint32_t h = 0; h < 3; ++h) {
            const uint32_t first = T[3 * h] / 4, groups = T[3 * h + 1];
            for (uint32_t e = 0; e < 4 * groups; ++e) {
                const uint32_t wo = first + 12 * (e >> 2) + (e & 3);
                const uint32_t pr = 131071u - 2u * T[GB_CLS_HDR + wo + 4];
                bins.push_back(count_le(c->h_primes, pr - 1) + 1);   // 2 -> 0, 3 -> 1, ...
            }
        }
        c->cls_recs = (uint32_t)bins.size();
        c->wgh_stride = (c->cls_recs + 1 + 15) / 16 * 16;   // 64-byte rows
        if (c->d_rec_bin) (void)hipFree(c->d_rec_bin);
        c->d_rec_bin = nullptr;
        GB_HIP(c, hipMalloc(&c->d_rec_bin, std::max<size_t>(bins.size(), 1) * 4));
        if (!bins.empty())
            GB_HIP(c, hipMemcpy(c->d_rec_bin, bins.data(), bins.size() * 4, hipMemcpyHostToDevice));
    }
    if (c->d_cls) (void)hipFree(c->d_cls);
    c->d_cls = nullptr;
    GB_HIP(c, hipMalloc(&c->d_cls, T.size() * 4));
    GB_HIP(c, hipMemcpy(c->d_cls, T.data(), T.size() * 4, hipMemcpyHostToDevice));
    GB_HIP(c, gb_cls_prepare(c->threads, c->lds6));
    int occ = 0;
    GB_HIP(c, gb_cls_occupancy(c->threads, c->lds6, &occ));
    c->occ6 = std::max(occ, 1);
    // plane i (c = 1, 5): bit k set iff 6k + c is prime to every wheel prime
    // 5 .. wheel_max (period the product of those primes)
    uint32_t P = 1;
    for (uint32_t q : wp)
        if (q >= 5 && q <= p.wheel_max) P *= q;
    const uint32_t stride = (P + 64 + 31) / 32 + 1;
    std::vector<uint32_t> pat6(2ull * stride, 0u);
    for (uint32_t i = 0; i < 2; ++i)
        for (uint32_t k = 0; k < P + 64; ++k) {
            const uint64_t v = 6ull * (k % P) + (i ? 5 : 1);
            bool ok = true;
            for (uint32_t q : wp)
                if (q >= 5 && q <= p.wheel_max && v % q == 0) ok = false;
            if (ok) pat6[i * stride + (k >> 5)] |= 1u << (k & 31);
        }
    if (c->d_wheel6) (void)hipFree(c->d_wheel6);
    c->d_wheel6 = nullptr;
    GB_HIP(c, hipMalloc(&c->d_wheel6, pat6.size() * 4));
    GB_HIP(c, hipMemcpy(c->d_wheel6, pat6.data(), pat6.size() * 4, hipMemcpyHostToDevice));
    c->wheel6_len = P;
    c->wheel6_stride = stride;
    c->ws.drop_graphs();
    return GB_OK;
}

// Split windows into tiles and fill the derived window fields; GB_ERANGE
// when a window reaches past the resident sieving primes.  For the search
// (minimal p and bulk, split by residue mod 6) each window's first n moves
// down to a multiple of 384, the n added in front counted in `lead` (the
// kernel masks them).
gb_status plan_windows(gb_ctx *c, Plan &pl, PlanKind kind)
{
    // the sieve dump cuts odd-number tiles; the searches residue-class ones
    const uint64_t T = kind == kPlanClass ? c->tile_n : kind == kPlanClassPlain ? c->tile_np : c->tile_n_odd;
    const uint64_t A = 384;
    uint64_t tb = 0, off = 0;
    for (auto &w : pl.w) {
        const uint64_t user_count = w.count;
        w.lead = (kind != kPlanSieve && user_count) ? (uint32_t)((w.first_n % A) / 2) : 0u;
        w.pad = 0;
        w.first_n -= 2ull * w.lead;
        w.count += w.lead;
        const uint64_t nt = (w.count + T - 1) / T;
        w.tile_base = tb;
        w.out_off = off;
        const uint64_t top = w.first_n + 2 * T * nt + 1;
        const uint64_t r = isqrt64(top);
        if (r > c->table_limit)
            return fail(c, GB_ERANGE, "window top beyond the resident sieving primes (raise max_hi)");
        w.np_sieve = count_le(c->h_primes, r);
        tb += nt;
        off += user_count;
    }
    pl.ntiles = tb;
    pl.total_n = off;
    return GB_OK;
}

gb_status ensure_workspace(gb_ctx *c, Workspace &ws, const Plan &pl, size_t nslots, size_t hist_rows)
{
    GB_HIP(c, ws.win.ensure(pl.w.size()));
    GB_HIP(c, ws.slots.ensure(nslots));
    GB_HIP(c, ws.hist.ensure(hist_rows * GB_HIST_BINS_I));
    GB_HIP(c, ws.recs.ensure(std::max<uint64_t>(pl.ntiles, 1)));
    GB_HIP(c, ws.wgh.ensure((size_t)c->num_cu * (size_t)c->occ6 * c->wgh_stride));
    GB_HIP(c, ws.h_slots.ensure(nslots));
    GB_HIP(c, ws.h_hist.ensure(hist_rows * GB_HIST_BINS_I));
    return GB_OK;
}

gb_status run_job(gb_ctx *c, Workspace &ws, const Job &j, const GraphKey &key, bool use_graph, hipStream_t st)
{
    if (!use_graph) {
        gb_status s = enqueue_init(c, ws, j, st);
        if (s != GB_OK) return s;
        GB_HIP(c, hipEventRecord(ws.evt0, st));
        s = enqueue_tiles(c, ws, j, st);
        if (s != GB_OK) return s;
        GB_HIP(c, hipEventRecord(ws.evt1, st));
        return enqueue_rest(c, ws, j, st);
    }
    if (!(ws.gexec[0] && ws.gkey == key)) {
        ws.drop_graphs();
        const PhaseFn fns[3] = {enqueue_init, enqueue_tiles, enqueue_rest};
        for (int i = 0; i < 3; ++i) {
            const gb_status s = capture(c, ws, fns[i], j, &ws.gexec[i]);
            if (s != GB_OK) {
                ws.drop_graphs();
                return s;
            }
        }
        ws.gkey = key;
    }
    GB_HIP(c, hipGraphLaunch(ws.gexec[0], st));
    GB_HIP(c, hipEventRecord(ws.evt0, st));
    GB_HIP(c, hipGraphLaunch(ws.gexec[1], st));
    GB_HIP(c, hipEventRecord(ws.evt1, st));
    GB_HIP(c, hipGraphLaunch(ws.gexec[2], st));
    return GB_OK;
}

gb_status enqueue_queries(gb_ctx *c, Workspace &ws, uint64_t k, const unsigned long long *dn,
                          unsigned long long *dp, hipStream_t st)
{
    GB_HIP(c, gb_launch_make_queries(ws.list.p, dn, k, ws.counters.p, st));
    const GbMrArgs m = mr_args(c, ws);
    GB_HIP(c, gb_launch_mr(m, (uint32_t)std::min<uint64_t>(mr_grid(c), (k + 3) / 4), st));
    GB_HIP(c, gb_launch_finish_queries(ws.list.p, k, dp, st));
    return GB_OK;
}

gb_status enqueue_sieve(gb_ctx *c, Workspace &ws, uint64_t w0, uint64_t nbits, uint32_t *bits, hipStream_t st)
{
    Plan pl;
    pl.w.resize(1);
    pl.w[0].first_n = w0 - 1 + 2ull * c->halo_bits;  // makes the tile window start at w0
    pl.w[0].count = nbits;
    pl.w[0].slot = 0;
    gb_status stt = plan_windows(c, pl, kPlanSieve);
    if (stt != GB_OK) return stt;
    stt = ensure_workspace(c, ws, pl, 1, 1);
    if (stt != GB_OK) return stt;
    GB_HIP(c, hipMemcpyAsync(ws.win.p, pl.w.data(), sizeof(GbWindow), hipMemcpyHostToDevice, st));
    GbTileArgs a = base_args(c, ws);
    a.win = ws.win.p;
    a.nwin = 1;
    a.tile0 = 0;
    a.sieve_out = bits;
    GB_HIP(c, gb_launch_tiles(a, (uint32_t)pl.ntiles, c->threads, c->lds, st));
    return GB_OK;
}

// The sieve of the search alone: planes over k in [k0, k0 + nk), as the
// tiles of one window of 3 nk even n from 6 k0 (k0, nk multiples of 64).
gb_status enqueue_sieve6(gb_ctx *c, Workspace &ws, uint64_t k0, uint64_t nk, uint32_t *planes, hipStream_t st)
{
    Plan pl;
    pl.w.resize(1);
    pl.w[0].first_n = 6ull * k0;
    pl.w[0].count = 3ull * nk;
    pl.w[0].slot = 0;
    gb_status stt = plan_windows(c, pl, kPlanClass);
    if (stt != GB_OK) return stt;
    stt = ensure_workspace(c, ws, pl, 1, 1);
    if (stt != GB_OK) return stt;
    GB_HIP(c, hipMemcpyAsync(ws.win.p, pl.w.data(), sizeof(GbWindow), hipMemcpyHostToDevice, st));
    GbTileArgs a = base_args(c, ws);
    a.tile_n = c->tile_n;
    a.win = ws.win.p;
    a.nwin = 1;
    a.tile0 = 0;
    a.sieve_out = planes;
    a.sieve_stride = nk / 32;
    GB_HIP(c, gb_launch_cls(a, (uint32_t)pl.ntiles, c->threads, c->lds6, 0, false, true, st));
    return GB_OK;
}

void merge_slot(gb_summary &acc, const GbSlot &s)
{
    acc.count += s.count;
    acc.checksum += s.checksum;
    acc.n_exhaustive += s.n_exhaustive;
    acc.n_failed += s.n_failed;
    const uint64_t ff = s.first_failed_n == ~0ull ? 0 : s.first_failed_n;
    if (ff && (acc.first_failed_n == 0 || ff < acc.first_failed_n)) acc.first_failed_n = ff;
    const uint64_t am = s.max_p ? s.argmax_n : 0;
    if (s.max_p > acc.max_p || (s.max_p == acc.max_p && s.max_p && am < acc.argmax_n)) {
        acc.max_p = s.max_p;
        acc.argmax_n = am;
    }
}

}  // namespace gbrt

using namespace gbrt;

namespace {

gb_status finish_list(gb_ctx *c)
{
    c->last_list_valid = false;
    const uint64_t cnt = c->ws.h_counters.p[0];
    if (cnt > c->prm.max_unresolved)
        return fail(c, GB_ENOMEM,
                    "exhaustive list overflow: " + std::to_string(cnt) + " n left by the fast path, capacity " +
                        std::to_string(c->prm.max_unresolved) + " (raise max_unresolved or pmax)");
    c->last_list.resize(cnt);
    if (cnt)
        GB_HIP(c, hipMemcpy(c->last_list.data(), c->ws.list.p, cnt * sizeof(GbExh), hipMemcpyDeviceToHost));
    c->last_list_valid = true;
    return GB_OK;
}

// bulk: verification only (no per-n p_min, histogram or checksum), which
// the tile kernel selects by a per-n output width of 1
gb_status run_range(gb_ctx *c, uint64_t lo, uint64_t hi, gb_result *res, void *stream, bool batched,
                    bool bulk = false)
{
    if (!c || !res) return fail(c, GB_EINVAL, "null context or result");
    if (hi > GB_MAX_N) return fail(c, GB_EINVAL, "hi above 2^63");
    if (hi > c->prm.max_hi) return fail(c, GB_ERANGE, "hi above the context's max_hi");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace &ws = c->ws;
    if (lo < 4) lo = 4;
    if (lo & 1) ++lo;
    if (hi & 1) --hi;
    res->count = res->max_p = res->argmax_n = res->checksum = 0;
    res->n_exhaustive = res->n_failed = res->first_failed_n = res->n_segments = 0;
    res->device_ms = res->tile_ms = 0;
    res->tile_launches = 0;
    if (res->hist) std::memset(res->hist, 0, GB_HIST_BINS * 8);
    if (lo > hi) return GB_OK;
    if (res->pmin && res->pmin_bits != 16 && res->pmin_bits != 32)
        return fail(c, GB_EINVAL, "pmin_bits must be 16 or 32");
    if (bulk && (res->pmin || res->hist || res->seg_hist))
        return fail(c, GB_EINVAL, "the bulk form gives no per-n output or histograms");
    const uint64_t C = (hi - lo) / 2 + 1;
    const uint64_t S = 1ull << c->prm.seg_log2;
    const uint64_t nseg = (C + S - 1) / S;
    if (res->seg_hist && res->seg_hist_rows < nseg) return fail(c, GB_EINVAL, "seg_hist has fewer rows than segments");
    // Segments share one summary slot unless the caller wants their
    // histograms apart: the host merges the slots anyway, and with one slot a
    // persistent workgroup flushes its slot sums once for all its tiles
    // instead of once per tile (its tiles lie in different segments).
    const uint64_t nslots = res->seg_hist ? nseg : 1;
    Plan pl;
    pl.w.resize(nseg);
    for (uint64_t s = 0; s < nseg; ++s) {
        pl.w[s].first_n = lo + 2 * S * s;
        pl.w[s].count = std::min(S, C - S * s);
        pl.w[s].slot = res->seg_hist ? (uint32_t)s : 0u;
    }
    gb_status stt = plan_windows(c, pl, batched ? kPlanClass : kPlanClassPlain);
    if (stt != GB_OK) return stt;
    const size_t hist_rows = res->seg_hist ? nseg : 1;
    stt = ensure_workspace(c, ws, pl, nslots, hist_rows);
    if (stt != GB_OK) return stt;
    const int pb = bulk ? 1 : (res->pmin ? (int)res->pmin_bits : 0);
    void *pmin_dev = nullptr;
    if (res->pmin) {
        if (res->pmin_on_device) {
            pmin_dev = res->pmin;
        } else {
            GB_HIP(c, ws.pmin.ensure(C * (pb / 8)));
            pmin_dev = ws.pmin.p;
        }
    }
    GB_HIP(c, hipMemcpyAsync(ws.win.p, pl.w.data(), nseg * sizeof(GbWindow), hipMemcpyHostToDevice, st));
    GB_HIP(c, hipEventRecord(ws.ev0, st));
    GraphKey key;
    key.generation = g_buffer_generation.load();
    key.kind = 1;
    key.nwin = nseg;
    key.ntiles = pl.ntiles;
    key.hist_rows = hist_rows;
    key.pmin = pmin_dev;
    key.pmin_bits = pb;
    key.stream = st;
    Job j;
    j.pl = &pl;
    j.nslots = nslots;
    j.hist_rows = hist_rows;
    j.pmin_dev = pmin_dev;
    j.pmin_bits = pb;
    j.persistent = batched;
    stt = run_job(c, ws, j, key, batched, st);
    if (stt != GB_OK) return stt;
    GB_HIP(c, hipEventRecord(ws.ev1, st));
    GB_HIP(c, hipStreamSynchronize(st));
    float ms = 0;
    GB_HIP(c, hipEventElapsedTime(&ms, ws.ev0, ws.ev1));
    res->device_ms = ms;
    GB_HIP(c, hipEventElapsedTime(&ms, ws.evt0, ws.evt1));
    res->tile_ms = ms;
    res->tile_launches = batched ? 1 : nseg;
    gb_summary tot{};
    for (uint64_t s = 0; s < nslots; ++s) merge_slot(tot, ws.h_slots.p[s]);
    res->count = tot.count;
    res->max_p = tot.max_p;
    res->argmax_n = tot.argmax_n;
    res->checksum = bulk ? 0 : tot.checksum;
    res->n_exhaustive = tot.n_exhaustive;
    res->n_failed = tot.n_failed;
    res->first_failed_n = tot.first_failed_n;
    res->n_segments = nseg;
    if (res->hist)
        for (size_t r = 0; r < hist_rows; ++r)
            for (uint32_t i = 0; i < GB_HIST_BINS; ++i) res->hist[i] += ws.h_hist.p[r * GB_HIST_BINS_I + i];
    if (res->seg_hist) std::memcpy(res->seg_hist, ws.h_hist.p, nseg * GB_HIST_BINS_I * 8);
    stt = finish_list(c);
    if (stt != GB_OK) return stt;
    if (res->pmin && !res->pmin_on_device)
        GB_HIP(c, hipMemcpy(res->pmin, pmin_dev, C * (pb / 8), hipMemcpyDeviceToHost));
    if (res->count != C)
        return fail(c, GB_EDEVICE, "internal: counted " + std::to_string(res->count) + " n, expected " +
                                       std::to_string(C));
    if (res->n_failed) return fail(c, GB_EUNRESOLVED, "n without a partition within the budget");
    return GB_OK;
}

}  // namespace

extern "C" {

const char *gb_status_str(gb_status st)
{
    switch (st) {
    case GB_OK: return "GB_OK";
    case GB_EINVAL: return "GB_EINVAL";
    case GB_ERANGE: return "GB_ERANGE";
    case GB_ENOMEM: return "GB_ENOMEM";
    case GB_EDEVICE: return "GB_EDEVICE";
    case GB_EUNRESOLVED: return "GB_EUNRESOLVED";
    }
    return "GB_UNKNOWN";
}

const char *gb_last_error(const gb_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

gb_status gb_create(gb_ctx **out, const gb_params *prm)
{
    if (!out) return GB_EINVAL;
    *out = nullptr;
    gb_ctx *c = new (std::nothrow) gb_ctx();
    if (!c) return GB_ENOMEM;
    gb_status st = apply_params(c, prm);
    if (st != GB_OK) {
        delete c;
        return st;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || c->prm.device < 0 || c->prm.device >= ndev) {
        delete c;
        return GB_EDEVICE;
    }
    auto bail = [&](gb_status s) {
        gb_destroy(c);
        return s;
    };
    if (hipSetDevice(c->prm.device) != hipSuccess) return bail(GB_EDEVICE);
    if (noalloc_setup(c->prm.device) != hipSuccess) return bail(GB_EDEVICE);
    st = build_tables(c);
    if (st != GB_OK) return bail(st);
    if (c->ws.init(c->prm.max_unresolved) != hipSuccess) return bail(GB_ENOMEM);
    st = setup_geometry(c);
    if (st != GB_OK) return bail(st);
    *out = c;
    return GB_OK;
}

void gb_destroy(gb_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->prm.device);
    (void)hipDeviceSynchronize();
    for (int l = 0; l < gb_ctx::kPlainLanes - 1; ++l) {
        if (c->plain_st[l]) (void)hipStreamDestroy(c->plain_st[l]);
        if (c->plain_join[l]) (void)hipEventDestroy(c->plain_join[l]);
    }
    if (c->plain_fork) (void)hipEventDestroy(c->plain_fork);
    c->ws.release();
    free_tables(c);
    delete c;
}

gb_status gb_get_params(const gb_ctx *c, gb_params *out)
{
    if (!c || !out) return GB_EINVAL;
    *out = c->prm;
    return GB_OK;
}

gb_status gb_tile_geometry(const gb_ctx *c, uint64_t *cls_tile_n, uint64_t *cls_lds_bytes,
                           uint64_t *cls_list_primes, uint64_t *bulk_tile_n)
{
    if (!c) return GB_EINVAL;
    if (cls_tile_n) *cls_tile_n = c->tile_n;
    if (cls_lds_bytes) *cls_lds_bytes = c->lds6;
    if (cls_list_primes) *cls_list_primes = c->np_cls;
    if (bulk_tile_n) *bulk_tile_n = c->tile_n;
    return GB_OK;
}

gb_status gb_verify_range(gb_ctx *c, uint64_t lo, uint64_t hi, gb_result *res, void *stream)
{
    if (!c) return GB_EINVAL;
    if (hipSetDevice(c->prm.device) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    return run_range(c, lo, hi, res, stream, false);
}

gb_status gb_verify_range_batched(gb_ctx *c, uint64_t lo, uint64_t hi, gb_result *res, void *stream)
{
    if (!c) return GB_EINVAL;
    if (hipSetDevice(c->prm.device) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    return run_range(c, lo, hi, res, stream, true);
}

gb_status gb_verify_range_bulk(gb_ctx *c, uint64_t lo, uint64_t hi, gb_result *res, void *stream)
{
    if (!c) return GB_EINVAL;
    if (hipSetDevice(c->prm.device) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    return run_range(c, lo, hi, res, stream, true, true);
}

gb_status gb_verify_windows(gb_ctx *c, const gb_window *w, size_t k, uint16_t *pmin, gb_summary *sums,
                            uint64_t *hist, void *stream)
{
    if (!c || (!w && k)) return fail(c, GB_EINVAL, "null context or windows");
    if (hipSetDevice(c->prm.device) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace &ws = c->ws;
    if (hist) std::memset(hist, 0, GB_HIST_BINS * 8);
    if (k == 0) return GB_OK;
    if (k > 0xFFFFFFFFull) return fail(c, GB_EINVAL, "too many windows");
    Plan pl;
    pl.w.resize(k);
    for (size_t i = 0; i < k; ++i) {
        if (w[i].len == 0 || w[i].start < 4 || (w[i].start & 1))
            return fail(c, GB_EINVAL, "window " + std::to_string(i) + ": start must be even and >= 4, len > 0");
        const uint64_t last = w[i].start + 2 * (w[i].len - 1);
        if (last < w[i].start || last > GB_MAX_N) return fail(c, GB_EINVAL, "window beyond 2^63");
        if (last > c->prm.max_hi) return fail(c, GB_ERANGE, "window above the context's max_hi");
        pl.w[i].first_n = w[i].start;
        pl.w[i].count = w[i].len;
        pl.w[i].slot = (uint32_t)i;
    }
    gb_status stt = plan_windows(c, pl);
    if (stt != GB_OK) return stt;
    stt = ensure_workspace(c, ws, pl, k, 1);
    if (stt != GB_OK) return stt;
    GB_HIP(c, hipMemcpyAsync(ws.win.p, pl.w.data(), k * sizeof(GbWindow), hipMemcpyHostToDevice, st));
    GB_HIP(c, hipEventRecord(ws.ev0, st));
    GraphKey key;
    key.generation = g_buffer_generation.load();
    key.kind = 2;
    key.nwin = k;
    key.ntiles = pl.ntiles;
    key.hist_rows = 1;
    key.pmin = pmin;
    key.pmin_bits = pmin ? 16 : 0;
    key.stream = st;
    Job j;
    j.pl = &pl;
    j.nslots = k;
    j.hist_rows = 1;
    j.pmin_dev = pmin;
    j.pmin_bits = pmin ? 16 : 0;
    j.persistent = true;
    stt = run_job(c, ws, j, key, true, st);
    if (stt != GB_OK) return stt;
    GB_HIP(c, hipEventRecord(ws.ev1, st));
    GB_HIP(c, hipStreamSynchronize(st));
    gb_status fin = GB_OK;
    for (size_t i = 0; i < k; ++i) {
        gb_summary s{};
        merge_slot(s, ws.h_slots.p[i]);
        if (sums) sums[i] = s;
        if (s.n_failed) fin = GB_EUNRESOLVED;
        if (s.count != w[i].len) return fail(c, GB_EDEVICE, "internal: window count mismatch");
    }
    if (hist)
        for (uint32_t i = 0; i < GB_HIST_BINS; ++i) hist[i] = ws.h_hist.p[i];
    stt = finish_list(c);
    if (stt != GB_OK) return stt;
    if (fin != GB_OK) return fail(c, fin, "n without a partition within the budget");
    return GB_OK;
}

gb_status gb_verify_many(gb_ctx *c, const uint64_t *n, uint64_t *p, size_t k, int on_device, void *stream)
{
    if (!c || (k && (!n || !p))) return fail(c, GB_EINVAL, "null argument");
    if (hipSetDevice(c->prm.device) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    if (k == 0) return GB_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace &ws = c->ws;
    if (k > c->prm.max_unresolved) return fail(c, GB_ENOMEM, "more queries than max_unresolved");
    const unsigned long long *dn = reinterpret_cast<const unsigned long long *>(n);
    unsigned long long *dp = reinterpret_cast<unsigned long long *>(p);
    std::vector<uint64_t> hn;
    if (!on_device) {
        for (size_t i = 0; i < k; ++i)
            if (n[i] < 4 || (n[i] & 1) || n[i] > GB_MAX_N)
                return fail(c, GB_EINVAL, "n must be even with 4 <= n <= 2^63");
        GB_HIP(c, ws.q.ensure(2 * k));
        GB_HIP(c, hipMemcpyAsync(ws.q.p, n, k * 8, hipMemcpyHostToDevice, st));
        dn = ws.q.p;
        dp = ws.q.p + k;
    } else {
        hn.resize(k);
        GB_HIP(c, hipMemcpyAsync(hn.data(), n, k * 8, hipMemcpyDeviceToHost, st));
        GB_HIP(c, hipStreamSynchronize(st));
        for (size_t i = 0; i < k; ++i)
            if (hn[i] < 4 || (hn[i] & 1) || hn[i] > GB_MAX_N)
                return fail(c, GB_EINVAL, "n must be even with 4 <= n <= 2^63");
    }
    gb_status stt = enqueue_queries(c, ws, k, dn, dp, st);
    if (stt != GB_OK) return stt;
    std::vector<uint64_t> hp(k);
    GB_HIP(c, hipMemcpyAsync(hp.data(), dp, k * 8, hipMemcpyDeviceToHost, st));
    GB_HIP(c, hipStreamSynchronize(st));
    if (!on_device) std::memcpy(p, hp.data(), k * 8);
    for (size_t i = 0; i < k; ++i)
        if (hp[i] == 0) return fail(c, GB_EUNRESOLVED, "n without a partition within the budget");
    return GB_OK;
}

gb_status gb_verify_one(gb_ctx *c, uint64_t n, uint64_t *p, void *stream)
{
    if (!c || !p) return fail(c, GB_EINVAL, "null argument");
    if (n < 4 || (n & 1) || n > GB_MAX_N) return fail(c, GB_EINVAL, "n must be even with 4 <= n <= 2^63");
    return gb_verify_many(c, &n, p, 1, 0, stream);
}

gb_status gb_sieve_window(gb_ctx *c, uint64_t w0, uint64_t nbits, uint32_t *bits, void *stream)
{
    if (!c || !bits) return fail(c, GB_EINVAL, "null argument");
    if (!(w0 & 1) || nbits == 0 || (nbits & 63))
        return fail(c, GB_EINVAL, "w0 must be odd, nbits a positive multiple of 64");
    if (hipSetDevice(c->prm.device) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint64_t top = w0 + 2 * nbits;
    if (top < w0 || top > c->prm.max_hi) return fail(c, GB_ERANGE, "window above the context's max_hi");
    gb_status stt = enqueue_sieve(c, c->ws, w0, nbits, bits, st);
    if (stt != GB_OK) return stt;
    GB_HIP(c, hipStreamSynchronize(st));
    return GB_OK;
}

gb_status gb_sieve_planes(gb_ctx *c, uint64_t k0, uint64_t nk, uint32_t *planes, void *stream)
{
    if (!c || !planes) return fail(c, GB_EINVAL, "null argument");
    if ((k0 & 63) || nk == 0 || (nk & 63)) return fail(c, GB_EINVAL, "k0 and nk must be multiples of 64, nk > 0");
    if (hipSetDevice(c->prm.device) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    if (k0 > c->prm.max_hi / 6 || nk > c->prm.max_hi / 6 - k0)
        return fail(c, GB_ERANGE, "planes above the context's max_hi");
    hipStream_t st = static_cast<hipStream_t>(stream);
    gb_status stt = enqueue_sieve6(c, c->ws, k0, nk, planes, st);
    if (stt != GB_OK) return stt;
    GB_HIP(c, hipStreamSynchronize(st));
    return GB_OK;
}

gb_status gb_exhaustive_list(gb_ctx *c, uint64_t *n, uint64_t *p, size_t cap, size_t *count)
{
    if (!c || !count) return GB_EINVAL;
    if (!c->last_list_valid) {
        *count = 0;
        return GB_OK;
    }
    *count = c->last_list.size();
    const size_t m = std::min(cap, c->last_list.size());
    for (size_t i = 0; i < m; ++i) {
        if (n) n[i] = c->last_list[i].n;
        if (p) p[i] = c->last_list[i].p;
    }
    return GB_OK;
}

}  // extern "C"
