// gb_tune.hip -- the autotuner behind gb_autotune().
//
// The paper fixes SEG_SIZE and P_SMALL and notes that data-centre GPUs need
// them tuned (Results, "Multi-GPU Scaling and Efficiency"; Discussion,
// "Limitations").  Here the shape of the tile kernel -- tile size T,
// workgroup size, fast-path bound P_max, wheel size -- is chosen by timing
// the batched form on a sample of windows, and the plain form's segment size
// S by timing it on a sample range.  Every configuration must give the same
// per-window results (p_min does not depend on any of these choices); a
// mismatch is reported as an error, never silently tuned away.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gb_runtime.h"

using namespace gbrt;

namespace {

struct Trial {
    gb_params prm;
    double ms = -1;       // device time of the timed run, or -1 if infeasible
    bool ok = false;
};

struct Outcome {
    std::vector<gb_summary> sums;
    std::vector<uint64_t> hist;
};

bool same_results(const Outcome &a, const Outcome &b, bool compare_exhaustive)
{
    if (a.sums.size() != b.sums.size() || a.hist != b.hist) return false;
    for (size_t i = 0; i < a.sums.size(); ++i) {
        const gb_summary &x = a.sums[i], &y = b.sums[i];
        if (x.count != y.count || x.max_p != y.max_p || x.argmax_n != y.argmax_n || x.checksum != y.checksum ||
            x.n_failed != y.n_failed || x.first_failed_n != y.first_failed_n)
            return false;
        if (compare_exhaustive && x.n_exhaustive != y.n_exhaustive) return false;
    }
    return true;
}

// Apply tile/workgroup/pmax/wheel/segment parameters to the live context.
gb_status reconfigure(gb_ctx *c, const gb_params &p)
{
    gb_params q = c->prm;
    q.tile_log2 = p.tile_log2;
    q.wg_threads = p.wg_threads;
    q.pmax = p.pmax;
    q.wheel_max = p.wheel_max;
    q.search_mode = p.search_mode;
    q.seg_log2 = std::max(p.seg_log2, p.tile_log2);
    gb_status st = apply_params(c, &q);
    if (st != GB_OK) return st;
    return setup_geometry(c);
}

// Run the sample twice (graph capture, then a timed replay); device time of
// the second run.
gb_status time_windows(gb_ctx *c, const gb_window *w, size_t k, Outcome &out, double &ms)
{
    out.sums.assign(k, gb_summary{});
    out.hist.assign(GB_HIST_BINS, 0);
    for (int rep = 0; rep < 2; ++rep) {
        gb_status st = gb_verify_windows(c, w, k, nullptr, out.sums.data(), out.hist.data(), nullptr);
        if (st != GB_OK) return st;
    }
    float f = 0;
    GB_HIP(c, hipEventElapsedTime(&f, c->ws.ev0, c->ws.ev1));
    ms = f;
    return GB_OK;
}

std::string params_json(const gb_params &p)
{
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "{\"tile_log2\": %u, \"wg_threads\": %u, \"search_mode\": %u, \"pmax\": %u, "
                  "\"wheel_max\": %u, \"seg_log2\": %u}",
                  p.tile_log2, p.wg_threads, p.search_mode, p.pmax, p.wheel_max, p.seg_log2);
    return buf;
}

}  // namespace

extern "C" gb_status gb_autotune(gb_ctx *c, const gb_window *sample, size_t k, const char *cache_path,
                                 gb_params *best)
{
    if (!c || !sample || k == 0) return fail(c, GB_EINVAL, "autotune needs a context and a non-empty sample");
    if (hipSetDevice(c->prm.device) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    const gb_params orig = c->prm;
    std::vector<Trial> log;
    Outcome ref;
    bool have_ref = false;
    gb_params cur = orig;
    double cur_ms = 1e300;

    auto try_point = [&](const gb_params &p, bool compare_exhaustive) -> gb_status {
        Trial t;
        t.prm = p;
        gb_status st = reconfigure(c, p);
        if (st == GB_EINVAL) {  // does not fit in LDS: skip
            log.push_back(t);
            return GB_OK;
        }
        if (st != GB_OK) return st;
        Outcome o;
        double ms = 0;
        st = time_windows(c, sample, k, o, ms);
        if (st != GB_OK && st != GB_EUNRESOLVED) return st;
        if (!have_ref) {
            ref = o;
            have_ref = true;
        } else if (!same_results(ref, o, compare_exhaustive)) {
            return fail(c, GB_EDEVICE, "autotune: configuration " + params_json(p) +
                                           " gives results different from " + params_json(log.front().prm));
        }
        t.ms = ms;
        t.ok = true;
        log.push_back(t);
        if (ms < cur_ms) {
            cur_ms = ms;
            cur = p;
        }
        return GB_OK;
    };

    // 1. tile and workgroup shape at the given P_max and wheel
    for (uint32_t tl : {16u, 17u, 18u, 19u, 20u})
        for (uint32_t nt : {256u, 512u, 1024u}) {
            gb_params p = orig;
            p.tile_log2 = tl;
            p.wg_threads = nt;
            gb_status st = try_point(p, true);
            if (st != GB_OK) {
                (void)reconfigure(c, orig);
                return st;
            }
        }
    // 2. fast-path bound (n_exhaustive legitimately depends on it)
    {
        const gb_params base = cur;
        for (uint32_t lg = 10; lg <= 16; ++lg) {
            gb_params p = base;
            p.pmax = std::min<uint32_t>(1u << lg, 65535u);
            if (p.pmax == base.pmax) continue;
            gb_status st = try_point(p, false);
            if (st != GB_OK) {
                (void)reconfigure(c, orig);
                return st;
            }
        }
    }
    // 3. wheel size
    {
        const gb_params base = cur;
        for (uint32_t wm : {13u, 17u, 19u}) {
            if (wm == base.wheel_max) continue;
            gb_params p = base;
            p.wheel_max = wm;
            gb_status st = try_point(p, false);
            if (st != GB_OK) {
                (void)reconfigure(c, orig);
                return st;
            }
        }
    }
    // 4. segment size of the plain form (one launch per segment), S = 2^20 ..
    // 2^26 even n, on 2^32 even n from the sample's first start: large
    // enough that the largest segments still make many launches
    uint64_t total = 0;
    for (size_t i = 0; i < k; ++i) total += sample[i].len;
    const uint64_t lo = sample[0].start;
    uint64_t span = 1ull << 32;
    uint64_t hi = lo + 2 * (span - 1);
    if (hi > c->prm.max_hi) hi = c->prm.max_hi;
    gb_params best_seg = cur;
    double best_seg_ms = 1e300;
    gb_summary seg_ref{};
    bool have_seg_ref = false;
    for (uint32_t sl = 20; sl <= 26; ++sl) {
        gb_params p = cur;
        p.seg_log2 = std::max(sl, p.tile_log2);
        gb_status st = reconfigure(c, p);
        if (st != GB_OK) {
            (void)reconfigure(c, orig);
            return st;
        }
        gb_result r{};
        double ms = 0;
        for (int rep = 0; rep < 2; ++rep) {
            std::memset(&r, 0, sizeof r);
            st = gb_verify_range(c, lo, hi, &r, nullptr);
            if (st != GB_OK && st != GB_EUNRESOLVED) {
                (void)reconfigure(c, orig);
                return st;
            }
            ms = r.device_ms;
        }
        if (!have_seg_ref) {
            seg_ref.count = r.count;
            seg_ref.checksum = r.checksum;
            seg_ref.max_p = r.max_p;
            seg_ref.argmax_n = r.argmax_n;
            have_seg_ref = true;
        } else if (r.count != seg_ref.count || r.checksum != seg_ref.checksum || r.max_p != seg_ref.max_p ||
                   r.argmax_n != seg_ref.argmax_n) {
            (void)reconfigure(c, orig);
            return fail(c, GB_EDEVICE, "autotune: segment size changes the results");
        }
        Trial t;
        t.prm = p;
        t.ms = ms;
        t.ok = true;
        log.push_back(t);
        if (ms < best_seg_ms) {
            best_seg_ms = ms;
            best_seg = p;
        }
    }
    gb_status st = reconfigure(c, best_seg);
    if (st != GB_OK) return st;
    if (best) *best = c->prm;
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "w");
        if (!f) return fail(c, GB_EINVAL, std::string("cannot write ") + cache_path);
        hipDeviceProp_t prop;
        (void)hipGetDeviceProperties(&prop, c->prm.device);
        std::fprintf(f, "{\"device\": \"%s\", \"cus\": %d, \"sample_windows\": %zu, \"sample_n\": %llu,\n",
                     prop.gcnArchName, prop.multiProcessorCount, k, (unsigned long long)total);
        std::fprintf(f, " \"tile_log2\": %u, \"wg_threads\": %u, \"search_mode\": %u, \"pmax\": %u, "
                        "\"wheel_max\": %u, \"seg_log2\": %u,\n",
                     c->prm.tile_log2, c->prm.wg_threads, c->prm.search_mode, c->prm.pmax, c->prm.wheel_max,
                     c->prm.seg_log2);
        std::fprintf(f, " \"trials\": [");
        for (size_t i = 0; i < log.size(); ++i)
            std::fprintf(f, "%s\n  {\"params\": %s, \"ms\": %.4f}", i ? "," : "", params_json(log[i].prm).c_str(),
                         log[i].ms);
        std::fprintf(f, "]}\n");
        std::fclose(f);
    }
    return GB_OK;
}
