// gb_runtime.h -- host-side runtime state shared by the C-ABI entry points
// (gb_host.hip) and the serving loop (gb_server.hip).  Not a public header.
#pragma once
#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/goldbach.h"
#include "gb_internal.h"

namespace gbrt {

constexpr uint64_t kDefaultMaxHi = 1ull << 50;
constexpr uint32_t kCounters = 4;  // [0] exhaustive-list length, [1] work queue, [2] argmax records

// Every move of a device or pinned scratch buffer bumps this, so a cached
// HIP graph that captured the old addresses is never replayed.
extern std::atomic<uint64_t> g_buffer_generation;

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n)
    {
        if (n <= cap && p) return hipSuccess;
        g_buffer_generation.fetch_add(1);
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        const size_t want = n ? n : 1;
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&p), want * sizeof(T));
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

template <class T>
struct PinBuf {
    T *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n)
    {
        if (n <= cap && p) return hipSuccess;
        g_buffer_generation.fetch_add(1);
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        const size_t want = n ? n : 1;
        hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&p), want * sizeof(T));
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release()
    {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
};

struct GraphKey {
    uint64_t generation = 0;
    int kind = 0;  // 1: range, 2: windows
    uint64_t nwin = 0, ntiles = 0, hist_rows = 0;
    void *pmin = nullptr;
    int pmin_bits = 0;
    hipStream_t stream = nullptr;
    bool operator==(const GraphKey &o) const
    {
        return generation == o.generation && kind == o.kind && nwin == o.nwin && ntiles == o.ntiles &&
               hist_rows == o.hist_rows && pmin == o.pmin && pmin_bits == o.pmin_bits && stream == o.stream;
    }
};

// Per-stream scratch: everything one in-flight computation writes.
struct Workspace {
    DevBuf<GbWindow> win;
    DevBuf<GbSlot> slots;
    DevBuf<unsigned long long> hist;
    DevBuf<GbTileRec> recs;
    DevBuf<uint32_t> wgh;                // per workgroup of a persistent launch: its stored histogram row
    DevBuf<GbExh> list;
    DevBuf<unsigned long long> counters;
    DevBuf<unsigned char> pmin;          // per-n output staging
    DevBuf<unsigned long long> q;        // single-n queries: n then p
    DevBuf<uint32_t> pc_bits;            // partition counts: odd-number bitset
    DevBuf<unsigned long long> pc_counts;  // partition counts when the caller passes none
    DevBuf<unsigned long long> pc_red;   // partition counts: sum, min key, max key
    PinBuf<unsigned long long> h_pc_red;
    DevBuf<uint32_t> big_n;              // beyond 64 bits: the n, K limbs each,
    DevBuf<uint32_t> big_state;          // per n: the table index its search resumes
                                         // from, that of its candidate p, the
                                         // resume index after the pass, its
                                         // confirmation flag, its answer (five
                                         // arrays of k), then the list lengths
    DevBuf<uint32_t> big_list;           // the n searched and confirmed in a pass
                                         // and in the next (two pairs of lists)
    PinBuf<uint32_t> h_big;              // host copies of the answers and lengths
    DevBuf<unsigned long long> big_p;    // the one-kernel form's answers
    PinBuf<GbSlot> h_slots;
    PinBuf<unsigned long long> h_hist;
    PinBuf<unsigned long long> h_counters;
    PinBuf<unsigned long long> h_q;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, evt0 = nullptr, evt1 = nullptr, done = nullptr;
    hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};  // init, tiles, rest
    GraphKey gkey;
    hipError_t init(uint64_t list_cap);
    void release();
    void drop_graphs();
};

// A list of windows split into tiles.
struct Plan {
    std::vector<GbWindow> w;
    uint64_t ntiles = 0;
    uint64_t total_n = 0;
};

// One computation over uploaded windows.
struct Job {
    const Plan *pl = nullptr;
    size_t nslots = 0, hist_rows = 1;
    void *pmin_dev = nullptr;
    int pmin_bits = 0;
    bool persistent = false;
};

}  // namespace gbrt

struct gb_ctx {
    gb_params prm{};
    int num_cu = 0;
    std::vector<uint32_t> h_primes;  // odd primes 3, 5, 7, ...
    uint32_t *d_primes = nullptr;
    unsigned long long *d_magic = nullptr;
    uint4 *d_prime6 = nullptr;       // sieve entries of the odd primes below 2^27
    uint32_t n_prime6 = 0;
    uint64_t ntab = 0;
    uint64_t table_limit = 0;        // every odd prime <= table_limit is in the table
    uint32_t threads = 0;
    // minimal-p search split by residue mod 6 (gb_class.hip): tiles of
    // tile_n = 192 sb_per_tile even n, windows aligned to 384
    uint32_t tile_n = 0, sb_per_tile = 0, hk = 0;
    uint32_t np_cls = 0;             // odd primes on the class probe lists
    uint32_t *d_cls = nullptr;       // class headers, sieve tables, probe records
    uint32_t cls_words = 0;
    uint32_t cls_recs = 0;           // probe records of the three class lists (the real groups)
    uint32_t *d_rec_bin = nullptr;   // histogram bin of each probe record, class order
    uint32_t wgh_stride = 0;         // words per workgroup row of Workspace::wgh
    uint32_t *d_wheel6 = nullptr;    // two plane patterns
    uint32_t wheel6_len = 0, wheel6_stride = 0;
    uint32_t k6_first = 0, k6_wave_end = 0, k6_single = 0;
    // the plain form's class tiles (one launch per segment, plain_lanes
    // segments in flight): small enough that those segments fill the device
    uint32_t sbp = 0, tile_np = 0, k6p_wave_end = 0, k6p_single = 0;
    size_t lds6p = 0;
    size_t lds6 = 0;
    int occ6 = 1;
    // the odd-number sieve dump (gb_kernels.hip): tiles of tile_n_odd bits
    // behind a halo of halo_bits
    uint32_t tile_n_odd = 0;
    uint32_t np_search = 0, k_first = 0, halo_bits = 0;
    uint32_t *d_wheel = nullptr;
    uint32_t wheel_len = 0;
    uint32_t k_wg_end = 0, k_wave_end = 0;
    size_t lds = 0;
    // plain form: segment launches go round-robin to the caller's stream and
    // these (created on first use), forked after the init kernel and joined
    // before the exhaustive phase.  It runs up to kPlainLanes segments side by side, one per
    // stream: no more than the process has hardware queues (plain_hwq, from
    // GPU_MAX_HW_QUEUES, 4 when unset; streams beyond that share queues and
    // run in turn), and no more than keep the tiles in flight within 1/8 of
    // the CU count (plain_lanes, set with the plain tile size).
    static constexpr int kPlainLanes = 8;
    int plain_hwq = 4;
    int plain_lanes = 4;
    hipStream_t plain_st[kPlainLanes - 1] = {};
    hipEvent_t plain_fork = nullptr, plain_join[kPlainLanes - 1] = {};
    gbrt::Workspace ws;              // scratch of the synchronous calls
    std::string err;
    std::vector<GbExh> last_list;
    bool last_list_valid = false;
};

namespace gbrt {

gb_status fail(gb_ctx *c, gb_status st, const std::string &msg);
uint64_t isqrt64(uint64_t x);
gb_status apply_params(gb_ctx *c, const gb_params *in);
gb_status setup_geometry(gb_ctx *c);
gb_status build_tables(gb_ctx *c);
void free_tables(gb_ctx *c);
// How a plan splits windows: the minimal-p search (tiles of tile_n, first
// n moved down to a multiple of 384), the bulk form (tiles of
// tile_n_odd, multiples of 128) or the odd-number sieve dump (no move).
enum PlanKind { kPlanClass, kPlanClassPlain, kPlanSieve };
gb_status plan_windows(gb_ctx *c, Plan &pl, PlanKind kind = kPlanClass);
gb_status ensure_workspace(gb_ctx *c, Workspace &ws, const Plan &pl, size_t nslots, size_t hist_rows);
// init + tiles + exhaustive phase + argmax + summary copies, on `st`,
// with ws.evt0/evt1 around the tile launches; with use_graph each phase is a
// cached executable graph keyed by `key`.
gb_status run_job(gb_ctx *c, Workspace &ws, const Job &j, const GraphKey &key, bool use_graph,
                  hipStream_t st);
// single-n queries already in ws.q (device, k entries): results to ws.q + k
gb_status enqueue_queries(gb_ctx *c, Workspace &ws, uint64_t k, const unsigned long long *dn,
                          unsigned long long *dp, hipStream_t st);
// the tile sieve alone: bits (device, nbits/32 words) of the odd numbers
// w0, w0 + 2, ... (w0 odd, nbits a multiple of 64), enqueued on st
gb_status enqueue_sieve(gb_ctx *c, Workspace &ws, uint64_t w0, uint64_t nbits, uint32_t *bits, hipStream_t st);
void merge_slot(gb_summary &acc, const GbSlot &s);
// Record the device address of the no-allocation form's scratch array on
// `device` (current), once per device; its result on later calls.
hipError_t noalloc_setup(int device);

}  // namespace gbrt

#define GB_HIP(c, expr)                                                                             \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return ::gbrt::fail((c), GB_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)
