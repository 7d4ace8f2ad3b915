// gb_big.hip -- minimal Goldbach prime of even n beyond 64 bits (paper
// section "Arbitrary Precision Checker": small primes p in ascending order,
// q = n - p tested with Miller-Rabin), up to n < 2^1024.
//
// n is held as K limbs of 28 bits (gb_bignum28.h): K = 4, 6, ..., 16 up to
// 446 bits, then K = 20, 24, 28, 32, 36 and 37 (up to 1034 bits).  The
// search runs in passes of one launch each, planned on the device (a
// small kernel after each pass writes the next pass's lists).  A launch is
// a list of lane tasks, 64 to a wavefront: first the search groups, then
// the confirmations.
//
// - Search: the odd primes p of the resident table are filtered, 64 at a
//   time, by the 24 odd prime bases r = 3 .. 97.  A q = n - p that r divides
//   fails the strong test to base r (a^d and its squarings mod q are then
//   multiples of r, never 1 or q - 1), so dropping p = n (mod r) leaves the
//   answer unchanged; about a quarter of the p survive.  A group of G lanes
//   (G = 32 or 64) takes G consecutive survivors of one n and tests their q
//   to base 2; the group's lowest passing lane gives the candidate, and an
//   atomic minimum over the groups of one n keeps the smallest.
// - Confirmation: 24 lanes per candidate, lane j testing its q to the j-th
//   odd base.  A candidate that fails one (a strong pseudoprime to base 2)
//   sends its n back to the search, which resumes after it.
//
// The answer is the first p whose q passes all 25 bases; every smaller p
// failed one, so its q is composite.  All lanes run the same windowed strong
// test (base 2 or an odd base), so search groups and confirmations share
// wavefronts.
#include <algorithm>
#include <cstring>

#include "gb_bignum28.h"
#include "gb_runtime.h"

namespace {

using namespace gbrt;

__constant__ uint32_t kBigBases[25] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41,
                                       43, 47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97};

constexpr uint32_t kOddBases[24] = {3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41,
                                     43, 47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97};

// n mod r for a small r (r < 2^12), most significant limb first
template <int K> __device__ __forceinline__ uint32_t mod_small(const gbbig28::Num<K> &n, uint32_t r)
{
    const uint32_t t = (1u << gbbig28::kBits) % r;
    uint32_t acc = 0;
#pragma unroll
    for (int i = K - 1; i >= 0; --i) acc = (acc * t + n.w[i] % r) % r;
    return acc;
}

// q = n - p for n (K 28-bit limbs) above p (p < 2^32: two limbs)
template <int K> __device__ __forceinline__ void big_sub_p(gbbig28::Num<K> &q, const uint32_t *n, uint32_t p)
{
    uint32_t br = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const uint32_t pi = i == 0 ? (p & gbbig28::kMask) : i == 1 ? (p >> gbbig28::kBits) : 0u;
        const uint32_t t = n[i] - pi - br;
        q.w[i] = t & gbbig28::kMask;
        br = t >> 31;
    }
}

// Lanes [lane0, lane0 + G) of the wavefront collect, into cand, the table
// indices of the surviving p of n_all[idx] ranked [G way, G way + G) from
// resume_in[idx] on; returns how many there are (fewer at the table's end).
// Way nways - 1 writes the table index after its group (nprimes at the
// table's end) to resume_out[idx].  resume_in is only read during the pass:
// the groups of one n run in any order, so a write into the array the others
// read would move their groups.
template <int K>
__device__ __forceinline__ uint32_t big_collect(uint32_t *cand, uint32_t G, uint32_t way, uint32_t nways,
                                                uint32_t idx, const uint32_t *n_all, const uint32_t *primes,
                                                uint32_t nprimes, const uint32_t *resume_in, uint32_t *resume_out)
{
    const uint32_t lane = threadIdx.x & 63u;
    gbbig28::Num<K> n;
#pragma unroll
    for (int i = 0; i < K; ++i) n.w[i] = n_all[(uint64_t)idx * K + i];
    // n mod r for the 24 odd bases (the same in every lane)
    uint32_t nres[24];
#pragma unroll
    for (int j = 0; j < 24; ++j) nres[j] = mod_small(n, kOddBases[j]);
    const uint32_t lo = G * way, hi = lo + G;
    uint32_t got = 0, next = resume_in[idx];
    while (got < hi && next < nprimes) {
        const uint32_t c = next + lane;
        const bool valid = c < nprimes;
        const uint32_t p = valid ? primes[c] : 0u;
        bool hit = false;
#pragma unroll
        for (int j = 0; j < 24; ++j) hit = hit || (p % kOddBases[j] == nres[j]);
        const bool keep = valid && !hit;
        const unsigned long long m = __builtin_amdgcn_ballot_w64(keep);
        const uint32_t g = got + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (keep && g >= lo && g < hi) cand[g - lo] = c;
        const uint32_t tot = (uint32_t)__popcll(m);
        if (got + tot > hi) {
            // the first surviving p past the group
            next += (uint32_t)__builtin_ctzll(__builtin_amdgcn_ballot_w64(keep && g == hi));
            got = hi;
        } else {
            next = next + 64u < nprimes ? next + 64u : nprimes;
            got += tot;
        }
    }
    if (way == nways - 1u && lane == 0u) resume_out[idx] = next;
    return got > lo ? got - lo : 0u;
}

// Pass shape.  A pass takes whole rounds of one wavefront per SIMD: the
// confirmations' rounds plus kExtraRounds (one round in the first pass),
// and the search gets as many groups per open n (ways, at most kMaxWays) as
// fill the rest, so that the n with large p_min do not run alone.  Groups
// hold kGroup survivors; in a first pass whose n do not fill the round with
// one group of kGroup each, they hold kSmallGroup (more, smaller groups per
// n: the first candidate lies in an earlier one); the host picks the
// kernel built for the pass's group size, and every wavefront derives the
// ways from the list lengths in device memory.
constexpr uint32_t kGroup = 32, kSmallGroup = 16, kExtraRounds = 1, kMaxWays = 16;

// The group size of a pass: kSmallGroup only in a first pass whose n do not
// fill one round with a group of kGroup each.
inline uint32_t big_group(bool first, uint64_t nsl, uint32_t simds)
{
    return first && nsl * kGroup < 64ull * simds ? kSmallGroup : kGroup;
}

// Groups per open n for a pass with groups of G
__host__ __device__ inline uint32_t big_ways(bool first, uint32_t G, uint32_t nsl, uint32_t ncl, uint32_t simds)
{
    const uint64_t cw = ((uint64_t)ncl * 24u + 63u) / 64u;
    const uint64_t rounds = first ? 1u : (cw + simds - 1u) / simds + kExtraRounds;
    const uint64_t room = rounds * simds > cw ? rounds * simds - cw : 0u;
    uint64_t ways = nsl ? room * 64u / ((uint64_t)nsl * G) : 1u;
    return (uint32_t)(ways < 1u ? 1u : ways > kMaxWays ? kMaxWays : ways);
}

// One pass.  The lists and their lengths are in device memory (written by
// k_big_plan after the pass before), so passes follow each other on the
// stream without the host.  Lane task t (64 per wavefront,
// blockIdx.x * 256 + threadIdx.x): t < S0 = nsl nways G is lane t mod G of
// search group t / G, which is way (t / G) mod nways of the
// ((t / G) / nways)-th n of the search list (every n in the first pass;
// their found entries are all ones before the pass); the next ncl * 24
// tasks confirm the candidates of the n of the confirm list, found in the
// pass before, one odd base each.  The grid covers the largest pass; the
// wavefronts past the tasks return at once.  Block 0 also clears the
// lengths of the next pass's lists (cnt_next).
template <int K, uint32_t G>
__global__ __launch_bounds__(256) void k_big_pass(const uint32_t *n_all, const uint32_t *lists, const uint32_t *cnt,
                                                  uint32_t *cnt_next, uint32_t first, uint32_t k, uint32_t simds,
                                                  const uint32_t *primes,
                                                  uint32_t nprimes, const uint32_t *resume_in, uint32_t *resume_out,
                                                  uint32_t *found, uint32_t *bad)
{
    __shared__ uint32_t cand_all[4][64];
    __shared__ uint32_t grp_all[4][4][2];           // per wavefront and group: n index, survivors
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the next pass's list lengths start from zero: the plan kernel of the
    // pass before, their last reader, has finished, and k_big_plan after
    // this pass counts into them
    if (blockIdx.x == 0u && threadIdx.x < 2u) cnt_next[threadIdx.x] = 0u;
    const uint32_t nsl = first ? k : cnt[0], ncl = first ? 0u : cnt[1];
    const uint32_t nways = big_ways(first != 0u, G, nsl, ncl, simds);
    const uint32_t *slist = first ? nullptr : lists, *clist = lists + k;
    const uint64_t t0 = ((uint64_t)blockIdx.x * 4u + wv) * 64u;
    const uint64_t S0 = (uint64_t)nsl * nways * G;
    const uint64_t total = S0 + (uint64_t)ncl * 24u;
    if (t0 >= total) return;                         // whole wave
    uint32_t *cand = cand_all[wv];
    // the search groups among this wave's lanes (G divides 64, so a group
    // never straddles two wavefronts)
    constexpr uint32_t ngw = 64u / G;
    for (uint32_t gi = 0; gi < ngw && t0 + (uint64_t)gi * G < S0; ++gi) {
        const uint32_t grp = (uint32_t)((t0 + (uint64_t)gi * G) / G);
        const uint32_t li = grp / nways, way = grp - li * nways;
        const uint32_t idx = slist ? slist[li] : li;
        const uint32_t cnt_g =
            big_collect<K>(cand + gi * G, G, way, nways, idx, n_all, primes, nprimes, resume_in, resume_out);
        if (lane == 0u) {
            grp_all[wv][gi][0] = idx;
            grp_all[wv][gi][1] = cnt_g;
        }
    }
    __builtin_amdgcn_wave_barrier();
    const uint64_t t = t0 + lane;
    const bool srch = t < S0;
    bool act = false;
    uint32_t idx = 0u, c = 0u, base = 2u;
    if (srch) {
        const uint32_t gi = lane / G;
        idx = grp_all[wv][gi][0];
        act = lane - gi * G < grp_all[wv][gi][1];
        c = act ? cand[lane] : 0u;
    } else if (t < total) {
        const uint64_t kk = t - S0;
        const uint32_t ci = (uint32_t)(kk / 24u), j = (uint32_t)(kk - (uint64_t)ci * 24u);
        idx = clist[ci];
        c = found[idx];
        act = c < nprimes;                           // else nothing to confirm
        base = kBigBases[j + 1u];
    }
    bool pass = false;
    if (act) {
        gbbig28::Num<K> q;
        big_sub_p(q, n_all + (uint64_t)idx * K, primes[c]);
        pass = gbbig28::strong_prp<K>(q, base);
    }
    const unsigned long long m = __builtin_amdgcn_ballot_w64(srch && pass);
    constexpr unsigned long long gmask = G == 64u ? ~0ull : (1ull << G) - 1ull;
#pragma unroll
    for (uint32_t gi = 0; gi < ngw; ++gi) {
        const unsigned long long gm = (m >> (gi * G)) & gmask;
        if (gm != 0ull && lane == 0u)
            __hip_atomic_fetch_min(&found[grp_all[wv][gi][0]],
                                   __builtin_amdgcn_readlane(c, gi * G + (uint32_t)__builtin_ctzll(gm)),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!srch && act && !pass) __hip_atomic_fetch_or(&bad[idx], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Appends idx to list (length *len) for the lanes where put holds: one
// atomic per wavefront, each lane at its rank among them.
__device__ __forceinline__ void big_append(bool put, uint32_t idx, uint32_t *list, uint32_t *len)
{
    const unsigned long long m = __builtin_amdgcn_ballot_w64(put);
    if (m == 0ull) return;
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    const uint32_t lead = (uint32_t)__builtin_ctzll(m);
    uint32_t base = 0u;
    if (put && rank == 0u) base = atomicAdd(len, (uint32_t)__popcll(m));
    base = __builtin_amdgcn_readlane(base, lead);
    if (put) list[base + rank] = idx;
}

// After a pass: the n whose candidate passed every base are answered
// (ans = its table index); a candidate that failed one sends its n back to
// the search after it; the searched n continue after their groups, to the
// confirm list when a group found a candidate, else to the search list
// (unless the table is spent: the n stays unanswered).  Writes the next
// pass's lists (lists_next, cnt_next, zero before) and resets found or bad
// for the entries it lists.
__global__ __launch_bounds__(256) void k_big_plan(const uint32_t *lists, const uint32_t *cnt, uint32_t first,
                                                  uint32_t k, uint32_t *lists_next, uint32_t *cnt_next,
                                                  uint32_t nprimes, uint32_t *resume, const uint32_t *rout,
                                                  uint32_t *found, uint32_t *bad, uint32_t *ans)
{
    const uint32_t nsl = first ? k : cnt[0], ncl = first ? 0u : cnt[1];
    const uint32_t *sl = lists, *cl = lists + k;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t e0 = blockIdx.x * blockDim.x; e0 < nsl + ncl; e0 += stride) {
        const uint32_t e = e0 + threadIdx.x;
        bool to_s = false, to_c = false;
        uint32_t idx = 0u;
        if (e < ncl) {
            idx = cl[e];
            const uint32_t f = found[idx];
            if (!bad[idx]) {
                ans[idx] = f;
            } else {
                resume[idx] = f + 1u;                // a base-2 pseudoprime: resume after it
                to_s = f + 1u < nprimes;
            }
        } else if (e < nsl + ncl) {
            idx = first ? e - ncl : sl[e - ncl];
            const uint32_t r = rout[idx];
            resume[idx] = r;
            to_c = found[idx] < nprimes;
            to_s = !to_c && r < nprimes;
        }
        if (to_s) found[idx] = ~0u;
        if (to_c) bad[idx] = 0u;
        big_append(to_s, idx, lists_next, cnt_next);
        big_append(to_c, idx, lists_next + k, cnt_next + 1);
    }
}

// Initial state: search from the table's start, nothing found or answered;
// list lengths zero (the first pass searches every n without a list).
__global__ void k_big_init(uint32_t k, uint32_t *resume, uint32_t *found, uint32_t *bad, uint32_t *ans, uint32_t *cnt)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) {
        resume[i] = 0u;
        found[i] = ~0u;
        bad[i] = 0u;
        ans[i] = ~0u;
    }
    if (i < 4u) cnt[i] = 0u;
}

// The n of one limb count K (28-bit limbs): h holds them, K limbs each
// (k n); their answers go to ans (table indices, UINT32_MAX for none).
// Passes are enqueued in batches of kBatch (each a k_big_pass and a
// k_big_plan); after a batch the host reads the next pass's list lengths
// and stops when both are zero.  Every pass moves each open n's resume
// point forward, so the passes end; the cap stops a call whose device
// results do not settle.
template <int K>
gb_status big28_passes(gb_ctx *c, const std::vector<uint32_t> &h, size_t k, std::vector<uint32_t> &ans,
                       hipStream_t st)
{
    constexpr int kBatch = 6, kMaxPasses = 1024;
    Workspace &ws = c->ws;
    GB_HIP(c, ws.big_n.ensure(h.size()));
    GB_HIP(c, hipMemcpyAsync(ws.big_n.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, st));
    GB_HIP(c, ws.big_state.ensure(5 * k + 4));
    GB_HIP(c, ws.big_list.ensure(4 * k));
    GB_HIP(c, ws.h_big.ensure(k + 4));
    const uint32_t np = (uint32_t)c->ntab, kk = (uint32_t)k, simds = (uint32_t)c->num_cu * 4u;
    uint32_t *d_resume = ws.big_state.p, *d_found = d_resume + k, *d_rout = d_found + k, *d_bad = d_rout + k,
             *d_ans = d_bad + k, *d_cnt = d_ans + k;   // d_cnt: lengths of list pair 0, then of pair 1
    uint32_t *h_ans = ws.h_big.p, *h_cnt = h_ans + k;
    hipLaunchKernelGGL(k_big_init, dim3((kk + 255u) / 256u), dim3(256), 0, st, kk, d_resume, d_found, d_bad, d_ans,
                       d_cnt);
    GB_HIP(c, hipGetLastError());
    // the largest pass: every n in groups of the larger G, every n confirming,
    // or the rounds the shape can ask for
    const uint64_t gmax = std::max(kGroup, kSmallGroup);
    const uint64_t conf_waves = ((uint64_t)k * 24u + 63u) / 64u;
    const uint64_t waves = std::max<uint64_t>(((uint64_t)k * gmax + 63u) / 64u + conf_waves,
                                              ((conf_waves + simds - 1u) / simds + kExtraRounds + 1u) * simds);
    const uint32_t pass_blocks = (uint32_t)((waves + 3u) / 4u);
    const uint32_t plan_blocks = (uint32_t)std::min<uint64_t>((k + 255u) / 256u, (uint64_t)c->num_cu * 4u);
    for (int pass = 0;;) {
        for (int b = 0; b < kBatch; ++b, ++pass) {
            const uint32_t par = (uint32_t)pass & 1u, first = pass == 0 ? 1u : 0u;
            const uint32_t *lists = ws.big_list.p + (size_t)par * 2u * k, *cnt = d_cnt + 2u * par;
            uint32_t *lists_next = ws.big_list.p + (size_t)(par ^ 1u) * 2u * k, *cnt_next = d_cnt + 2u * (par ^ 1u);
            if (big_group(first != 0u, k, simds) == kSmallGroup)
                hipLaunchKernelGGL((k_big_pass<K, kSmallGroup>), dim3(pass_blocks), dim3(256), 0, st, ws.big_n.p, lists,
                                   cnt, cnt_next, first, kk, simds, c->d_primes, np, d_resume, d_rout, d_found, d_bad);
            else
                hipLaunchKernelGGL((k_big_pass<K, kGroup>), dim3(pass_blocks), dim3(256), 0, st, ws.big_n.p, lists, cnt,
                                   cnt_next, first, kk, simds, c->d_primes, np, d_resume, d_rout, d_found, d_bad);
            GB_HIP(c, hipGetLastError());
            hipLaunchKernelGGL(k_big_plan, dim3(plan_blocks), dim3(256), 0, st, lists, cnt, first, kk, lists_next,
                               cnt_next, np, d_resume, d_rout, d_found, d_bad, d_ans);
            GB_HIP(c, hipGetLastError());
        }
        const uint32_t *cnt_now = d_cnt + 2u * ((uint32_t)pass & 1u);
        GB_HIP(c, hipMemcpyAsync(h_cnt, cnt_now, 8, hipMemcpyDeviceToHost, st));
        GB_HIP(c, hipStreamSynchronize(st));
        if (h_cnt[0] == 0u && h_cnt[1] == 0u) break;
        if (pass >= kMaxPasses) return fail(c, GB_EDEVICE, "big-n search did not settle");
    }
    GB_HIP(c, hipMemcpyAsync(h_ans, d_ans, k * 4, hipMemcpyDeviceToHost, st));
    GB_HIP(c, hipStreamSynchronize(st));
    ans.assign(h_ans, h_ans + k);
    return GB_OK;
}

}  // namespace

using namespace gbrt;

gb_status gb_verify_big(gb_ctx *c, const uint32_t *n, uint32_t nlimbs, size_t k, uint64_t *p, void *stream)
{
    if (!c || (k && (!n || !p))) return fail(c, GB_EINVAL, "null argument");
    if (nlimbs < 3 || nlimbs > 32) return fail(c, GB_EINVAL, "nlimbs must be in 3..32");
    if (k == 0) return GB_OK;
    if (k > (1ull << 24)) return fail(c, GB_EINVAL, "at most 2^24 n per call");
    // every n even and at least 2^64; the bit length of each
    std::vector<uint16_t> bits(k, 0);
    for (size_t i = 0; i < k; ++i) {
        const uint32_t *w = n + i * nlimbs;
        bool big = false;
        for (uint32_t j = 2; j < nlimbs; ++j) big = big || w[j] != 0u;
        if ((w[0] & 1u) || !big) return fail(c, GB_EINVAL, "n must be even and at least 2^64");
        for (uint32_t j = nlimbs; j-- > 0;)
            if (w[j]) {
                bits[i] = (uint16_t)(32u * j + 32u - (uint32_t)__builtin_clz(w[j]));
                break;
            }
    }
    if (hipSetDevice(c->prm.device) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // Forms: the smallest K of the list with 28K - 2 >= bits, one pass
    // sequence per K present.  Consecutive K differ by at most 2 up to 16 and
    // by at most 4 above, so q = n - p >= 2^(28 (K - 2) - 3) (2^(28 (K - 4) - 3)
    // above 16), as the quotient estimate of the 28-bit arithmetic needs
    // (q >= 2^(28 (K - E) + 24) with E = 3, resp. 5).
    static constexpr int kForms[] = {4, 6, 8, 10, 12, 14, 16, 20, 24, 28, 32, 36, 37};
    constexpr int nforms = (int)(sizeof kForms / sizeof kForms[0]);
    std::vector<uint32_t> sel[nforms];
    for (size_t i = 0; i < k; ++i) {
        int f = 0;
        while (28 * kForms[f] - 2 < (int)bits[i]) ++f;   // bits <= 1024 <= 28 * 37 - 2
        sel[f].push_back((uint32_t)i);
    }
    bool unresolved = false;
    for (int f = 0; f < nforms; ++f) {
        if (sel[f].empty()) continue;
        const int K = kForms[f];
        const size_t kk = sel[f].size();
        // K limbs of 28 bits: limb l is bits 28 l .. 28 l + 27
        std::vector<uint32_t> h(kk * (size_t)K, 0u);
        for (size_t a = 0; a < kk; ++a) {
            const uint32_t *w = n + (size_t)sel[f][a] * nlimbs;
            for (int l = 0; l < K; ++l) {
                const uint32_t b0 = 28u * (uint32_t)l, j = b0 >> 5, o = b0 & 31u;
                uint64_t v = j < nlimbs ? w[j] : 0u;
                if (j + 1 < nlimbs) v |= (uint64_t)w[j + 1] << 32;
                h[a * K + l] = (uint32_t)(v >> o) & gbbig28::kMask;
            }
        }
        std::vector<uint32_t> ans;
        gb_status r;
        switch (K) {
        case 4: r = big28_passes<4>(c, h, kk, ans, st); break;
        case 6: r = big28_passes<6>(c, h, kk, ans, st); break;
        case 8: r = big28_passes<8>(c, h, kk, ans, st); break;
        case 10: r = big28_passes<10>(c, h, kk, ans, st); break;
        case 12: r = big28_passes<12>(c, h, kk, ans, st); break;
        case 14: r = big28_passes<14>(c, h, kk, ans, st); break;
        case 16: r = big28_passes<16>(c, h, kk, ans, st); break;
        case 20: r = big28_passes<20>(c, h, kk, ans, st); break;
        case 24: r = big28_passes<24>(c, h, kk, ans, st); break;
        case 28: r = big28_passes<28>(c, h, kk, ans, st); break;
        case 32: r = big28_passes<32>(c, h, kk, ans, st); break;
        case 36: r = big28_passes<36>(c, h, kk, ans, st); break;
        default: r = big28_passes<37>(c, h, kk, ans, st); break;
        }
        if (r != GB_OK) return r;
        for (size_t a = 0; a < kk; ++a) {
            const uint32_t i = sel[f][a];
            p[i] = ans[a] < c->ntab ? c->h_primes[ans[a]] : 0ull;
            unresolved = unresolved || p[i] == 0;
        }
    }
    if (unresolved) return fail(c, GB_EUNRESOLVED, "no partition with p in the resident prime table");
    return GB_OK;
}
