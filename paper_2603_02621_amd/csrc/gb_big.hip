// gb_big.hip -- minimal Goldbach prime of even n beyond 64 bits (paper
// section "Arbitrary Precision Checker": small primes p in ascending order,
// q = n - p tested with Miller-Rabin), up to n < 2^1024.
//
// Below 2^446 (n as K = 4, 6, ..., 16 limbs of 28 bits, gb_bignum28.h) the
// host runs passes of one launch each.  A launch is a list of lane tasks,
// 64 to a wavefront: first the search groups, then the confirmations.
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
// wavefronts.  From 447 bits on (32 limbs of 32 bits, gb_bignum.h) one
// wavefront per n does the search and confirmation in one kernel.
#include <algorithm>
#include <cstring>

#include "gb_bignum.h"
#include "gb_bignum28.h"
#include "gb_runtime.h"

namespace {

using namespace gbrt;
using gbbig::Num;

__constant__ uint32_t kBigBases[25] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41,
                                       43, 47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97};

constexpr uint32_t kOddBases[24] = {3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41,
                                     43, 47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97};

// n mod r for a small r (r < 2^12), most significant limb first (32- and
// 28-bit limbs)
template <int K> __device__ __forceinline__ uint32_t mod_small(const Num<K> &n, uint32_t r)
{
    const uint32_t t = (uint32_t)((1ull << 32) % r);
    uint32_t acc = 0;
#pragma unroll
    for (int i = K - 1; i >= 0; --i) acc = (acc * t + n.w[i] % r) % r;
    return acc;
}

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

// One pass.  Lane task t (64 per wavefront, blockIdx.x * 256 + threadIdx.x):
// t < S0 = nslist nways G is lane t mod G of search group t / G, which is way
// (t / G) mod nways of the ((t / G) / nways)-th n of slist (of all n when
// slist is null; their found entries are all ones before the pass); the
// next nclist * 24 tasks confirm the candidates of the n of clist, found in
// the pass before, one odd base each.
template <int K>
__global__ __launch_bounds__(256) void k_big_pass(const uint32_t *n_all, const uint32_t *slist, uint32_t nslist,
                                                  uint32_t G, uint32_t nways, const uint32_t *clist, uint32_t nclist,
                                                  const uint32_t *primes, uint32_t nprimes, const uint32_t *resume_in,
                                                  uint32_t *resume_out, uint32_t *found, uint32_t *bad)
{
    __shared__ uint32_t cand_all[4][64];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t t0 = ((uint64_t)blockIdx.x * 4u + wv) * 64u;
    const uint64_t S0 = (uint64_t)nslist * nways * G;
    const uint64_t total = S0 + (uint64_t)nclist * 24u;
    if (t0 >= total) return;                         // whole wave
    uint32_t *cand = cand_all[wv];
    // the search groups among this wave's lanes (G divides 64, so a group
    // never straddles two wavefronts)
    uint32_t gidx0 = 0u, gidx1 = 0u, gcnt0 = 0u, gcnt1 = 0u;
    const uint32_t ngw = 64u / G;
    for (uint32_t gi = 0; gi < ngw && t0 + (uint64_t)gi * G < S0; ++gi) {
        const uint32_t grp = (uint32_t)((t0 + (uint64_t)gi * G) / G);
        const uint32_t li = grp / nways, way = grp - li * nways;
        const uint32_t idx = slist ? slist[li] : li;
        const uint32_t cnt =
            big_collect<K>(cand + gi * G, G, way, nways, idx, n_all, primes, nprimes, resume_in, resume_out);
        if (gi == 0u) {
            gidx0 = idx;
            gcnt0 = cnt;
        } else {
            gidx1 = idx;
            gcnt1 = cnt;
        }
    }
    __builtin_amdgcn_wave_barrier();
    const uint64_t t = t0 + lane;
    const bool srch = t < S0;
    bool act = false;
    uint32_t idx = 0u, c = 0u, base = 2u;
    if (srch) {
        const uint32_t gi = lane / G;
        idx = gi ? gidx1 : gidx0;
        act = lane - gi * G < (gi ? gcnt1 : gcnt0);
        c = act ? cand[lane] : 0u;
    } else if (t < total) {
        const uint64_t k = t - S0;
        const uint32_t ci = (uint32_t)(k / 24u), j = (uint32_t)(k - (uint64_t)ci * 24u);
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
    for (uint32_t gi = 0; gi < ngw; ++gi) {
        const unsigned long long gm = G == 64u ? m : (m >> (gi * 32u)) & 0xFFFFFFFFull;
        if (gm != 0ull && lane == 0u)
            __hip_atomic_fetch_min(&found[gi ? gidx1 : gidx0],
                                   __builtin_amdgcn_readlane(c, gi * G + (uint32_t)__builtin_ctzll(gm)),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!srch && act && !pass) __hip_atomic_fetch_or(&bad[idx], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The one-kernel form, used for 32 limbs: the same filter and base-2 search
// in one wavefront per n, the lowest passing lane's q then tested to the
// other 24 bases by lanes 0 .. 23 of the same wavefront (next passing lane,
// then the next 64 surviving p, when it fails one).  The two-kernel form at
// 32 limbs did not finish a 520-bit case on the GPU; its cause is not
// known, so that form is kept to 4 .. 16 limbs.
template <int K>
__global__ __launch_bounds__(256) void k_big_wave(const uint32_t *n_all, uint64_t k, const uint32_t *primes,
                                                  uint64_t nprimes, unsigned long long *p_out)
{
    __shared__ uint32_t cand_all[4][64];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t idx = (uint64_t)blockIdx.x * 4u + wv;
    if (idx >= k) return;                            // whole wave
    uint32_t *cand = cand_all[wv];
    Num<K> n;
#pragma unroll
    for (int i = 0; i < K; ++i) n.w[i] = n_all[idx * K + i];
    uint32_t nres[24];
#pragma unroll
    for (int j = 0; j < 24; ++j) nres[j] = mod_small(n, kOddBases[j]);
    uint64_t next = 0;
    for (;;) {
        uint32_t cnt = 0;
        while (cnt < 64u && next < nprimes) {
            const uint64_t c = next + lane;
            const bool valid = c < nprimes;
            const uint32_t p = valid ? primes[c] : 0u;
            bool hit = false;
#pragma unroll
            for (int j = 0; j < 24; ++j) hit = hit || (p % kOddBases[j] == nres[j]);
            const bool keep = valid && !hit;
            const unsigned long long m = __builtin_amdgcn_ballot_w64(keep);
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            const uint32_t room = 64u - cnt;
            if (keep && rank < room) cand[cnt + rank] = p;
            const uint32_t tot = (uint32_t)__popcll(m);
            if (tot > room) {
                next += (uint64_t)__builtin_ctzll(__builtin_amdgcn_ballot_w64(keep && rank == room));
                cnt = 64u;
            } else {
                next += 64u;
                cnt += tot;
            }
        }
        if (cnt == 0u) break;                        // table exhausted
        __builtin_amdgcn_wave_barrier();
        const bool act = lane < cnt;
        const uint32_t p = act ? cand[lane] : 3u;
        __builtin_amdgcn_wave_barrier();
        Num<K> q;
        {
            uint64_t br = p;
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const uint64_t t = (uint64_t)n.w[i] - br;
                q.w[i] = (uint32_t)t;
                br = (t >> 63) & 1u;
            }
        }
        const bool pass2 = act && gbbig::strong_prp<K>(q, 2u);
        unsigned long long m = __builtin_amdgcn_ballot_w64(pass2);
        while (m) {
            const uint32_t L = (uint32_t)__builtin_ctzll(m);
            m &= m - 1ull;
            Num<K> qL;
#pragma unroll
            for (int i = 0; i < K; ++i) qL.w[i] = __builtin_amdgcn_readlane(q.w[i], L);
            const bool ok = lane >= 24u || gbbig::strong_prp<K>(qL, kBigBases[lane + 1u]);
            if (__builtin_amdgcn_ballot_w64(!ok) == 0ull) {
                if (lane == 0u) p_out[idx] = __builtin_amdgcn_readlane(p, L);
                return;
            }
        }
    }
    if (lane == 0u) p_out[idx] = 0ull;               // no partition with p in the table
}

template <int K>
hipError_t launch_pass(const uint32_t *n, const uint32_t *slist, uint32_t nslist, uint32_t G, uint32_t nways,
                       const uint32_t *clist, uint32_t nclist, const uint32_t *primes, uint32_t nprimes,
                       const uint32_t *resume_in, uint32_t *resume_out, uint32_t *found, uint32_t *bad, hipStream_t st)
{
    const uint64_t tasks = (uint64_t)nslist * nways * G + (uint64_t)nclist * 24u;
    hipLaunchKernelGGL(k_big_pass<K>, dim3((uint32_t)((tasks + 255u) / 256u)), dim3(256), 0, st, n, slist, nslist, G,
                       nways, clist, nclist, primes, nprimes, resume_in, resume_out, found, bad);
    return hipGetLastError();
}

// Pass shape: the first pass gives every n one group of kFirstGroup
// survivors; later passes give each open n kLaterGroup-lane groups, as many
// ways as keep about one search wavefront per SIMD busy (at most 16), so
// that the n with large p_min do not run alone.
constexpr uint32_t kFirstGroup = 32, kLaterGroup = 32, kMaxWays = 16;

// The n of one limb count K (28-bit limbs): h holds them, K limbs each
// (k n); their answers go to ans (table indices, UINT32_MAX for none).
template <int K>
gb_status big28_passes(gb_ctx *c, const std::vector<uint32_t> &h, size_t k, std::vector<uint32_t> &ans,
                       hipStream_t st)
{
    Workspace &ws = c->ws;
    GB_HIP(c, ws.big_n.ensure(h.size()));
    GB_HIP(c, hipMemcpyAsync(ws.big_n.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, st));
    GB_HIP(c, ws.big_state.ensure(4 * k));
    GB_HIP(c, ws.big_list.ensure(2 * k));
    GB_HIP(c, ws.h_big.ensure(6 * k));
    const uint32_t np = (uint32_t)c->ntab;
    // pinned host copies of the four device arrays (resume point in, found,
    // resume point out, bad; k each), then the two lists
    uint32_t *resume = ws.h_big.p, *found = resume + k, *rout = found + k, *bad = rout + k, *hsl = bad + k,
             *hcl = hsl + k;
    uint32_t *d_resume = ws.big_state.p, *d_found = d_resume + k, *d_rout = d_found + k, *d_bad = d_rout + k;
    std::fill(resume, resume + k, 0u);
    ans.assign(k, UINT32_MAX);
    std::vector<uint32_t> sl, cl, nsl, ncl;
    bool all = true;                                 // the first pass searches every n
    uint32_t G = kFirstGroup, nways = 1;
    // Each pass searches the open n and confirms the candidates found in the
    // pass before.  Every pass moves each open n's resume point forward, so
    // the loop ends; the cap stops a call whose device results do not settle.
    const uint64_t target = (uint64_t)c->num_cu * 4u * 64u;   // search lanes: one wavefront per SIMD
    for (int pass = 0;; ++pass) {
        if (pass == 1024) return fail(c, GB_EDEVICE, "big-n search did not settle");
        const uint32_t nslist = all ? (uint32_t)k : (uint32_t)sl.size(), nclist = (uint32_t)cl.size();
        if (all)
            std::fill(found, found + k, UINT32_MAX);
        else
            for (uint32_t i : sl) found[i] = UINT32_MAX;
        std::copy(sl.begin(), sl.end(), hsl);
        std::copy(cl.begin(), cl.end(), hcl);
        GB_HIP(c, hipMemcpyAsync(d_resume, resume, 2 * k * 4, hipMemcpyHostToDevice, st));   // resume in, found
        GB_HIP(c, hipMemsetAsync(d_bad, 0, k * 4, st));
        // the two lists share one buffer: the search list, then the confirm list
        if (!all && nslist) GB_HIP(c, hipMemcpyAsync(ws.big_list.p, hsl, nslist * 4, hipMemcpyHostToDevice, st));
        if (nclist) GB_HIP(c, hipMemcpyAsync(ws.big_list.p + k, hcl, nclist * 4, hipMemcpyHostToDevice, st));
        const uint32_t *dsl = all ? nullptr : ws.big_list.p, *dcl = ws.big_list.p + k;
        GB_HIP(c, launch_pass<K>(ws.big_n.p, dsl, nslist, G, nways, dcl, nclist, c->d_primes, np, d_resume, d_rout,
                                 d_found, d_bad, st));
        GB_HIP(c, hipMemcpyAsync(found, d_found, 3 * k * 4, hipMemcpyDeviceToHost, st));   // found, resume out, bad
        GB_HIP(c, hipStreamSynchronize(st));
        // the searched n continue after the groups this pass took
        for (uint32_t li = 0; li < nslist; ++li) {
            const uint32_t i = all ? li : sl[li];
            resume[i] = rout[i];
        }
        nsl.clear();
        ncl.clear();
        for (uint32_t i : cl) {
            if (!bad[i]) {
                ans[i] = found[i];
                continue;
            }
            resume[i] = found[i] + 1u;               // a base-2 pseudoprime: resume after it
            if (resume[i] < np) nsl.push_back(i);    // else the table ends: unresolved
        }
        for (uint32_t li = 0; li < nslist; ++li) {
            const uint32_t i = all ? li : sl[li];
            if (found[i] < np)
                ncl.push_back(i);
            else if (resume[i] < np)
                nsl.push_back(i);
        }
        if (nsl.empty() && ncl.empty()) break;
        sl.swap(nsl);
        cl.swap(ncl);
        all = false;
        G = kLaterGroup;
        nways = sl.empty() ? 1u
                           : (uint32_t)std::max<uint64_t>(1u, std::min<uint64_t>(kMaxWays, target / ((uint64_t)sl.size() * G)));
    }
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
    // Forms: the smallest even K with 28K - 2 >= bits (n of at most 446 bits,
    // so q = n - p has 28K - 58 bits or more, which the 28-bit arithmetic
    // needs), one pass sequence per K present; 32 limbs of 32 bits (the
    // one-kernel form) from 447 bits on.  The two-kernel form at 32 limbs did
    // not finish a 520-bit case on the GPU and a 24-limb 32-bit form returned
    // wrong answers (both explained by a base-2 test that failed primes), so
    // they are not used.
    std::vector<uint32_t> wide;
    std::vector<uint32_t> sel[17];
    for (size_t i = 0; i < k; ++i) {
        if (bits[i] > 446) {
            wide.push_back((uint32_t)i);
            continue;
        }
        const uint32_t K = std::max(4u, (((uint32_t)bits[i] + 2u + 27u) / 28u + 1u) & ~1u);
        sel[K].push_back((uint32_t)i);
    }
    bool unresolved = false;
    for (int K = 4; K <= 16; K += 2) {
        if (sel[K].empty()) continue;
        const size_t kk = sel[K].size();
        // K limbs of 28 bits: limb l is bits 28 l .. 28 l + 27
        std::vector<uint32_t> h(kk * (size_t)K, 0u);
        for (size_t a = 0; a < kk; ++a) {
            const uint32_t *w = n + (size_t)sel[K][a] * nlimbs;
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
        default: r = big28_passes<16>(c, h, kk, ans, st); break;
        }
        if (r != GB_OK) return r;
        for (size_t a = 0; a < kk; ++a) {
            const uint32_t i = sel[K][a];
            p[i] = ans[a] < c->ntab ? c->h_primes[ans[a]] : 0ull;
            unresolved = unresolved || p[i] == 0;
        }
    }
    if (!wide.empty()) {
        const size_t kw = wide.size();
        std::vector<uint32_t> h(kw * 32, 0u);                // padded to 32 limbs of 32 bits
        for (size_t a = 0; a < kw; ++a) std::memcpy(&h[a * 32], n + (size_t)wide[a] * nlimbs, nlimbs * 4);
        Workspace &ws = c->ws;
        GB_HIP(c, ws.big_n.ensure(h.size()));
        GB_HIP(c, hipMemcpyAsync(ws.big_n.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, st));
        GB_HIP(c, ws.big_p.ensure(kw));
        hipLaunchKernelGGL(k_big_wave<32>, dim3((uint32_t)((kw + 3) / 4)), dim3(256), 0, st, ws.big_n.p, (uint64_t)kw,
                           c->d_primes, c->ntab, ws.big_p.p);
        GB_HIP(c, hipGetLastError());
        std::vector<unsigned long long> pw(kw);
        GB_HIP(c, hipMemcpyAsync(pw.data(), ws.big_p.p, kw * 8, hipMemcpyDeviceToHost, st));
        GB_HIP(c, hipStreamSynchronize(st));
        for (size_t a = 0; a < kw; ++a) {
            p[wide[a]] = pw[a];
            unresolved = unresolved || pw[a] == 0;
        }
    }
    if (unresolved) return fail(c, GB_EUNRESOLVED, "no partition with p in the resident prime table");
    return GB_OK;
}
