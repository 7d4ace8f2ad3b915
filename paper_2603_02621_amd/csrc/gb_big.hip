// gb_big.hip -- minimal Goldbach prime of even n beyond 64 bits (paper
// section "Arbitrary Precision Checker": small primes p in ascending order,
// q = n - p tested with Miller-Rabin), up to n < 2^1024.
//
// Below 2^448 (n as 4 .. 16 limbs of 28 bits, gb_bignum28.h) each pass is
// one launch whose blocks either search or confirm.  The search takes one
// wavefront per n and group of candidates.  The odd primes p of the resident
// table are first filtered, 64 at a time, by the 24 odd prime bases
// r = 3 .. 97: a q = n - p that r divides fails the strong test to base r
// (a^d and its squarings mod q are then multiples of r, never 1 or q - 1),
// so dropping p = n (mod r) leaves the answer unchanged; about a quarter of
// the p survive.  Lane l then takes the l-th of the group's 64 surviving p
// and runs the strong probable-prime test to base 2 on its q; the lowest
// passing lane gives the candidate.  The confirmation, in the next pass,
// tests each candidate's q to the other 24 bases, one (n, base) per lane.  A
// candidate that fails a base (a strong pseudoprime to base 2) sends its n
// back to the search, which resumes after it.  The answer is the first p
// whose q passes all 25 bases; every smaller p failed one, so its q is
// composite.  From 449 bits on (32 limbs of 32 bits, gb_bignum.h) one
// wavefront per n does the same in one kernel.
#include <algorithm>
#include <cstring>

#include "gb_bignum.h"
#include "gb_bignum28.h"
#include "gb_runtime.h"

namespace {

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

// One pass of the search: nways wavefronts per listed n, wavefront w taking
// the w-th group of 64 surviving p from resume_in[idx] on and testing it to
// base 2.  found[idx] (all ones before the pass) receives the smallest table
// index that passed; the last wavefront writes the table index after its
// group (nprimes at the table's end) to resume_out[idx].  resume_in is only
// read during the pass: the wavefronts of one n run in any order, so a write
// into the array the others read would move their groups.
template <int K>
__device__ __forceinline__ void big_search(uint32_t blk, const uint32_t *n_all, const uint32_t *list, uint32_t nlist,
                                           uint32_t nways, const uint32_t *primes, uint32_t nprimes,
                                           const uint32_t *resume_in, uint32_t *resume_out, uint32_t *found)
{
    __shared__ uint32_t cand_all[4][64];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t slot = blk * 4u + wv;
    if (slot >= nlist * nways) return;               // whole wave
    const uint32_t li = slot / nways, way = slot - li * nways;
    const uint32_t idx = list ? list[li] : li;
    uint32_t *cand = cand_all[wv];
    gbbig28::Num<K> n;
#pragma unroll
    for (int i = 0; i < K; ++i) n.w[i] = n_all[(uint64_t)idx * K + i];
    // n mod r for the 24 odd bases (the same in every lane)
    uint32_t nres[24];
#pragma unroll
    for (int j = 0; j < 24; ++j) nres[j] = mod_small(n, kOddBases[j]);
    // table indices of the surviving p ranked [lo, hi) from resume_in[idx] on
    const uint32_t lo = 64u * way, hi = lo + 64u;
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
    const uint32_t cnt = got > lo ? got - lo : 0u;
    if (cnt == 0u) return;                           // the table ends before the group
    __builtin_amdgcn_wave_barrier();
    const bool act = lane < cnt;
    const uint32_t c = act ? cand[lane] : 0u;
    const uint32_t p = act ? primes[c] : 3u;
    // q = n - p (n >= 2^64 > p)
    gbbig28::Num<K> q;
    big_sub_p(q, n.w, p);
    const bool pass2 = act && gbbig28::strong_prp2<K>(q);
    const unsigned long long m = __builtin_amdgcn_ballot_w64(pass2);
    if (m != 0ull && lane == 0u)
        __hip_atomic_fetch_min(&found[idx], __builtin_amdgcn_readlane(c, (uint32_t)__builtin_ctzll(m)), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

// One lane per (n, base 3 .. 97): bad[idx] is set when the candidate's q
// fails a base.
template <int K>
__device__ __forceinline__ void big_confirm(uint32_t blk, const uint32_t *n_all, const uint32_t *list, uint32_t nlist,
                                            const uint32_t *primes, uint32_t nprimes, const uint32_t *found,
                                            uint32_t *bad)
{
    const uint32_t g = blk * 256u + threadIdx.x;
    if (g >= nlist * 24u) return;
    const uint32_t slot = g / 24u, j = g - slot * 24u;
    const uint32_t idx = list ? list[slot] : slot;
    const uint32_t c = found[idx];
    if (c >= nprimes) return;                        // nothing to confirm
    const uint32_t p = primes[c];
    gbbig28::Num<K> q;
    big_sub_p(q, n_all + (uint64_t)idx * K, p);
    if (!gbbig28::strong_prp<K>(q, kBigBases[j + 1u]))
        __hip_atomic_fetch_or(&bad[idx], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One pass: blocks [0, sblocks) search the open n of slist (nslist n,
// nways wavefronts each; entries of found for them all ones), the other
// blocks confirm the candidates of the n in clist, found in the pass before,
// so that both run side by side.
template <int K>
__global__ __launch_bounds__(256) void k_big_pass(const uint32_t *n_all, const uint32_t *slist, uint32_t nslist,
                                                  uint32_t nways, uint32_t sblocks, const uint32_t *clist,
                                                  uint32_t nclist, const uint32_t *primes, uint32_t nprimes,
                                                  const uint32_t *resume_in, uint32_t *resume_out, uint32_t *found,
                                                  uint32_t *bad)
{
    if (blockIdx.x < sblocks)
        big_search<K>(blockIdx.x, n_all, slist, nslist, nways, primes, nprimes, resume_in, resume_out, found);
    else
        big_confirm<K>(blockIdx.x - sblocks, n_all, clist, nclist, primes, nprimes, found, bad);
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
hipError_t launch_pass(const uint32_t *n, const uint32_t *slist, uint32_t nslist, uint32_t nways, const uint32_t *clist,
                       uint32_t nclist, const uint32_t *primes, uint32_t nprimes, const uint32_t *resume_in,
                       uint32_t *resume_out, uint32_t *found, uint32_t *bad, hipStream_t st)
{
    const uint32_t sblocks = (uint32_t)(((uint64_t)nslist * nways + 3u) / 4u);
    const uint32_t cblocks = (uint32_t)(((uint64_t)nclist * 24u + 255u) / 256u);
    hipLaunchKernelGGL(k_big_pass<K>, dim3(sblocks + cblocks), dim3(256), 0, st, n, slist, nslist, nways, sblocks, clist,
                       nclist, primes, nprimes, resume_in, resume_out, found, bad);
    return hipGetLastError();
}

}  // namespace

using namespace gbrt;

gb_status gb_verify_big(gb_ctx *c, const uint32_t *n, uint32_t nlimbs, size_t k, uint64_t *p, void *stream)
{
    if (!c || (k && (!n || !p))) return fail(c, GB_EINVAL, "null argument");
    if (nlimbs < 3 || nlimbs > 32) return fail(c, GB_EINVAL, "nlimbs must be in 3..32");
    if (k == 0) return GB_OK;
    if (k > (1ull << 24)) return fail(c, GB_EINVAL, "at most 2^24 n per call");
    // every n even and at least 2^64; the bit length of the largest
    uint32_t bits = 0;
    for (size_t i = 0; i < k; ++i) {
        const uint32_t *w = n + i * nlimbs;
        bool big = false;
        for (uint32_t j = 2; j < nlimbs; ++j) big = big || w[j] != 0u;
        if ((w[0] & 1u) || !big) return fail(c, GB_EINVAL, "n must be even and at least 2^64");
        for (uint32_t j = nlimbs; j-- > 0;)
            if (w[j]) {
                bits = std::max(bits, 32u * j + 32u - (uint32_t)__builtin_clz(w[j]));
                break;
            }
    }
    // Forms compiled: 4, 8, 12 and 16 limbs of 28 bits (n below 2^448, the
    // two-kernel form), and 32 limbs of 32 bits (the one-kernel form).  A
    // 24-limb form of 32 bits returned wrong answers on gfx950 (its host build
    // is right; its device code keeps the multiplier in scratch), and the
    // two-kernel form at 32 limbs did not finish a 520-bit case, so every n
    // of 449 bits or more runs in the one-kernel 32-limb form.
    const int K = bits <= 112 ? 4 : bits <= 224 ? 8 : bits <= 336 ? 12 : bits <= 448 ? 16 : 32;
    if (hipSetDevice(c->prm.device) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<uint32_t> h((size_t)k * K, 0u);
    if (K == 32) {
        // padded to 32 limbs of 32 bits
        for (size_t i = 0; i < k; ++i) std::memcpy(&h[i * K], n + i * nlimbs, nlimbs * 4);
    } else {
        // K limbs of 28 bits: limb l is bits 28 l .. 28 l + 27
        for (size_t i = 0; i < k; ++i) {
            const uint32_t *w = n + i * nlimbs;
            for (int l = 0; l < K; ++l) {
                const uint32_t b0 = 28u * (uint32_t)l, j = b0 >> 5, o = b0 & 31u;
                uint64_t v = j < nlimbs ? w[j] : 0u;
                if (j + 1 < nlimbs) v |= (uint64_t)w[j + 1] << 32;
                h[i * K + l] = (uint32_t)(v >> o) & gbbig28::kMask;
            }
        }
    }
    Workspace &ws = c->ws;
    GB_HIP(c, ws.big_n.ensure(h.size()));
    GB_HIP(c, hipMemcpyAsync(ws.big_n.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, st));
    if (K == 32) {
        GB_HIP(c, ws.big_p.ensure(k));
        hipLaunchKernelGGL(k_big_wave<32>, dim3((uint32_t)((k + 3) / 4)), dim3(256), 0, st, ws.big_n.p, (uint64_t)k,
                           c->d_primes, c->ntab, ws.big_p.p);
        GB_HIP(c, hipGetLastError());
        GB_HIP(c, hipMemcpyAsync(p, ws.big_p.p, k * 8, hipMemcpyDeviceToHost, st));
        GB_HIP(c, hipStreamSynchronize(st));
        for (size_t i = 0; i < k; ++i)
            if (p[i] == 0) return fail(c, GB_EUNRESOLVED, "no partition with p in the resident prime table");
        return GB_OK;
    }
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
    std::vector<uint32_t> ans(k, UINT32_MAX), sl, cl, nsl, ncl;
    bool all = true;                                 // the first pass searches every n
    uint32_t nways = 1;
    // Each pass searches the open n and confirms the candidates found in the
    // pass before.  The n still open get several wavefronts each, one per
    // group of 64 surviving p, so that the last n do not run alone.  Every
    // pass moves each open n's resume point forward, so the loop ends; the
    // cap stops a call whose device results do not settle.
    const uint32_t target = (uint32_t)c->num_cu * 16u;
    for (int pass = 0;; ++pass) {
        if (pass == 256) return fail(c, GB_EDEVICE, "big-n search did not settle");
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
        hipError_t e;
        switch (K) {
        case 4: e = launch_pass<4>(ws.big_n.p, dsl, nslist, nways, dcl, nclist, c->d_primes, np, d_resume, d_rout, d_found, d_bad, st); break;
        case 8: e = launch_pass<8>(ws.big_n.p, dsl, nslist, nways, dcl, nclist, c->d_primes, np, d_resume, d_rout, d_found, d_bad, st); break;
        case 12: e = launch_pass<12>(ws.big_n.p, dsl, nslist, nways, dcl, nclist, c->d_primes, np, d_resume, d_rout, d_found, d_bad, st); break;
        default: e = launch_pass<16>(ws.big_n.p, dsl, nslist, nways, dcl, nclist, c->d_primes, np, d_resume, d_rout, d_found, d_bad, st); break;
        }
        GB_HIP(c, e);
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
        nways = sl.empty() ? 1u : std::max(1u, std::min(16u, target / (uint32_t)sl.size()));
    }
    bool unresolved = false;
    for (size_t i = 0; i < k; ++i) {
        p[i] = ans[i] < np ? c->h_primes[ans[i]] : 0ull;
        unresolved = unresolved || p[i] == 0;
    }
    if (unresolved) return fail(c, GB_EUNRESOLVED, "no partition with p in the resident prime table");
    return GB_OK;
}
