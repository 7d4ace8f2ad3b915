// gb_big.hip -- minimal Goldbach prime of even n beyond 64 bits (paper
// section "Arbitrary Precision Checker": small primes p in ascending order,
// q = n - p tested with Miller-Rabin), up to n < 2^1024.
//
// One wavefront per n.  Lane l takes the l-th next odd prime p of the
// resident table and runs the strong probable-prime test to base 2 on its
// q = n - p (multi-limb Montgomery arithmetic, gb_bignum.h).  The lowest
// passing lane's q is then tested to the other 24 prime bases 3 .. 97, one
// base per lane; if all pass, that p is the answer (every smaller p failed a
// base, so its q is composite); otherwise the next passing lane is tried,
// then the next 64 primes.
#include <cstring>

#include "gb_bignum.h"
#include "gb_runtime.h"

namespace {

using gbbig::Num;

__constant__ uint32_t kBigBases[25] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41,
                                       43, 47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97};

template <int K>
__global__ __launch_bounds__(256) void k_big(const uint32_t *n_all, uint64_t k, const uint32_t *primes,
                                             uint64_t nprimes, unsigned long long *p_out)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t idx = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
    if (idx >= k) return;                            // whole wave
    Num<K> n;
    for (int i = 0; i < K; ++i) n.w[i] = n_all[idx * K + i];
    for (uint64_t base = 0; base < nprimes; base += 64) {
        const uint64_t c = base + lane;
        const bool valid = c < nprimes;
        const uint32_t p = valid ? primes[c] : 3u;
        // q = n - p (n >= 2^64 > p)
        Num<K> q;
        {
            uint64_t br = p;
            for (int i = 0; i < K; ++i) {
                const uint64_t t = (uint64_t)n.w[i] - br;
                q.w[i] = (uint32_t)t;
                br = (t >> 63) & 1u;
            }
        }
        const bool pass2 = valid && gbbig::strong_prp<K>(q, 2u);
        unsigned long long m = __builtin_amdgcn_ballot_w64(pass2);
        while (m) {
            const uint32_t L = (uint32_t)__builtin_ctzll(m);
            m &= m - 1ull;
            // the candidate's q in every lane, then one more base per lane
            Num<K> qL;
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
hipError_t launch_big(const uint32_t *n, uint64_t k, const uint32_t *primes, uint64_t nprimes,
                      unsigned long long *p, hipStream_t st)
{
    hipLaunchKernelGGL(k_big<K>, dim3((uint32_t)((k + 3) / 4)), dim3(256), 0, st, n, k, primes, nprimes, p);
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
    // limb counts compiled: 4, 8, 12, 16, 24, 32
    const int K = nlimbs <= 4 ? 4 : nlimbs <= 8 ? 8 : nlimbs <= 12 ? 12 : nlimbs <= 16 ? 16 : nlimbs <= 24 ? 24 : 32;
    // every n even and at least 2^64
    for (size_t i = 0; i < k; ++i) {
        const uint32_t *w = n + i * nlimbs;
        bool big = false;
        for (uint32_t j = 2; j < nlimbs; ++j) big = big || w[j] != 0u;
        if ((w[0] & 1u) || !big) return fail(c, GB_EINVAL, "n must be even and at least 2^64");
    }
    if (hipSetDevice(c->prm.device) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // padded to K limbs per n
    std::vector<uint32_t> h((size_t)k * K, 0u);
    for (size_t i = 0; i < k; ++i) std::memcpy(&h[i * K], n + i * nlimbs, nlimbs * 4);
    Workspace &ws = c->ws;
    GB_HIP(c, ws.big_n.ensure(h.size()));
    GB_HIP(c, ws.big_p.ensure(k));
    GB_HIP(c, hipMemcpyAsync(ws.big_n.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, st));
    switch (K) {
    case 4: GB_HIP(c, launch_big<4>(ws.big_n.p, k, c->d_primes, c->ntab, ws.big_p.p, st)); break;
    case 8: GB_HIP(c, launch_big<8>(ws.big_n.p, k, c->d_primes, c->ntab, ws.big_p.p, st)); break;
    case 12: GB_HIP(c, launch_big<12>(ws.big_n.p, k, c->d_primes, c->ntab, ws.big_p.p, st)); break;
    case 16: GB_HIP(c, launch_big<16>(ws.big_n.p, k, c->d_primes, c->ntab, ws.big_p.p, st)); break;
    case 24: GB_HIP(c, launch_big<24>(ws.big_n.p, k, c->d_primes, c->ntab, ws.big_p.p, st)); break;
    default: GB_HIP(c, launch_big<32>(ws.big_n.p, k, c->d_primes, c->ntab, ws.big_p.p, st)); break;
    }
    GB_HIP(c, hipMemcpyAsync(p, ws.big_p.p, k * 8, hipMemcpyDeviceToHost, st));
    GB_HIP(c, hipStreamSynchronize(st));
    for (size_t i = 0; i < k; ++i)
        if (p[i] == 0) return fail(c, GB_EUNRESOLVED, "no partition with p in the resident prime table");
    return GB_OK;
}
