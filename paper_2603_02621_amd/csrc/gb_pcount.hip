// gb_pcount.hip -- Goldbach partition counts c(n) for a range of even n
// (paper section "Future work": large-scale counts of the partitions
// n = p + q into primes p <= q), on the odd-number bitset of the tile sieve.
//
// With m = n/2 - 1 and bit i of the bitset B standing for 2i + 1, the odd
// partitions of n >= 6 are the pairs (i, m - i) with B[i] = B[m - i] = 1 and
// i <= m/2, so c(n) = sum over i <= floor(m/2) of B[i] B[m - i].  A lane
// owns one n; a workgroup of 512 lanes owns 512 consecutive n and walks i in
// steps of 32: the word X = B[32a .. 32a + 31] is the same for every lane,
// and a lane's partner bits B[m - 32a - t], t = 0..31, are 32 consecutive
// bits of the bit-reversed bitset.  The workgroup stages both in LDS a chunk
// of steps at a time (the q side reversed once per word), after which a step
// is one funnel shift, one AND and one popcount-accumulate per lane.  The
// range of steps of a block is split over several workgroups, which add
// their partial counts with 64-bit atomics.
#include <algorithm>
#include <cstring>

#include "gb_runtime.h"

namespace {

constexpr uint32_t PC_NT = 512;    // consecutive n (lanes) per workgroup
constexpr uint32_t PC_C = 2048;    // steps of 32 values of i per staged chunk
constexpr uint32_t PC_R = PC_C + PC_NT / 32 + 8;  // staged words of the q side

typedef uint32_t pc_v4 __attribute__((ext_vector_type(4)));

struct PcArgs {
    const uint32_t *bits;          // odd-number bitset, bit i <-> 2i + 1
    uint64_t nwords;               // its length in 32-bit words
    uint64_t m_first;              // m = n/2 - 1 of the first n >= 6
    uint64_t nm;                   // number of n >= 6
    unsigned long long *counts;    // count of m_first + j at index out_off + j
    uint64_t out_off;
    uint32_t nsplit;               // workgroups per block of PC_NT n
};

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s)
{
    return __builtin_amdgcn_alignbit(hi, lo, s);
}

// popcount(x) + acc in one v_bcnt_u32_b32 (the compiler otherwise counts
// from zero and adds the counts separately)
__device__ __forceinline__ uint32_t popc_acc(uint32_t x, uint32_t acc)
{
    uint32_t d;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(d) : "v"(x), "v"(acc));
    return d;
}

__global__ __launch_bounds__(PC_NT) void k_pcount(PcArgs a)
{
    __shared__ __align__(16) uint32_t xs[PC_C + 4];
    __shared__ uint32_t rs[PC_R];
    const uint32_t tid = threadIdx.x;
    const uint64_t blk = blockIdx.x / a.nsplit;
    const uint32_t part = blockIdx.x % a.nsplit;
    const uint64_t m0 = a.m_first + blk * PC_NT;
    const uint64_t mend = a.m_first + a.nm;
    const uint64_t mlast = (m0 + PC_NT < mend ? m0 + PC_NT : mend) - 1;
    const uint64_t m = m0 + tid;
    const uint64_t lim = m / 2;                       // i <= floor(m/2)
    // steps a = 0 .. amax cover i up to the block's largest floor(m/2); below
    // afull every i of the step is within every lane's bound
    const uint64_t amax = (mlast / 2) >> 5;
    const uint64_t afull = (m0 / 2) >> 5;
    const uint64_t per = (amax + a.nsplit) / a.nsplit;
    const uint64_t ab = (uint64_t)part * per;
    const uint64_t ae = ab + per < amax + 1 ? ab + per : amax + 1;
    // bit offset of the lane's partner window within a staged word pair
    const uint32_t sh = (uint32_t)((31u - (uint32_t)m) & 31u);
    uint32_t acc = 0;

    for (uint64_t a0 = ab; a0 < ae; a0 += PC_C) {
        const uint32_t ns = ae - a0 < PC_C ? (uint32_t)(ae - a0) : PC_C;
        // The q side of step a for lane l spans bits m_l - 32a - 31 .. m_l - 32a
        // of B: over the chunk and the block, words maxw down to maxw - K + 1.
        // rs[k] holds word maxw - k bit-reversed (zero outside the bitset), so
        // B bit x sits at rs position 32 maxw + 31 - x, and the 32 partner bits
        // of a step are rs positions u .. u + 31, u = 32 maxw + 31 - m + 32a.
        const uint64_t maxw = (m0 + PC_NT - 1 - 32 * a0) >> 5;
        const uint32_t K = ns + PC_NT / 32 + 6;
        __syncthreads();                                // the previous chunk is done
        for (uint32_t k = tid; k < K; k += PC_NT) {
            const uint64_t w = maxw - k;                 // wraps below zero
            rs[k] = __builtin_bitreverse32(w < a.nwords ? a.bits[w] : 0u);
        }
        for (uint32_t k = tid; k < ((ns + 3u) & ~3u); k += PC_NT)
            xs[k] = (k < ns && a0 + k < a.nwords) ? a.bits[a0 + k] : 0u;
        __syncthreads();

        const uint64_t u0 = 32 * maxw + 31 - m + 32 * a0;   // >= 0: m <= m0 + PC_NT - 1
        const uint32_t *rp = rs + (uint32_t)(u0 >> 5);
        uint32_t lo = rp[0];
        uint32_t s = 0;
        const uint32_t nfull = afull <= a0 ? 0u : (afull - a0 < ns ? (uint32_t)(afull - a0) : ns);
        // two running counts, so that consecutive popcounts do not wait on
        // each other
        uint32_t acc2 = 0;
        for (; s + 8 <= nfull; s += 8) {
            const pc_v4 x = *reinterpret_cast<const pc_v4 *>(xs + s);
            const pc_v4 y = *reinterpret_cast<const pc_v4 *>(xs + s + 4);
            const uint32_t w1 = rp[s + 1], w2 = rp[s + 2], w3 = rp[s + 3], w4 = rp[s + 4];
            const uint32_t w5 = rp[s + 5], w6 = rp[s + 6], w7 = rp[s + 7], w8 = rp[s + 8];
            acc = popc_acc(funnel(w1, lo, sh) & x.x, acc);
            acc2 = popc_acc(funnel(w2, w1, sh) & x.y, acc2);
            acc = popc_acc(funnel(w3, w2, sh) & x.z, acc);
            acc2 = popc_acc(funnel(w4, w3, sh) & x.w, acc2);
            acc = popc_acc(funnel(w5, w4, sh) & y.x, acc);
            acc2 = popc_acc(funnel(w6, w5, sh) & y.y, acc2);
            acc = popc_acc(funnel(w7, w6, sh) & y.z, acc);
            acc2 = popc_acc(funnel(w8, w7, sh) & y.w, acc2);
            lo = w8;
        }
        acc += acc2;
        for (; s < ns; ++s) {
            const uint32_t hi = rp[s + 1];
            uint32_t v = funnel(hi, lo, sh) & xs[s];
            // i = 32(a0 + s) + t must not exceed floor(m/2)
            const int64_t rem = (int64_t)lim - 32 * (int64_t)(a0 + s);
            v &= rem >= 31 ? ~0u : (rem < 0 ? 0u : (2u << (uint32_t)rem) - 1u);
            acc += __popc(v);
            lo = hi;
        }
    }
    if (m <= mlast && acc) atomicAdd(&a.counts[a.out_off + (m - a.m_first)], (unsigned long long)acc);
}

// counts[0..n) = 0 (1 at index 0 when the range starts at n = 4); the
// reduction slots to their identities
__global__ void k_pc_fill(unsigned long long *counts, uint64_t n, int has4, unsigned long long *red)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = i; k < n; k += stride) counts[k] = (k == 0 && has4) ? 1ull : 0ull;
    if (i == 0) {
        red[0] = 0ull;           // sum
        red[1] = ~0ull;          // smallest (c << 25) | index
        red[2] = 0ull;           // largest (c << 25) | (2^25 - 1 - index)
    }
}

// sum, and the smallest and largest count with the smallest index attaining
// each, as 64-bit keys (at most 2^25 n per call, counts below 2^39)
__global__ void k_pc_summary(const unsigned long long *counts, uint64_t n, unsigned long long *red)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long sum = 0, kmin = ~0ull, kmax = 0;
    for (uint64_t k = i; k < n; k += stride) {
        const unsigned long long c = counts[k];
        sum += c;
        const unsigned long long k1 = (c << 25) | k, k2 = (c << 25) | ((1ull << 25) - 1 - k);
        kmin = k1 < kmin ? k1 : kmin;
        kmax = k2 > kmax ? k2 : kmax;
    }
    for (int off = 32; off > 0; off >>= 1) {
        sum += __shfl_xor(sum, off);
        const unsigned long long o1 = __shfl_xor(kmin, off), o2 = __shfl_xor(kmax, off);
        kmin = o1 < kmin ? o1 : kmin;
        kmax = o2 > kmax ? o2 : kmax;
    }
    if ((threadIdx.x & 63u) == 0u) {
        if (sum) atomicAdd(&red[0], sum);
        if (kmin != ~0ull) atomicMin(&red[1], kmin);
        if (kmax) atomicMax(&red[2], kmax);
    }
}

}  // namespace

using namespace gbrt;

gb_status gb_partition_counts(gb_ctx *c, uint64_t lo, uint64_t hi, uint64_t *counts, gb_pc_result *res,
                              void *stream)
{
    if (!c || !res) return fail(c, GB_EINVAL, "null argument");
    std::memset(res, 0, sizeof *res);
    if (hi > (1ull << 63)) return fail(c, GB_EINVAL, "hi above 2^63");
    uint64_t n_first = std::max<uint64_t>(lo, 4);
    n_first += n_first & 1;
    const uint64_t n_last = hi - (hi & 1);
    if (lo > hi || n_first > n_last) return GB_OK;
    const uint64_t C = (n_last - n_first) / 2 + 1;
    if (C > (1ull << 25)) return fail(c, GB_EINVAL, "more than 2^25 even n in one call");
    if (hi > c->prm.max_hi) return fail(c, GB_ERANGE, "hi above the context's max_hi");
    if (hipSetDevice(c->prm.device) != hipSuccess) return fail(c, GB_EDEVICE, "hipSetDevice failed");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace &ws = c->ws;

    // the odd numbers 1 .. n_last - 3 (the largest q), rounded up to 64 bits
    const uint64_t n6 = std::max<uint64_t>(n_first, 6);
    const bool any6 = n6 <= n_last;
    const uint64_t nbits = any6 ? (((n_last - 3 - 1) / 2 + 1 + 63) & ~63ull) : 64;
    const uint64_t bytes = nbits / 8 + (counts ? 0 : C * 8);
    if (bytes > c->prm.mem_budget) return fail(c, GB_ENOMEM, "bitset and counts above mem_budget");
    GB_HIP(c, ws.pc_bits.ensure(nbits / 32));
    GB_HIP(c, ws.pc_red.ensure(3));
    GB_HIP(c, ws.h_pc_red.ensure(3));
    unsigned long long *out = reinterpret_cast<unsigned long long *>(counts);
    if (!out) {
        GB_HIP(c, ws.pc_counts.ensure(C));
        out = ws.pc_counts.p;
    }
    GB_HIP(c, hipEventRecord(ws.ev0, st));
    const uint32_t fill_grid = (uint32_t)std::min<uint64_t>((C + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pc_fill, dim3(fill_grid), dim3(256), 0, st, out, C, n_first == 4 ? 1 : 0, ws.pc_red.p);
    GB_HIP(c, hipGetLastError());
    if (any6) {
        gb_status stt = enqueue_sieve(c, ws, 1, nbits, ws.pc_bits.p, st);
        if (stt != GB_OK) return stt;
        PcArgs a{};
        a.bits = ws.pc_bits.p;
        a.nwords = nbits / 32;
        a.m_first = n6 / 2 - 1;
        a.nm = (n_last - n6) / 2 + 1;
        a.counts = out;
        a.out_off = (n6 - n_first) / 2;
        const uint64_t nblk = (a.nm + PC_NT - 1) / PC_NT;
        const uint64_t steps = ((a.m_first + a.nm - 1) / 2 >> 5) + 1;   // of the last block, the most
        // enough workgroups to fill the chip several times over, but at least
        // one chunk of steps each
        const uint64_t want = (8ull * (uint64_t)c->num_cu + nblk - 1) / nblk;
        a.nsplit = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, steps / PC_C));
        GB_HIP(c, hipEventRecord(ws.evt0, st));
        hipLaunchKernelGGL(k_pcount, dim3((uint32_t)(nblk * a.nsplit)), dim3(PC_NT), 0, st, a);
        GB_HIP(c, hipGetLastError());
        GB_HIP(c, hipEventRecord(ws.evt1, st));
    }
    const uint32_t sum_grid = (uint32_t)std::min<uint64_t>((C + 255) / 256, 1024);
    hipLaunchKernelGGL(k_pc_summary, dim3(sum_grid), dim3(256), 0, st, out, C, ws.pc_red.p);
    GB_HIP(c, hipGetLastError());
    GB_HIP(c, hipMemcpyAsync(ws.h_pc_red.p, ws.pc_red.p, 3 * 8, hipMemcpyDeviceToHost, st));
    GB_HIP(c, hipEventRecord(ws.ev1, st));
    GB_HIP(c, hipStreamSynchronize(st));

    const unsigned long long *r = ws.h_pc_red.p;
    const uint64_t mask = (1ull << 25) - 1;
    res->count = C;
    res->sum = r[0];
    res->min_c = r[1] >> 25;
    res->argmin_n = n_first + 2 * (r[1] & mask);
    res->max_c = r[2] >> 25;
    res->argmax_n = n_first + 2 * (mask - (r[2] & mask));
    float ms = 0.f;
    GB_HIP(c, hipEventElapsedTime(&ms, ws.ev0, ws.ev1));
    res->device_ms = ms;
    if (any6) {
        GB_HIP(c, hipEventElapsedTime(&ms, ws.evt0, ws.evt1));
        res->kernel_ms = ms;
    }
    return GB_OK;
}
