// gb_pcount.hip -- Goldbach partition counts c(n) for a range of even n
// (paper section "Future work": large-scale counts of the partitions
// n = p + q into primes p <= q), on the odd-number bitset of the tile sieve.
//
// With m = n/2 - 1 and bit i of the bitset B standing for 2i + 1, the odd
// partitions of n >= 6 are the pairs (i, m - i) with B[i] = B[m - i] = 1 and
// i <= m/2, so c(n) = sum over i <= floor(m/2) of B[i] B[m - i].  A lane
// owns one n and walks i in steps of 32: the word B[32a .. 32a + 31] is the
// same for every lane, and a lane's partner bits B[m - 32a - t], t = 0..31,
// are 32 consecutive bits of the bit-reversed bitset.  Lanes are laid out so
// that all lanes of a wave share those bits' offset within a word (one
// residue of m mod 32 per wave); each wave then stages its partner words
// shifted and reversed once per chunk of steps, and a step is one AND and
// one popcount-accumulate per lane.  The steps of a block are split over
// several workgroups, which add their partial counts with 64-bit atomics.
#include <algorithm>
#include <cstring>

#include "gb_runtime.h"

namespace {

typedef uint32_t pc_v4 __attribute__((ext_vector_type(4)));
typedef uint32_t pc_v16 __attribute__((ext_vector_type(16)));
// the p-side words are the same for every lane: read through the constant
// address space, they arrive in scalar registers, 16 per load
typedef __attribute__((address_space(4))) const pc_v16 const_v16;
typedef __attribute__((address_space(4))) const uint32_t const_u32;

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

// A block of 2048 consecutive m (m0 a multiple of 32) is covered by 4
// workgroups of 8 waves,
// wave w of group g taking the residue r = 8g + w and lane l the
// m = m0 + 32l + r.  All lanes of a wave then share the partner window's bit
// shift (r + 1) mod 32, so the wave builds its shifted, bit-reversed partner
// words once per chunk and a lane reads one of them per step: a step is one
// AND and one popcount-accumulate (no funnel shift per step).
constexpr uint32_t PR_NT = 512;              // 8 waves = 8 residues
constexpr uint32_t PR_BM = 2048;             // m per block (64 lanes x 32 residues)
constexpr uint32_t PR_C = 1024;              // steps per staged chunk
constexpr uint32_t PR_S = PR_C + 64;         // shifted partner words per wave
constexpr uint32_t PR_B = PR_C + 72;         // staged bitset words per workgroup

struct PcResArgs {
    const uint32_t *bits;
    uint64_t nwords;
    uint64_t m_first, m_last;      // the m = n/2 - 1 of the first and last n >= 6
    uint64_t m_base;               // m_first rounded down to a multiple of 32
    unsigned long long *counts;    // count of m at index out_off + (m - m_first)
    uint64_t out_off;
    uint32_t nsplit;
};

__global__ __launch_bounds__(PR_NT) void k_pcount_res(PcResArgs a)
{
    __shared__ uint32_t bs[PR_B];
    __shared__ uint32_t sw[PR_NT / 64][PR_S];
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63u;
    const uint32_t part = blockIdx.x % a.nsplit;
    const uint64_t grp = blockIdx.x / a.nsplit;       // block * 4 + residue group
    const uint64_t blk = grp >> 2;
    const uint32_t r = 8u * (uint32_t)(grp & 3u) + wave;
    const uint64_t m0 = a.m_base + blk * PR_BM;
    const uint64_t m = m0 + 32u * lane + r;
    const bool valid = m >= a.m_first && m <= a.m_last;
    const uint64_t lim = m / 2;
    // the block's valid m and its steps
    const uint64_t mlo = m0 > a.m_first ? m0 : a.m_first;
    const uint64_t mhi = m0 + PR_BM - 1 < a.m_last ? m0 + PR_BM - 1 : a.m_last;
    const uint64_t amax = (mhi / 2) >> 5;
    const uint64_t afull = (mlo / 2) >> 5;
    const uint64_t per = (amax + a.nsplit) / a.nsplit;
    const uint64_t ab = (uint64_t)part * per;
    const uint64_t ae = ab + per < amax + 1 ? ab + per : amax + 1;
    // the wave's partner windows start at bit m0 + r - 31 + 32 (l - a): word
    // m0/32 - 1 + delta + (l - a), bit offset (r + 1) mod 32
    const uint32_t sh = (r + 1u) & 31u;
    const uint32_t delta = r == 31u ? 1u : 0u;
    uint32_t acc = 0;

    for (uint64_t a0 = ab; a0 < ae; a0 += PR_C) {
        const uint32_t ns = ae - a0 < PR_C ? (uint32_t)(ae - a0) : PR_C;
        // bitset words m0/32 - 1 - (a0 + ns - 1) + k, k < ns + 66 (zero
        // outside the bitset), and the p-side words a0 .. a0 + ns - 1
        const uint64_t wlo = m0 / 32 - 1 - (a0 + ns - 1);   // wraps below zero
        __syncthreads();
        for (uint32_t k = tid; k < ns + 66u; k += PR_NT) {
            const uint64_t w = wlo + k;
            bs[k] = w < a.nwords ? a.bits[w] : 0u;
        }
        __syncthreads();
        // p side: words a0 .. a0 + ns - 1 of the bitset (a0 + ns - 1 <= amax
        // < nwords: the bitset reaches the largest q >= the largest p)
        const_u32 *xg = reinterpret_cast<const_u32 *>(reinterpret_cast<uintptr_t>(a.bits + a0));
        // this wave's shifted, bit-reversed partner words, in the order the
        // steps read them: the window of (l - a) with a = a0 + s is word
        // j = l - s + ns - 1 of the staged bits (bs[j + delta], bs[j + delta
        // + 1]), stored at sw[wave][ns + 62 - j], so lane l at step s reads
        // sw[wave][63 - l + s]
        for (uint32_t k = lane; k < ns + 63u; k += 64u) {
            const uint32_t j = ns + 62u - k;
            sw[wave][k] = __builtin_bitreverse32(funnel(bs[j + delta + 1u], bs[j + delta], sh));
        }
        __syncthreads();
        const uint32_t *sp = sw[wave] + 63u - lane;   // step s reads sp[s]
        uint32_t s = 0;
        const uint32_t nfull = afull <= a0 ? 0u : (afull - a0 < ns ? (uint32_t)(afull - a0) : ns);
        uint32_t acc2 = 0;
        for (; s + 16 <= nfull; s += 16) {
            const pc_v16 x = *reinterpret_cast<const_v16 *>(xg + s);
            const uint32_t *q = sp + s;
#pragma unroll
            for (int t = 0; t < 16; t += 2) {
                acc = popc_acc(q[t] & x[t], acc);
                acc2 = popc_acc(q[t + 1] & x[t + 1], acc2);
            }
        }
        acc += acc2;
        for (; s < ns; ++s) {
            uint32_t v = sp[s] & xg[s];
            const int64_t rem = (int64_t)lim - 32 * (int64_t)(a0 + s);
            v &= rem >= 31 ? ~0u : (rem < 0 ? 0u : (2u << (uint32_t)rem) - 1u);
            acc += __popc(v);
        }
    }
    if (valid && acc) atomicAdd(&a.counts[a.out_off + (m - a.m_first)], (unsigned long long)acc);
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
        PcResArgs a{};
        a.bits = ws.pc_bits.p;
        a.nwords = nbits / 32;
        a.m_first = n6 / 2 - 1;
        a.m_last = n_last / 2 - 1;
        a.m_base = a.m_first & ~31ull;
        a.counts = out;
        a.out_off = (n6 - n_first) / 2;
        const uint64_t ngrp = 4 * ((a.m_last + 1 - a.m_base + PR_BM - 1) / PR_BM);
        const uint64_t steps = ((a.m_last / 2) >> 5) + 1;   // of the last block, the most
        // enough workgroups to fill the chip several times over, but at least
        // one chunk of steps each
        const uint64_t want = (8ull * (uint64_t)c->num_cu + ngrp - 1) / ngrp;
        a.nsplit = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, steps / PR_C));
        GB_HIP(c, hipEventRecord(ws.evt0, st));
        hipLaunchKernelGGL(k_pcount_res, dim3((uint32_t)(ngrp * a.nsplit)), dim3(PR_NT), 0, st, a);
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
