// gb_class.hip -- the minimal-p sieve-and-search tile kernel of the
// segmented Goldbach verifier, with the n and the q of the search split by
// residue mod 6 (gfx950, wave64).
//
// The method is the paper's segmented double sieve (section "Segmented
// Double-Sieve Verifier", subsection "Correct segmentation"): sieve the
// window of q = n - p, then take the candidate primes p in ascending order
// and mark every n for which n - p is prime; the first p that marks n is
// p_min(n).
//
// n side.  A tile holds the even n of M stretches of 384 integers,
// n = N0 + 384 K + 6 j + a with N0 a multiple of 384, 0 <= K < M,
// 0 <= j < 64 and a = 0, 2, 4.  The 64 n of one stretch K and one class a
// form one block, bit j of a 64-bit mask of unresolved n.
//
// q side.  q = n - p > 3 can only be prime when it is 1 or 5 mod 6, i.e.
// when a - p is not a multiple of 3.  For a = 2 (a = 4) that leaves the
// primes p = 1 (5) mod 6 and p = 3, half of them; for a = 0 all but 3.  The
// window keeps the numbers v = 6 k + 1 and v = 6 k + 5 as two bit planes
// over k (word w of plane i at LDS word 2 w + i; 2/3 of the odd numbers),
// and each class gets its own probe list of the primes that can give it a
// prime q (the others change no p_min).  For such p, q = 6 (N0/6 + 64 K + j
// - d) + c with c = (a - p) mod 6 and d = (p - a + c)/6: the q of a block
// are 64 consecutive bits of plane c.  A block needs 35.5 probes at 10^12
// instead of the 65 of a block of 64 consecutive n.
//
// Probes.  A list is read in groups of four, 48 bytes each: four packed
// words, four g = 2^16 - (p+1)/2 and four hit counters.  The four probes of
// a group start within two rows of the group's lowest start: one 32-byte
// read of rows R .. R+3 of both planes serves all four (the host checks the
// span and pads a group with copies of its previous entry where it would be
// wider).  A packed word holds the funnel shift in bits 4..0, the probe's
// row offset (0 or 1) in bit 5, its plane in bit 6 and the byte offset of
// the group's window from the block's first plane row in bits 31..16.
//
// Sieve.  The planes are cleared of the multiples m p (m = 1 or 5 mod 6,
// m p >= p^2) of every sieving prime above the wheel (the wheel pattern
// removes the multiples of 5 .. wheel_max; 2 and 3 never occur): for each
// plane the multiples form one progression of stride p in k.  Primes up to
// the plane length / 64 stride with one wave each, larger ones with one lane
// per prime (both planes).  Planes are marked with
// 1 = composite (LDS OR atomics) and inverted before the search.
//
// A hit (prime p, mask h of the n it settles) adds the popcount of h to
// p's hit counter and three multiply-adds to the checksum sums; a block
// keeps the key of its last hit, which carries its largest p_min.  The
// checksum weight of n is 2^33 b(n) + (2c+1) 2^i with b(n) = N0/128 + the
// block index 3 K + a/2 and j = 32 c + i.  Lanes take blocks as they finish
// them, from chunks their wave takes off a workgroup counter.
#include <type_traits>

#include "gb_internal.h"
#include "gb_device.h"

namespace {

// OR m into the LDS word at byte address addr.
__device__ __forceinline__ void lds_or(uint32_t addr, uint32_t m)
{
    __hip_atomic_fetch_or(reinterpret_cast<lds_u32 *>(static_cast<uintptr_t>(addr)), m, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Bit B of x copied to all 32 bits (v_bfe_i32).
template <int B>
__device__ __forceinline__ uint32_t flag_mask(uint32_t x)
{
    uint32_t d;
    asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(d) : "v"(x), "i"(B));
    return d;
}

// (m & a) | (~m & b) in one v_bfi_b32.
__device__ __forceinline__ uint32_t bsel(uint32_t m, uint32_t a, uint32_t b)
{
    uint32_t d;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(d) : "v"(m), "v"(a), "v"(b));
    return d;
}

// Byte offset of the plane word holding bit k of plane i (word w of plane i
// at LDS word 2 w + i).
__device__ __forceinline__ uint32_t plane_off(uint32_t k, uint32_t i) { return ((k >> 2) & ~7u) + 4u * i; }

// LDS carve-up of one workgroup (offsets in 32-bit words).
struct ClsLds {
    uint32_t *planes;          // 2 (Lk/32 + 4) words: the planes and padding rows
    uint32_t *cls;             // class headers and probe records (GB_CLS_*)
    unsigned long long *red;   // 7: checksum, n_exhaustive, max key, OR words, deficits
    unsigned long long *carry; // 6: the slot carry
    unsigned long long *tile;  // persistent mode: the tile just taken
    uint32_t *next;            // next block of the tile to hand out
    uint32_t *orw;             // 7: argmax recovery, OR of the windows per class, least n
};

__device__ __forceinline__ ClsLds carve_cls(uint32_t *smem, const GbTileArgs &a)
{
    ClsLds L;
    uint32_t o = 0;
    L.planes = smem;
    o += 2u * ((a.hk + 64u * a.sb_per_tile) / 32u + 4u);
    o = (o + 3u) & ~3u;   // records are read 16 bytes at a time
    L.cls = smem + o;
    o += a.cls_words;
    o = (o + 1u) & ~1u;   // 64-bit reductions
    L.red = reinterpret_cast<unsigned long long *>(smem + o);
    o += 2u * 7u;
    L.carry = reinterpret_cast<unsigned long long *>(smem + o);
    o += 2u * 6u;
    L.tile = reinterpret_cast<unsigned long long *>(smem + o);
    o += 2u;
    L.next = smem + o;
    o += 2u;
    L.orw = smem + o;
    return L;
}

// First strikes of the prime p in both planes: the least k (relative to
// the planes' first bit, value X + 6 k + c_i with X = 6 Kb) of a multiple
// m p >= max(X, p^2) with m p = c_i mod 6, i.e. m = p (plane 0, c = 1) or
// m = 5 p (plane 1, c = 5) mod 6.
//
// strikes_fast: X >= p^2 and 0 <= Kb < 2^50.  The multiples of p in plane i
// sit at k = b_i - Kb mod p, with b_0 the least k >= 0 with p | 6 k + 1 and
// b_1 = p - 1 - b_0 (the GB_PRIME6 entry e).  Kb mod p comes from the
// double nearest 1/p: floor(Kb/p) is then off by at most one (relative
// error below 2^-52 on a quotient below 2^50), and the residual Kb - q p is
// exact in one fma; both corrections are a three-way unsigned min.
__device__ __forceinline__ void strikes_fast(double kbd, uint4 e, uint32_t &k0, uint32_t &k1)
{
    const uint32_t p = e.x, b0 = e.y;
    const double pd = (double)p;
    const double x = __hiloint2double((int)e.w, (int)e.z);
    const double qd = floor(kbd * x);
    uint32_t t = (uint32_t)(int)fma(-qd, pd, kbd);   // Kb mod p, or that -p or +p
    t = min(t, min(t + p, t - p));
    const uint32_t u0 = b0 - t, u1 = (p - 1u - b0) - t;
    k0 = min(u0, u0 + p);
    k1 = min(u1, u1 + p);
}

// The same from the 64-bit reciprocal magic = floor((2^64-1)/p), for any
// Kb (negative, or X below p^2: then the strikes start at p^2).  The
// results can exceed 2^32.
__device__ __forceinline__ void strikes_slow(long long Kb, uint32_t p, unsigned long long magic,
                                             unsigned long long &k0, unsigned long long &k1)
{
    const unsigned long long pp = (unsigned long long)p * p;
    const long long X = 6ll * Kb;
    const unsigned long long Y = (X < 0 || (unsigned long long)X < pp) ? pp : (unsigned long long)X;
    unsigned long long q = __umul64hi(Y, magic);
    unsigned long long r = Y - q * p;
    if (r >= p) {
        r -= p;
        ++q;
    }
    const unsigned long long m0 = q + (r != 0ull);
    const uint32_t mu = (uint32_t)(m0 % 6ull), pr = p % 6u;
    const uint32_t d0 = (pr + 12u - mu) % 6u, d1 = (12u - pr - mu) % 6u;
    const unsigned long long base = m0 * p - (unsigned long long)X;   // >= 0
    k0 = (base + (unsigned long long)d0 * p) / 6u;
    k1 = (base + (unsigned long long)d1 * p) / 6u;
}

// Both first strikes of prime index k clamped to Lk (= no strike in the
// tile), as 32-bit plane bits, and p.
__device__ __forceinline__ uint32_t strikes_clamped(const GbTileArgs &a, bool fast, long long Kb, double kbd,
                                                    uint32_t k, uint32_t Lk, uint32_t &s0, uint32_t &s1)
{
    if (fast) {
        const uint4 e = a.prime6[k];
        strikes_fast(kbd, e, s0, s1);
        s0 = min(s0, Lk);
        s1 = min(s1, Lk);
        return e.x;
    }
    const uint32_t p = a.primes[k];
    unsigned long long k0, k1;
    strikes_slow(Kb, p, a.magic[k], k0, k1);
    s0 = k0 < Lk ? (uint32_t)k0 : Lk;
    s1 = k1 < Lk ? (uint32_t)k1 : Lk;
    return p;
}

// Hit counts of the workgroup's probe records into histogram row `row`, then
// cleared (threads stride over every record of every class).  The first
// flush of a persistent workgroup stores them, zeros included, as its own
// row of a.wg_hist (plain coalesced stores: 4 bytes per record instead of a
// device-scope atomic per record with hits); later ones, and every flush
// without wg_hist, add them to the histogram with 64-bit atomics.
__device__ void flush_hist_cls(const GbTileArgs &a, const ClsLds &L, uint32_t row, HistCarry &hc)
{
    unsigned long long *hist = a.hist + (unsigned long long)row * GB_HIST_BINS_I;
    uint32_t *rec = L.cls + GB_CLS_HDR;
    const bool store = a.wg_hist != nullptr && !hc.stored;
    uint32_t *own = store ? a.wg_hist + (unsigned long long)blockIdx.x * a.wg_hist_stride : nullptr;
    if (store && threadIdx.x == 0) own[0] = row;
    uint32_t r0 = 1;   // record index in class order, after the row word
    for (uint32_t h = 0; h < 3u; ++h) {
        const uint32_t first = L.cls[3u * h] / 4u, groups = L.cls[3u * h + 1u];
        for (uint32_t e = threadIdx.x; e < 4u * groups; e += blockDim.x) {
            const uint32_t wo = first + 12u * (e >> 2) + (e & 3u);
            const uint32_t c = rec[wo + 8u];
            if (store) {
                own[r0 + e] = c;
                rec[wo + 8u] = 0u;
            } else if (c) {
                // the prime from g = 2^16 - (p+1)/2, its index by bisection
                const uint32_t p = 131071u - 2u * rec[wo + 4u];
                uint32_t lo = 0, hi = a.np_cls;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (a.primes[mid] < p) lo = mid + 1u; else hi = mid;
                }
                atomicAdd(&hist[lo + 1u], (unsigned long long)c);
                rec[wo + 8u] = 0u;
            }
        }
        r0 += 4u * groups;
    }
    if (store) hc.stored = true;
}

template <int NT, int PB, bool SIEVE_ONLY>
__device__ void cls_tile(const GbTileArgs &a, unsigned long long g, const ClsLds &L, HistCarry &hc)
{
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    constexpr uint32_t NWAVES = NT / 64;

    // ---- the tile's window and geometry ------------------------------------
    uint32_t wi = 0;
    if (a.nwin > 1) {
        uint32_t lo = 0, hi = a.nwin - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (a.win[mid].tile_base <= g) lo = mid; else hi = mid - 1;
        }
        wi = lo;
    }
    const GbWindow W = a.win[wi];
    const unsigned long long t = g - W.tile_base;
    const unsigned long long N0 = W.first_n + 2ull * a.tile_n * t;   // a multiple of 384
    const unsigned long long rem = W.count - (unsigned long long)a.tile_n * t;
    const uint32_t cnt = rem < a.tile_n ? (uint32_t)rem : a.tile_n;
    const uint32_t M = (cnt + 191u) / 192u;            // stretches of 384 in this tile
    const uint32_t nblk = 3u * M;
    const uint32_t Hk = a.hk;
    const uint32_t Lk = Hk + 64u * M;                  // plane bits
    const uint32_t nw = Lk / 32u;                      // words per plane
    const long long Kb = (long long)(N0 / 6ull) - (long long)Hk;
    const double kbd = (double)Kb;
    const uint32_t np = W.np_sieve;
    const uint32_t ptop = np ? a.primes[np - 1] : 0u;
    const bool fast = Kb >= 0 && Kb < (1ll << 50) && (unsigned long long)(6 * Kb) >= (unsigned long long)ptop * ptop &&
                      np <= a.n_prime6;

    uint32_t base_a = (uint32_t)(uintptr_t)(lds_u32 *)L.planes;
    asm volatile("" : "+s"(base_a));
    const uint32_t end_a = base_a + 8u * nw;

    // ---- per-tile reductions; the workgroup's histogram row ----------------
    if (!SIEVE_ONLY) {
        if (tid < 7) L.red[tid] = 0ull;
        if (tid < 7) L.orw[tid] = tid < 6 ? 0u : 0xFFFFFFFFu;
        if (tid == 0) *L.next = NT;
        const uint32_t row = a.hist_per_slot ? W.slot : 0u;
        if (row != hc.row || hc.n + cnt > 0x7FFFFFFFull) {
            if (hc.row != kNoRow) flush_hist_cls(a, L, hc.row, hc);
            hc.row = row;
            hc.n = 0;
        }
        hc.n += cnt;
    }

    // ---- wheel pattern, 1 = composite --------------------------------------
    // Word w of plane i holds k = Kb + 32 w + b; pattern bit (Kb + 32 w + b)
    // mod P is 1 when 6 k + c_i is prime to every wheel prime 5 .. wheel_max.
    // Each thread keeps one plane (NT is even).
    {
        const uint32_t P = a.wheel6_len;
        const uint32_t i = tid & 1u;
        const uint32_t ci = i ? 5u : 1u;
        const uint32_t *pat = a.wheel6 + (unsigned long long)i * a.wheel6_stride;
        const long long k0 = Kb + 32ll * (long long)(tid >> 1);
        uint32_t ph = (uint32_t)(((k0 % (long long)P) + (long long)P) % (long long)P);
        const uint32_t step = (uint32_t)((32ull * (NT / 2)) % P);
        for (uint32_t idx = tid; idx < 2u * (nw + 4u); idx += NT) {
            const uint32_t w = idx >> 1;
            uint32_t v = ~__builtin_amdgcn_alignbit(pat[(ph >> 5) + 1u], pat[ph >> 5], ph & 31u);
            const long long kw = Kb + 32ll * (long long)w;
            if (kw <= 3ll || w >= nw) {
                // numbers below 2 (and the padding rows) are composite, the
                // wheel primes themselves prime (a rare path, kept rolled)
#pragma unroll 1
                for (uint32_t bt = 0; bt < 32; ++bt) {
                    const long long val = 6ll * (kw + (long long)bt) + (long long)ci;
                    if (val < 2 || w >= nw) v |= 1u << bt;
                    else if (val <= (long long)a.wheel_max &&
                             (val == 5 || val == 7 || val == 11 || val == 13 || val == 17 || val == 19))
                        v &= ~(1u << bt);
                }
            }
            L.planes[idx] = v;
            ph += step;
            if (ph >= P) ph -= P;
        }
    }
    __syncthreads();

    // ---- marking -------------------------------------------------------------
    // medium primes: one wave per prime, 32 lanes per plane, lane stride
    // 32 p.  Rounds of NT primes: lane j of wave w finds the first strikes
    // of prime w + NWAVES j of the round, then the wave takes its primes in
    // turn, each broadcast from its lane.
    {
        const uint32_t kbeg = a.k6_first;
        const uint32_t kend = min(a.k6_wave_end, np);
        const uint32_t i = lane & 1u;
        for (uint32_t kr = kbeg + __builtin_amdgcn_readfirstlane(wave); kr < kend; kr += NT) {
            const uint32_t k = kr + NWAVES * lane;
            uint32_t p = 0, f0 = Lk, f1 = Lk;
            if (k < kend) p = strikes_clamped(a, fast, Kb, kbd, k, Lk, f0, f1);
            const uint32_t nj = min(64u, (kend - kr + NWAVES - 1u) / NWAVES);
            for (uint32_t j = 0; j < nj; ++j) {
                const uint32_t pj = __builtin_amdgcn_readlane(p, j);
                const uint32_t s0 = __builtin_amdgcn_readlane(f0, j);
                const uint32_t s1 = __builtin_amdgcn_readlane(f1, j);
                const uint32_t kk = (i ? s1 : s0) + __umul24(lane >> 1, pj);   // s <= Lk, 31 pj < Lk
                if (kk < Lk) {
                    const uint32_t m = 1u << (kk & 31u);
                    const uint32_t stride = 8u * pj;   // bytes: 32 p bits
                    for (uint32_t wa = base_a + plane_off(kk, i); wa < end_a; wa += stride) lds_or(wa, m);
                }
            }
        }
    }
    // large primes: one lane per prime, both planes, a few strikes each;
    // from prime index k6_single on (p >= the plane length of a full tile)
    // at most one per plane.  Bit k of plane i is LDS byte ((k + kofs) >> 5)
    // 8 + 4 i with kofs = 4 base_a (base_a a multiple of 8, so the bit index
    // stays k mod 32).  The fast form loads the lane's next entry before it
    // marks this one (from an index clamped to the last prime, so every load
    // is in bounds).
    {
        const uint32_t kbeg = max(a.k6_wave_end, a.k6_first);
        const uint32_t kmid = min(max(a.k6_single, kbeg), np);
        const uint32_t kofs = 4u * base_a, kend_b = Lk + kofs;
        uint32_t k = kbeg + tid;
        if (fast && kbeg < np) {
            const uint32_t klast = np - 1u;   // < n_prime6
            uint4 e = a.prime6[min(k, klast)];
            for (; k < kmid; k += NT) {
                const uint4 en = a.prime6[min(k + NT, klast)];
                uint32_t f0, f1;
                strikes_fast(kbd, e, f0, f1);   // both below p
                for (uint32_t kk = f0 + kofs; kk < kend_b; kk += e.x) lds_or((kk >> 2) & ~7u, 1u << (kk & 31u));
                for (uint32_t kk = f1 + kofs; kk < kend_b; kk += e.x) lds_or(((kk >> 2) & ~7u) + 4u, 1u << (kk & 31u));
                e = en;
            }
            for (; k < np; k += NT) {
                const uint4 en = a.prime6[min(k + NT, klast)];
                uint32_t f0, f1;
                strikes_fast(kbd, e, f0, f1);
                const uint32_t k0 = f0 + kofs, k1 = f1 + kofs;
                if (k0 < kend_b) lds_or((k0 >> 2) & ~7u, 1u << (k0 & 31u));
                if (k1 < kend_b) lds_or(((k1 >> 2) & ~7u) + 4u, 1u << (k1 & 31u));
                e = en;
            }
        } else {
            for (; k < np; k += NT) {
                uint32_t f0, f1;
                const uint32_t p = strikes_clamped(a, false, Kb, kbd, k, Lk, f0, f1);
                for (uint32_t kk = f0 + kofs; kk < kend_b; kk += p) lds_or((kk >> 2) & ~7u, 1u << (kk & 31u));
                for (uint32_t kk = f1 + kofs; kk < kend_b; kk += p) lds_or(((kk >> 2) & ~7u) + 4u, 1u << (kk & 31u));
            }
        }
    }
    __syncthreads();
    for (uint32_t idx = tid; idx < 2u * (nw + 4u); idx += NT) L.planes[idx] = ~L.planes[idx];
    __syncthreads();

    if constexpr (SIEVE_ONLY) {
        // plane dump: tile t owns output bits [64 M_full t, 64 M_full t + 64 M) of each plane
        const unsigned long long obase = 2ull * a.sb_per_tile * t;
        for (uint32_t idx = tid; idx < 2u * 2u * M; idx += NT) {
            const uint32_t i = idx & 1u, w = idx >> 1;
            a.sieve_out[i * a.sieve_stride + obase + w] = L.planes[2u * (Hk / 32u + w) + i];
        }
        __syncthreads();
        return;
    } else {

    // ---- search ----------------------------------------------------------------
    const uint32_t slot = W.slot;
    const uint32_t hrow = a.hist_per_slot ? slot : 0u;
    unsigned long long *hist = a.hist + (unsigned long long)hrow * GB_HIST_BINS_I;
    const uint32_t lead = t == 0 ? W.lead : 0u;
    // per-n output index of n = N0 (wraps below zero when lead > 0)
    const unsigned long long outb = W.out_off - W.lead + (unsigned long long)a.tile_n * t;
    const uint32_t lo_off = 2u * lead, hi_off = 2u * (cnt - 1u);   // valid n - N0
    // blocks below bmask_lo or from bmask_hi on may hold n outside the tile
    const uint32_t bmask_lo = lead ? 3u : 0u;
    const uint32_t bmask_hi = 3u * (cnt / 192u);
    const bool first0 = N0 == 0ull;
    // n = 4 (p = 2) and n = 6 (q = 3 is not in the planes) are settled
    // apart: block 2 bit 0 and block 0 bit 1 when N0 = 0, when the tile
    // holds them and p <= P_max (else the exhaustive phase takes them)
    auto special_p = [&](uint32_t bb) -> uint32_t {
        if (!first0 || (bb != 0u && bb != 2u)) return 0u;
        const uint32_t off = bb == 2u ? 4u : 6u, p = bb == 2u ? 2u : 3u;
        if (off < lo_off || off > hi_off || p > a.pmax_fast) return 0u;
        return p;
    };
    auto block_mask = [&](uint32_t bb, uint32_t &mlo, uint32_t &mhi) {
        mlo = ~0u;
        mhi = ~0u;
        if (bb < bmask_lo || bb >= bmask_hi) {
            const uint32_t K = bb / 3u, base = 384u * K + 2u * (bb - 3u * K);
            unsigned long long m = 0ull;
            if (base <= hi_off) {
                const uint32_t jmin = lo_off > base ? (lo_off - base + 5u) / 6u : 0u;
                const uint32_t jmax = min(63u, (hi_off - base) / 6u);
                if (jmin <= jmax) m = (~0ull >> (63u - jmax)) & (~0ull << jmin);
            }
            mlo = (uint32_t)m;
            mhi = (uint32_t)(m >> 32);
        }
        if (special_p(bb)) mlo &= bb == 2u ? ~1u : ~2u;
    };

    uint32_t minkey = 0xFFFFFFFFu;
    uint32_t sumg = 0;
    unsigned long long accbg = 0;
    unsigned long long s0 = 0, s1 = 0;
    auto deficit = [&](uint32_t blk, uint32_t mlo, uint32_t mhi) {
        const uint32_t c = __popc(mlo) + __popc(mhi);
        if (c == 0u) return;
        atomicAdd(&L.red[4], ((N0 >> 7) + blk) * (unsigned long long)c);
        if (mlo) atomicAdd(&L.red[5], (unsigned long long)mlo);
        if (mhi) atomicAdd(&L.red[6], (unsigned long long)mhi);
    };
    auto push_unresolved = [&](uint32_t blk, uint32_t ulo, uint32_t uhi) {
        deficit(blk, ulo, uhi);
        const uint32_t K = blk / 3u, ai = blk - 3u * K;
        unsigned long long u = ((unsigned long long)uhi << 32) | ulo;
        while (u) {
            const uint32_t j = (uint32_t)__builtin_ctzll(u);
            u &= u - 1ull;
            const unsigned long long e = atomicAdd(a.list_count, 1ull);
            if (e < a.list_cap) {
                GbExh x;
                x.n = N0 + 384ull * K + 6ull * j + 2ull * ai;
                x.out_index = outb + 192ull * K + 3ull * j + ai;
                x.slot = slot;
                x.start_k = a.np_cls;
                x.p = 0;
                a.list[e] = x;
            }
        }
    };

    const uint32_t cls_a = (uint32_t)(uintptr_t)(lds_u32 *)L.cls;
    const uint32_t rec_a = cls_a + 4u * GB_CLS_HDR;
    // block state: unresolved mask U, LDS byte address of the next group of
    // four probe records (ka) and of the end of the class list (ka_end), LDS
    // byte address of the block's first plane row (bw), g << 16 of the
    // block's last hit
    uint32_t b = tid, ka = 0, ka_end = 0, Ulo = 0, Uhi = 0, lastkey = 0xFFFFFFFFu, bw = 0;
    unsigned long long ob = 0;   // per-n output index of the block's j = 0
    auto set_block = [&](uint32_t bb) {
        const uint32_t K = bb / 3u, ai = bb - 3u * K;
        ka = rec_a + L.cls[3u * ai];
        ka_end = rec_a + L.cls[3u * ai + 2u];
        bw = base_a + 16u * K;
        if constexpr (PB != 0) ob = outb + 192ull * K + ai;
        lastkey = 0xFFFFFFFFu;
        Ulo = ~0u;
        Uhi = ~0u;
    };
    // the rare blocks that need masking or hold a special n, or whose class
    // has no probe list
    auto edge_block = [&](uint32_t bb) {
        block_mask(bb, Ulo, Uhi);
        const uint32_t sp = special_p(bb);
        if (sp) {
            lastkey = sp == 2u ? 0xFFFF0000u : ((65536u - 2u) << 16);
            if constexpr (PB != 1) atomicAdd(&hist[sp == 2u ? 0u : 1u], 1ull);
            if constexpr (PB != 0)
                if (a.pmin) store_p<PB>(a.pmin, outb + (bb == 2u ? 2u : 3u), sp);
        }
    };
    auto empty_list = [&](uint32_t bb) {
        if (Ulo | Uhi) push_unresolved(bb, Ulo, Uhi);
        Ulo = Uhi = 0u;
    };
    constexpr uint32_t kChunk = 128u;
    uint32_t c_next = 0, c_end = 0;
    if (b < nblk) {
        set_block(b);
        if (b < bmask_lo || b >= bmask_hi || first0) edge_block(b);
        if (ka == ka_end) empty_list(b);
    }
    while (b < nblk) {
        constexpr uint32_t kGroupsPerCheck = 3u;
#pragma unroll
        for (uint32_t gg = 0; gg < kGroupsPerCheck; ++gg) {
            const v4u32 xv = *reinterpret_cast<const lds_v4 *>(static_cast<uintptr_t>(ka));
            const uint32_t xs[4] = {xv.x, xv.y, xv.z, xv.w};
            // rows R .. R+3 of both planes (word 2 t + i is plane i, row R + t)
            const lds_u64 *wp = reinterpret_cast<const lds_u64 *>(probe_addr(xs[0], bw));
            uint32_t wv[8];
#pragma unroll
            for (uint32_t t2 = 0; t2 < 4; ++t2) {
                const unsigned long long v = wp[t2];
                wv[2 * t2] = (uint32_t)v;
                wv[2 * t2 + 1] = (uint32_t)(v >> 32);
            }
            v4u32 gv = *reinterpret_cast<const lds_v4 *>(static_cast<uintptr_t>(ka + 16u));
            asm volatile("" : "+v"(gv.x), "+v"(gv.y), "+v"(gv.z), "+v"(gv.w));
            const uint32_t gs[4] = {gv.x, gv.y, gv.z, gv.w};
            uint32_t pcs[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                const uint32_t x = xs[u];
                // the probe's plane (bit 6), then its row (bit 5)
                const uint32_t mi = flag_mask<6>(x), mr = flag_mask<5>(x);
                uint32_t v4[4];
#pragma unroll
                for (uint32_t t2 = 0; t2 < 4; ++t2) v4[t2] = bsel(mi, wv[2 * t2 + 1], wv[2 * t2]);
                const uint32_t w0 = bsel(mr, v4[1], v4[0]), w1 = bsel(mr, v4[2], v4[1]), w2 = bsel(mr, v4[3], v4[2]);
                const uint32_t hlo = __builtin_amdgcn_alignbit(w1, w0, x) & Ulo;
                const uint32_t hhi = __builtin_amdgcn_alignbit(w2, w1, x) & Uhi;
                if constexpr (PB == 1) {
                    // bulk: only the unresolved mask and the key of the last hit
                    lastkey = (hlo | hhi) != 0u ? gs[u] << 16 : lastkey;
                    Ulo ^= hlo;
                    Uhi ^= hhi;
                    continue;
                }
                pcs[u] = __popc(hlo) + __popc(hhi);
                if (pcs[u] != 0u) {
                    const uint32_t pc = pcs[u];
                    sumg = mad_lo16(gs[u], pc, sumg);
                    s0 += (unsigned long long)gs[u] * hlo;
                    s1 += (unsigned long long)gs[u] * hhi;
                    lastkey = gs[u] << 16;
                    if constexpr (PB != 0) {
                        if (a.pmin) {
                            const uint32_t p = 131071u - 2u * gs[u];
                            unsigned long long hb = ((unsigned long long)hhi << 32) | hlo;
                            while (hb) {
                                store_p<PB>(a.pmin, ob + 3ull * (unsigned long long)__builtin_ctzll(hb), p);
                                hb &= hb - 1ull;
                            }
                        }
                    }
                    Ulo ^= hlo;
                    Uhi ^= hhi;
                }
            }
            if constexpr (PB != 1) {
                lds_u64 *lh2 = reinterpret_cast<lds_u64 *>(static_cast<uintptr_t>(ka + 32u));
                const unsigned long long c01 = (unsigned long long)pcs[0] | ((unsigned long long)pcs[1] << 32);
                const unsigned long long c23 = (unsigned long long)pcs[2] | ((unsigned long long)pcs[3] << 32);
                if (c01 != 0ull) __hip_atomic_fetch_add(&lh2[0], c01, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (c23 != 0ull) __hip_atomic_fetch_add(&lh2[1], c23, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            ka += 48u;
        }
        // lanes that finish a block take the next blocks of their wave's
        // chunk; a wave whose chunk runs short takes a new one of kChunk
        // blocks (at least 64, so that one refill serves every lane)
        const unsigned long long dm =
            __builtin_amdgcn_uicmp(Ulo | Uhi, 0u, 32) | __builtin_amdgcn_uicmp(ka, ka_end, 35);  // ==, >=
        if (dm != 0ull) {
            const uint32_t cn2 = (uint32_t)__popcll(dm);
            const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(dm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)dm, 0u));
            uint32_t nb = c_next + r;
            if (c_end - c_next >= cn2) {
                c_next += cn2;
            } else {
                const uint32_t rm = c_end - c_next;
                const uint32_t leader = (uint32_t)__builtin_ctzll(dm);
                uint32_t cn = 0;
                if (lane == leader) {
                    uint32_t na = (uint32_t)(uintptr_t)(lds_u32 *)L.next;
                    asm volatile("" : "+v"(na));
                    cn = __hip_atomic_fetch_add(reinterpret_cast<lds_u32 *>(static_cast<uintptr_t>(na)), kChunk,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                cn = __builtin_amdgcn_readlane(cn, leader);
                nb = r < rm ? nb : cn + (r - rm);
                c_next = cn + (cn2 - rm);
                c_end = cn + kChunk;
            }
            if ((Ulo | Uhi) == 0u || ka >= ka_end) {
                accbg += (unsigned long long)(long long)((int)b - (int)nb) * sumg;
                minkey = min(minkey, lastkey | (b / 3u));
                if (Ulo | Uhi) push_unresolved(b, Ulo, Uhi);
                b = nb;
                if (b < nblk) {
                    set_block(b);
                    if (__builtin_amdgcn_ballot_w64(b < bmask_lo || b >= bmask_hi || first0 || ka == ka_end) != 0ull) {
                        if (b < bmask_lo || b >= bmask_hi || first0) edge_block(b);
                        if (ka == ka_end) empty_list(b);
                    }
                }
            }
        }
    }

    // ---- tile summary ------------------------------------------------------
    // The checksum of the resolved n as in the consecutive-n kernel, with the
    // block weight b(n) = N0/128 + block index; threads 0..5 remove the n the
    // blocks of the first and last stretch do not hold (deficits), and
    // thread 0 adds the special n explicitly.
    if (tid < 6u) {
        const uint32_t bb = tid < 3u ? tid : nblk - 6u + tid;
        if (bb < nblk && (tid < 3u || bb >= 3u)) {
            uint32_t mlo, mhi;
            block_mask(bb, mlo, mhi);
            deficit(bb, ~mlo, ~mhi);
        }
    }
    accbg += (unsigned long long)b * sumg;
    unsigned long long ysum = 0ull - 2ull * ((N0 >> 7) * sumg + accbg);
    unsigned long long zsum = (0ull - 2ull * s0) + 3ull * (0ull - 2ull * s1);
    if (tid == 0u) {
        const unsigned long long nb = nblk;
        const unsigned long long sum_b = nb * (N0 >> 7) + nb * (nb - 1ull) / 2ull;
        ysum += 131071ull * 64ull * sum_b;
        zsum += 4ull * 131071ull * (nb * 0xFFFFFFFFull);
        // n = 4: b = 2, j = 0, weight 2^34 + 1; n = 6: b = 0, j = 1, weight 2
        const uint32_t sp4 = special_p(2u), sp6 = special_p(0u);
        if (sp4) {
            ysum += 2ull * sp4;
            zsum += sp4;
        }
        if (sp6) zsum += 2ull * sp6;
    }
    const unsigned long long cs = (ysum << 33) + zsum;
    const uint32_t gmax = minkey >> 16, mK0 = minkey & 0xFFFFu;
    const uint32_t maxp = minkey == 0xFFFFFFFFu ? 0u : (gmax == 0xFFFFu ? 2u : 131071u - 2u * gmax);
    const unsigned long long key = ((unsigned long long)maxp << 32) | (0xFFFFFFFFu - mK0);
    if (cs) atomicAdd(&L.red[0], cs);
    if (maxp) atomicMax(&L.red[2], key);
    __syncthreads();
    if (wave == 0) {
        const unsigned long long csum = L.red[0] + ((0ull - 131071ull * L.red[4]) << 33) +
                                        (0ull - 131071ull * L.red[5]) + 3ull * (0ull - 131071ull * L.red[6]);
        const unsigned long long kmax = L.red[2];
        const uint32_t mp = (uint32_t)(kmax >> 32);
        const uint32_t mK = 0xFFFFFFFFu - (uint32_t)(kmax & 0xFFFFFFFFu);
        // smallest n of stretch mK with p_min = mp: in each class a whose list
        // holds mp, the n of the block that mp hits and no smaller listed
        // prime does
        uint32_t am = 0xFFFFFFFFu;
        if (mp != 0u) {
            const uint32_t gmp = 65536u - (mp + 1u) / 2u;
            const uint32_t bwm = base_a + 16u * mK;
            for (uint32_t ai = 0; ai < 3u; ++ai) {
                const uint32_t first = L.cls[3u * ai] / 4u, groups = L.cls[3u * ai + 1u];
                const uint32_t *rec = L.cls + GB_CLS_HDR + first;
                uint32_t olo = 0, ohi = 0;
                for (uint32_t e = lane; e < 4u * groups; e += 64u) {
                    const uint32_t wo = 12u * (e >> 2) + (e & 3u);
                    if (rec[wo + 4u] > gmp) {
                        const uint32_t x = rec[wo];
                        const uint32_t wa = bwm + (x >> 16) + 8u * ((x >> 5) & 1u) + 4u * ((x >> 6) & 1u);
                        const lds_u32 *wq = reinterpret_cast<const lds_u32 *>(static_cast<uintptr_t>(wa));
                        olo |= __builtin_amdgcn_alignbit(wq[2], wq[0], x);
                        ohi |= __builtin_amdgcn_alignbit(wq[4], wq[2], x);
                    }
                }
                if (olo) atomicOr(&L.orw[2u * ai], olo);
                if (ohi) atomicOr(&L.orw[2u * ai + 1u], ohi);
            }
            __builtin_amdgcn_wave_barrier();
            if (lane < 3u) {
                const uint32_t ai = lane, a2 = 2u * ai;
                const uint32_t bb = 3u * mK + ai;
                uint32_t cand = 0xFFFFFFFFu;
                if (special_p(bb) == mp) cand = bb == 2u ? 4u : 6u;
                const uint32_t c = (a2 + 6u - mp % 6u) % 6u;
                if (cand == 0xFFFFFFFFu && (c == 1u || c == 5u)) {
                    uint32_t mlo, mhi;
                    block_mask(bb, mlo, mhi);
                    const uint32_t d = (mp - a2 + c) / 6u;
                    const uint32_t s = Hk + 64u * mK - d, pi = c == 5u ? 1u : 0u;
                    const lds_u32 *wq = reinterpret_cast<const lds_u32 *>(static_cast<uintptr_t>(base_a + plane_off(s, pi)));
                    const uint32_t hlo = __builtin_amdgcn_alignbit(wq[2], wq[0], s) & mlo & ~L.orw[2u * ai];
                    const uint32_t hhi = __builtin_amdgcn_alignbit(wq[4], wq[2], s) & mhi & ~L.orw[2u * ai + 1u];
                    if (hlo | hhi) {
                        const uint32_t j = hlo ? (uint32_t)__builtin_ctz(hlo) : 32u + (uint32_t)__builtin_ctz(hhi);
                        cand = 384u * mK + 6u * j + a2;
                    }
                }
                if (cand != 0xFFFFFFFFu) atomicMin(&L.orw[6], cand);
            }
            __builtin_amdgcn_wave_barrier();
            am = L.orw[6];
        }
        if (lane == 0) {
            unsigned long long *C = L.carry;
            if (C[CY_SLOT] != slot) {
                flush_slot(a, C);
                C[CY_COUNT] = C[CY_SUM] = C[CY_EXH] = C[CY_MAXP] = 0ull;
                C[CY_ARGN] = ~0ull;
                C[CY_SLOT] = slot;
            }
            C[CY_COUNT] += cnt - lead;
            C[CY_SUM] += csum;
            const unsigned long long an = N0 + am;
            if (mp != 0u && am != 0xFFFFFFFFu && (mp > C[CY_MAXP] || (mp == C[CY_MAXP] && an < C[CY_ARGN]))) {
                C[CY_MAXP] = mp;
                C[CY_ARGN] = an;
            }
        }
    }
    __syncthreads();
    }
}

template <int NT, int PB, bool PERS, bool SIEVE_ONLY>
__global__ __launch_bounds__(NT) void k_cls(GbTileArgs a)
{
    extern __shared__ uint32_t smem[];
    const ClsLds L = carve_cls(smem, a);
    HistCarry hc;
    // the class headers and probe records (hit counts zero), once
    for (uint32_t i = threadIdx.x; i < a.cls_words; i += NT) L.cls[i] = a.cls[i];
    if (threadIdx.x == 0) L.carry[CY_SLOT] = kNoSlot;
    if constexpr (PERS) {
        // the workgroup's share of the first static_tiles tiles, then the
        // queue (one device-scope atomic per tile taken from it)
        __syncthreads();
        for (unsigned long long g = blockIdx.x; g < a.static_tiles && g < a.ntiles; g += gridDim.x)
            cls_tile<NT, PB, SIEVE_ONLY>(a, g, L, hc);
        for (;;) {
            if (threadIdx.x == 0) *L.tile = a.static_tiles + atomicAdd(a.queue, 1ull);
            __syncthreads();
            const unsigned long long g = *L.tile;
            if (g >= a.ntiles) break;
            cls_tile<NT, PB, SIEVE_ONLY>(a, g, L, hc);
        }
    } else {
        __syncthreads();
        cls_tile<NT, PB, SIEVE_ONLY>(a, a.tile0 + blockIdx.x, L, hc);
    }
    if constexpr (!SIEVE_ONLY) {
        if (hc.row != kNoRow) flush_hist_cls(a, L, hc.row, hc);
        // a row that holds nothing of this launch is marked so
        if (a.wg_hist != nullptr && !hc.stored && threadIdx.x == 0)
            a.wg_hist[(unsigned long long)blockIdx.x * a.wg_hist_stride] = kNoRow;
        if (threadIdx.x == 0) flush_slot(a, L.carry);
    }
}

template <int NT, int PB, bool PERS, bool SO>
hipError_t launch_cls_one(const GbTileArgs &a, uint32_t grid, size_t lds, hipStream_t st)
{
    hipLaunchKernelGGL((k_cls<NT, PB, PERS, SO>), dim3(grid), dim3(NT), lds, st, a);
    return hipGetLastError();
}

template <int NT, int PB, bool PERS, bool SO>
hipError_t allow_cls(size_t lds)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_cls<NT, PB, PERS, SO>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int NT>
hipError_t allow_cls_nt(size_t lds)
{
    hipError_t e = hipSuccess, r;
    if ((r = allow_cls<NT, 0, false, true>(lds)) != hipSuccess) e = r;
    if ((r = allow_cls<NT, 0, true, false>(lds)) != hipSuccess) e = r;
    if ((r = allow_cls<NT, 1, true, false>(lds)) != hipSuccess) e = r;
    if ((r = allow_cls<NT, 1, false, false>(lds)) != hipSuccess) e = r;
    if ((r = allow_cls<NT, 16, true, false>(lds)) != hipSuccess) e = r;
    if ((r = allow_cls<NT, 32, true, false>(lds)) != hipSuccess) e = r;
    if ((r = allow_cls<NT, 0, false, false>(lds)) != hipSuccess) e = r;
    if ((r = allow_cls<NT, 16, false, false>(lds)) != hipSuccess) e = r;
    if ((r = allow_cls<NT, 32, false, false>(lds)) != hipSuccess) e = r;
    return e;
}

template <int NT>
hipError_t launch_cls_nt(const GbTileArgs &a, uint32_t grid, size_t lds, int pb, bool pers, bool so, hipStream_t st)
{
    if (so) return launch_cls_one<NT, 0, false, true>(a, grid, lds, st);
    if (pers) {
        if (pb == 1) return launch_cls_one<NT, 1, true, false>(a, grid, lds, st);
        if (pb == 16) return launch_cls_one<NT, 16, true, false>(a, grid, lds, st);
        if (pb == 32) return launch_cls_one<NT, 32, true, false>(a, grid, lds, st);
        return launch_cls_one<NT, 0, true, false>(a, grid, lds, st);
    }
    if (pb == 1) return launch_cls_one<NT, 1, false, false>(a, grid, lds, st);
    if (pb == 16) return launch_cls_one<NT, 16, false, false>(a, grid, lds, st);
    if (pb == 32) return launch_cls_one<NT, 32, false, false>(a, grid, lds, st);
    return launch_cls_one<NT, 0, false, false>(a, grid, lds, st);
}

}  // namespace

size_t gb_cls_lds_bytes(uint32_t sb_per_tile, uint32_t hk, uint32_t cls_words)
{
    // the same carve-up as carve_cls()
    size_t words = 2 * ((size_t)(hk + 64 * sb_per_tile) / 32 + 4);
    words = (words + 3) & ~(size_t)3;
    words += cls_words;
    words = (words + 1) & ~(size_t)1;
    words += 2 * 7 + 2 * 6 + 2 + 2 + 7;
    return words * 4;
}

hipError_t gb_cls_prepare(uint32_t threads, size_t lds_bytes)
{
    switch (threads) {
    case 256: return allow_cls_nt<256>(lds_bytes);
    case 512: return allow_cls_nt<512>(lds_bytes);
    case 1024: return allow_cls_nt<1024>(lds_bytes);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gb_cls_occupancy(uint32_t threads, size_t lds_bytes, int *blocks_per_cu)
{
    switch (threads) {
    case 256: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_cls<256, 0, true, false>, 256, lds_bytes);
    case 512: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_cls<512, 0, true, false>, 512, lds_bytes);
    case 1024: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_cls<1024, 0, true, false>, 1024, lds_bytes);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gb_launch_cls(const GbTileArgs &a, uint32_t grid, uint32_t threads, size_t lds_bytes, int pmin_bits,
                         bool persistent, bool sieve_only, hipStream_t st)
{
    if (grid == 0) return hipSuccess;
    switch (threads) {
    case 256: return launch_cls_nt<256>(a, grid, lds_bytes, pmin_bits, persistent, sieve_only, st);
    case 512: return launch_cls_nt<512>(a, grid, lds_bytes, pmin_bits, persistent, sieve_only, st);
    case 1024: return launch_cls_nt<1024>(a, grid, lds_bytes, pmin_bits, persistent, sieve_only, st);
    default: return hipErrorInvalidValue;
    }
}
