// gb_kernels.hip -- HIP kernels (gfx950, wave64) of the segmented Goldbach
// verifier.
//
// k_tile: one workgroup owns one tile of T consecutive even n, n = N0 + 2j.
// It sieves the odd numbers w0 + 2i, w0 = N0 + 1 - 2*HB, 0 <= i < T + HB, into
// an LDS bitset (bit = 1 for a prime), then runs the paper's inverted loop
// (section "Segmented Double-Sieve Verifier", subsection "Correct
// segmentation": iterate over candidate primes p and mark the n for which
// n - p is prime) on it: for a fixed p the bits of q = n - p for the 64 even n
// of one block n0, n0+2, ..., n0+126 are 64 consecutive bits of the window,
// starting at bit j0 + HB - (p+1)/2, so one 64-bit funnel extract ANDed with
// the block's mask of still-unresolved n probes 64 n at once.  Primes are
// taken in ascending order, so the first p that hits an n is p_min(n).
// The halo HB >= (P_max+1)/2 keeps every q = n - p with p <= P_max inside
// the window, which is the paper's three-way primality oracle (small-prime
// table, segment bitset, Miller-Rabin) collapsed into one lookup.
// n that no p <= P_max resolves go to a device list for k_mr, the
// exhaustive phase (the paper's Phase 2; on the GPU here).
// A hit (prime p, mask h of the n it settles) costs a popcount for the
// per-prime histogram and three multiply-adds for the checksum; a block only
// remembers the p of its last hit, which is its largest p_min, and the tile
// recovers the smallest n with the tile's largest p_min at its end.
//
// k_mr: one wavefront per listed n.  Lane l takes the l-th next candidate
// prime p, screens q = n - p with a base-2 strong probable-prime test in
// Montgomery arithmetic, and the lowest passing lane (ballot + first set bit)
// is confirmed with the other eleven bases of the deterministic 64-bit test
// (bases 2..37), one base per lane.
#include <algorithm>
#include <type_traits>

#include "gb_internal.h"
#include "gb_device.h"

namespace {

__device__ __forceinline__ unsigned long long fastmod64(unsigned long long x, uint32_t p,
                                                        unsigned long long magic)
{
    // magic = floor((2^64-1)/p) underestimates 2^64/p by less than 1, so the
    // quotient estimate is floor(x/p) or one less: one correction step.
    unsigned long long q = __umul64hi(x, magic);
    unsigned long long r = x - q * (unsigned long long)p;
    return r >= p ? r - p : r;
}

// Smallest bit index t >= 0 such that w0 + 2t is an odd multiple of p and at
// least p*p (the first composite the prime p strikes in the window).
__device__ __forceinline__ unsigned long long first_index(long long w0, uint32_t p,
                                                          unsigned long long magic)
{
    unsigned long long pp = (unsigned long long)p * p;
    if (w0 <= 0 || (unsigned long long)w0 <= pp)
        return (pp - (unsigned long long)w0) >> 1;
    unsigned long long r = fastmod64((unsigned long long)w0, p, magic);
    uint32_t d = r ? p - (uint32_t)r : 0u;  // w0 + d is the next multiple
    return (d & 1u) ? ((unsigned long long)d + p) >> 1 : (unsigned long long)(d >> 1);
}

// Same as first_index when p*p <= w0 < 2^53, from the prime alone.  With
// b = 2p and y = w0 - p the gap to the next odd multiple of p is
// d = ceil(y/b)*b - y.  The reciprocal of b is the hardware estimate refined
// by two Newton steps (relative error near 2^-52), so the quotient y/b < 2^52
// is off by less than one and ceil() by at most one either way; the FMA
// residual is an exact small integer, corrected once in each direction.
__device__ __forceinline__ uint32_t first_index_rcp(double w0d, uint32_t p)
{
    const double pd = (double)p;
    const double b = pd + pd;
    double x = __builtin_amdgcn_rcp(b);
    x = fma(x, fma(-b, x, 1.0), x);
    x = fma(x, fma(-b, x, 1.0), x);
    const double y = w0d - pd;
    const double q = ceil(y * x);
    int d = (int)fma(q, b, -y);
    const int b2 = (int)(2u * p);
    if (d < 0) d += b2;
    if (d >= b2) d -= b2;
    return (uint32_t)d >> 1;
}

// Bit 16 of x copied to all 32 bits (v_bfe_i32).
__device__ __forceinline__ uint32_t sext_bit16(uint32_t x)
{
    uint32_t d;
    asm("v_bfe_i32 %0, %1, 16, 1" : "=v"(d) : "v"(x));
    return d;
}

// (m & a) | (~m & b) in one v_bfi_b32.
__device__ __forceinline__ uint32_t bitsel(uint32_t m, uint32_t a, uint32_t b)
{
    uint32_t d;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(d) : "v"(m), "v"(a), "v"(b));
    return d;
}

// Clear the bits of m's zeros in the LDS word at byte address addr.
__device__ __forceinline__ void lds_and(uint32_t addr, uint32_t m)
{
    __hip_atomic_fetch_and(reinterpret_cast<lds_u32 *>(static_cast<uintptr_t>(addr)), m, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Packed word of a fast-path prime p, h = (p+1)/2: bits 15..0 hold
// g = 2^16 - h, so bits 4..0 are the funnel shift (-h) mod 32 of a probe and
// p = 2^17 - 1 - 2g; bits 31..16 hold PX_BIAS - 4 ceil(h/32), the byte offset
// of the probe's first word below the block's base word, biased to be >= 0.
constexpr uint32_t PX_BIAS = 4096;   // 4 ceil(h/32) <= 4096 for h <= 32768

// Checksum weight of an even n: 2^33 b + (2c+1) 2^i with
// b = 3 floor(n/384) + (n mod 6)/2 (the index of n's block of 64 n of one
// class mod 6 in the minimal-p search) and floor(n/6) mod 64 = 32c + i (n's
// bit in it).  The checksum is the sum of weight * p_min mod 2^64; it is
// not in the paper, and this form is the one the bit-sliced search
// accumulates with two 32x32 -> 64-bit multiply-adds per hit.
__device__ __forceinline__ unsigned long long checksum_weight(unsigned long long n)
{
    const unsigned long long k = n / 6ull;
    const uint32_t j = (uint32_t)k & 63u;
    const unsigned long long b = 3ull * (k >> 6) + (n - 6ull * k) / 2ull;
    return (b << 33) + ((unsigned long long)(2u * (j >> 5) + 1u) << (j & 31u));
}

__device__ __forceinline__ bool is_wheel_prime(long long v, uint32_t wmax)
{
    return v <= (long long)wmax &&
           (v == 3 || v == 5 || v == 7 || v == 11 || v == 13 || v == 17 || v == 19);
}

// Word offsets of prime i's packed word, g and hit count in TileLds::pr.
__device__ __forceinline__ uint32_t pr_px(uint32_t i) { return 12u * (i >> 2) + (i & 3u); }
__device__ __forceinline__ uint32_t pr_gl(uint32_t i) { return pr_px(i) + 4u; }
__device__ __forceinline__ uint32_t pr_lh(uint32_t i) { return pr_px(i) + 8u; }

// LDS carve-up of one tile workgroup (offsets in 32-bit words).
struct TileLds {
    uint32_t *bits;           // (T + HB)/32 words: the tile's window, 1 = prime
    // odd primes p <= P_max (padded with copies of the last through two more
    // groups) in groups of
    // four, 12 words per group: the four packed words, the four g =
    // 2^16 - (p+1)/2, the four hit counts of this tile
    uint32_t *pr;
    uint32_t *offs;           // first bit index (or ~0) of each small/medium sieving prime
    unsigned long long *red;  // 7: checksum, n_exhaustive, max key, OR words,
                              // deficits (floor(n/128), 2^i of half 0, half 1)
    // the slot summaries of the workgroup's current run of tiles of one slot
    // (thread 0 only): count, checksum, n_exhaustive, argmax n, slot, max p
    unsigned long long *carry;
    unsigned long long *tile; // persistent mode: the tile just taken
    uint32_t *next;           // next block of the tile to hand out
};

__device__ __forceinline__ TileLds carve(uint32_t *smem, const GbTileArgs &a)
{
    TileLds L;
    uint32_t o = 0;
    L.bits = smem + o;
    o += (a.tile_n + a.halo_bits) / 32;
    o = (o + 3) & ~3u;   // 16-byte aligned: a group reads its four words at once
    L.pr = smem + o;
    o += 12u * ((a.np_search + 3u) / 4u + 2u);
    L.offs = smem + o;
    o += a.n_off;
    o = (o + 1) & ~1u;
    L.red = reinterpret_cast<unsigned long long *>(smem + o);
    o += 2 * 7;
    L.carry = reinterpret_cast<unsigned long long *>(smem + o);
    o += 2 * 6;
    o = (o + 1) & ~1u;
    L.tile = reinterpret_cast<unsigned long long *>(smem + o);
    o += 2;
    L.next = smem + o;
    return L;
}

// Fast-path prime list in LDS, once per workgroup: odd primes p <= P_max in
// groups of four (packed words, g, hit counts), padded with copies of the last
// prime through the end of the second group after the last prime's group (a
// lane runs three groups per exit check and may start on the last one).
template <int NT, bool VERIFY, bool GW>
__device__ void setup_primes(const GbTileArgs &a, const TileLds &L)
{
    const uint32_t nps = a.np_search;
    const uint32_t npad = 4u * ((nps + 3u) / 4u + 2u);
    for (uint32_t i = threadIdx.x; i < npad; i += NT) {
        const uint32_t p = a.primes[i < nps ? i : (nps ? nps - 1 : 0)];
        const uint32_t h = (p + 1u) >> 1;
        uint32_t hi = PX_BIAS - 4u * ((h + 31u) >> 5);
        if (GW && (i & 3u) != 3u) {
            // group-window form: the high half of a group's first three
            // words says whether the probe starts one word above the
            // group's base word (that of its last prime)
            const uint32_t i3 = i | 3u;
            const uint32_t p3 = a.primes[i3 < nps ? i3 : (nps ? nps - 1 : 0)];
            hi = ((((p3 + 1u) >> 1) + 31u) >> 5) - ((h + 31u) >> 5);
        }
        L.pr[pr_px(i)] = (hi << 16) | (65536u - h);
        L.pr[pr_gl(i)] = VERIFY ? (65536u - h) << 16 : 65536u - h;
        L.pr[pr_lh(i)] = 0;
    }
}

// Add the workgroup's per-prime hit counts to histogram row `row` and clear
// them (each thread its own primes).
__device__ void flush_hist(const GbTileArgs &a, const TileLds &L, uint32_t row)
{
    unsigned long long *hist = a.hist + (unsigned long long)row * GB_HIST_BINS_I;
    for (uint32_t i = threadIdx.x; i < a.np_search; i += blockDim.x) {
        const uint32_t c = L.pr[pr_lh(i)];
        if (c) {
            atomicAdd(&hist[i + 1], (unsigned long long)c);
            L.pr[pr_lh(i)] = 0;
        }
    }
}

template <int NT, int PB, bool SIEVE_ONLY, bool GW>
__device__ void process_tile(const GbTileArgs &a, unsigned long long g, const TileLds &L, HistCarry &hc)
{
    // made opaque per tile: otherwise the compiler hoists values derived
    // from the thread index out of a persistent workgroup's tile loop and
    // keeps them live in registers across it (87 instead of 49 VGPRs)
    // PB == 1: bulk verification (section "Discussion": the verified set as
    // a bitset that each prime's shifted window is OR-ed into); no per-n
    // output, histogram or checksum, only count, max p_min and its n,
    // n_exhaustive and failures
    constexpr bool VERIFY = PB == 1;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    constexpr uint32_t NWAVES = NT / 64;

    // ---- locate the tile's window ----------------------------------------
    uint32_t wi = 0;
    if (a.nwin > 1) {
        uint32_t lo = 0, hi = a.nwin - 1;
        while (lo < hi) {
            uint32_t mid = (lo + hi + 1) >> 1;
            if (a.win[mid].tile_base <= g) lo = mid; else hi = mid - 1;
        }
        wi = lo;
    }
    const GbWindow W = a.win[wi];
    const unsigned long long t = g - W.tile_base;
    const unsigned long long N0 = W.first_n + 2ull * a.tile_n * t;
    const unsigned long long rem = W.count - (unsigned long long)a.tile_n * t;
    const uint32_t cnt = rem < a.tile_n ? (uint32_t)rem : a.tile_n;
    const uint32_t nblk = (cnt + 63u) >> 6;
    const uint32_t HB = a.halo_bits;
    const uint32_t nbits = nblk * 64u + HB;
    const uint32_t nw32 = nbits >> 5;
    const long long w0 = (long long)(N0 + 1ull - 2ull * HB);
    const uint32_t np = W.np_sieve;
    const uint32_t nps = a.np_search;
    const bool small_w0 = w0 < (1ll << 53);   // exact as a double
    const double w0d = (double)w0;

    // ---- per-tile reductions; the workgroup's histogram row ----------------
    if (!SIEVE_ONLY) {
        if (tid < 7) L.red[tid] = 0ull;   // tile sums, max key, OR words, deficits
        if (tid == 0) *L.next = NT;       // blocks 0..NT-1 go to the threads in order
        // The per-prime hit counts in L.pr stay in LDS across the tiles of a
        // workgroup and go to the histogram when its row changes (one row per
        // window with per-slot histograms), before 2^31 n could overflow a
        // 32-bit count, and when the workgroup ends.  Each thread flushes and
        // clears its own primes' counts; the counts are next written in the
        // search phase, behind the sieve's barriers.
        if (!VERIFY) {
            const uint32_t row = a.hist_per_slot ? W.slot : 0u;
            if (row != hc.row || hc.n + cnt > 0x7FFFFFFFull) {
                if (hc.row != kNoRow) flush_hist(a, L, hc.row);
                hc.row = row;
                hc.n = 0;
            }
            hc.n += cnt;
        }
    }
    // ---- first strike of every small and medium sieving prime, once -------
    // When the window starts at or above the square of its largest sieving
    // prime (and below 2^53) every first strike comes from the prime alone
    // (first_index_rcp); otherwise from the 64-bit reciprocal table.  Each
    // lane loads its next prime ahead.
    const uint32_t kmid = min(a.k_wave_end, np);
    const uint32_t ptop = np ? a.primes[np - 1] : 0u;
    const bool fast = small_w0 && w0 >= (long long)((unsigned long long)ptop * ptop);
    auto strikes = [&](auto fast_c) {
        constexpr bool FAST = decltype(fast_c)::value;
        uint32_t k = a.k_first + tid;
        uint32_t pn = 0;
        unsigned long long mn = 0;
        if (k < kmid) {
            pn = a.primes[k];
            if (!FAST) mn = a.magic[k];
        }
        for (; k < kmid; k += NT) {
            const uint32_t p = pn;
            const unsigned long long mg = mn;
            if (k + NT < kmid) {
                pn = a.primes[k + NT];
                if (!FAST) mn = a.magic[k + NT];
            }
            const unsigned long long t0 = FAST ? first_index_rcp(w0d, p) : first_index(w0, p, mg);
            L.offs[k - a.k_first] = t0 < nbits ? (uint32_t)t0 : 0xFFFFFFFFu;
        }
    };
    if (fast) strikes(std::true_type{}); else strikes(std::false_type{});

    // ---- wheel pre-pattern: clears the odd multiples of 3..wheel_max ------
    // Pattern bit g is 1 iff 2g+1 is coprime to every wheel prime; tile bit i
    // (value w0 + 2i) has pattern phase ((w0-1)/2 + i) mod wheel_len.  The
    // pattern words of a lane's next word are loaded ahead.
    {
        const uint32_t Lw = a.wheel_len;
        const uint32_t g0 = (uint32_t)(((N0 >> 1) % Lw + Lw - (HB % Lw)) % Lw);
        uint32_t ph = (g0 + 32u * tid) % Lw;
        const uint32_t step = (32u * NT) % Lw;
        uint32_t lo = 0, hi = 0;
        if (tid < nw32) {
            lo = a.wheel[ph >> 5];
            hi = a.wheel[(ph >> 5) + 1];
        }
        for (uint32_t i = tid; i < nw32; i += NT) {
            uint32_t v = __builtin_amdgcn_alignbit(hi, lo, ph & 31u);
            ph += step;
            if (ph >= Lw) ph -= Lw;
            if (i + NT < nw32) {
                lo = a.wheel[ph >> 5];
                hi = a.wheel[(ph >> 5) + 1];
            }
            const long long vfirst = w0 + 64ll * i;
            if (vfirst <= (long long)a.wheel_max) {
                // the window reaches the wheel primes themselves, or 1 and below
                // (a rare path: kept rolled so it holds no registers elsewhere)
#pragma unroll 1
                for (uint32_t bt = 0; bt < 32; ++bt) {
                    const long long val = vfirst + 2ll * bt;
                    if (val < 2) v &= ~(1u << bt);
                    else if (is_wheel_prime(val, a.wheel_max)) v |= (1u << bt);
                }
            }
            L.bits[i] = v;
        }
    }
    __syncthreads();

    // ---- strided marking of the odd multiples of each sieving prime -------
    {
        // LDS byte address of the window, made opaque to the compiler so
        // that the loops step one address instead of re-adding the base
        uint32_t bits_a = (uint32_t)(uintptr_t)(lds_u32 *)L.bits;
        asm volatile("" : "+s"(bits_a));
        const uint32_t end_a = bits_a + 4u * nw32;   // nbits = 32 * nw32
        // primes with many hits per tile: the whole workgroup strides over
        // one prime; the stride NT*p is a multiple of 32 bits, so the bit
        // within the word stays put and only the word address moves
        // (the next prime and its first strike are read ahead)
        const uint32_t kend = min(a.k_wg_end, np);
        if (a.k_first < kend) {
            uint32_t t0 = L.offs[0], p = a.primes[a.k_first];
            for (uint32_t k = a.k_first; k < kend; ++k) {
                const uint32_t kn = min(k + 1u, kend - 1u);
                const uint32_t t0n = L.offs[kn - a.k_first], pn = a.primes[kn];
                const uint32_t idx = t0 + tid * p;
                if (t0 != 0xFFFFFFFFu && idx < nbits) {
                    const uint32_t m = ~(1u << (idx & 31u));
                    const uint32_t stride = (NT / 8u) * p;
                    for (uint32_t wa = bits_a + 4u * (idx >> 5); wa < end_a; wa += stride) lds_and(wa, m);
                }
                t0 = t0n;
                p = pn;
            }
        }
        // medium primes: one wavefront per prime, lanes stride by 64p bits
        const uint32_t kbeg2 = max(a.k_wg_end, a.k_first);
        if (kbeg2 + wave < kmid) {
            uint32_t t0 = L.offs[kbeg2 + wave - a.k_first], p = a.primes[kbeg2 + wave];
            for (uint32_t k = kbeg2 + wave; k < kmid; k += NWAVES) {
                const uint32_t kn = min(k + NWAVES, kmid - 1u);
                const uint32_t t0n = L.offs[kn - a.k_first], pn = a.primes[kn];
                const uint32_t idx = t0 + lane * p;
                if (t0 != 0xFFFFFFFFu && idx < nbits) {
                    const uint32_t m = ~(1u << (idx & 31u));
                    for (uint32_t wa = bits_a + 4u * (idx >> 5); wa < end_a; wa += 8u * p) lds_and(wa, m);
                }
                t0 = t0n;
                p = pn;
            }
        }
        // large primes: one lane per prime, a few hits each; the lane loads
        // its next prime ahead
        const uint32_t kbeg3 = max(a.k_wave_end, a.k_first);
        auto large = [&](auto fast_c) {
            constexpr bool FAST = decltype(fast_c)::value;
            uint32_t k = kbeg3 + tid;
            uint32_t pn = 0;
            unsigned long long mn = 0;
            if (k < np) {
                pn = a.primes[k];
                if (!FAST) mn = a.magic[k];
            }
            for (; k < np; k += NT) {
                const uint32_t p = pn;
                const unsigned long long mg = mn;
                if (k + NT < np) {
                    pn = a.primes[k + NT];
                    if (!FAST) mn = a.magic[k + NT];
                }
                const unsigned long long t0 = FAST ? first_index_rcp(w0d, p) : first_index(w0, p, mg);
                if (t0 >= nbits) continue;
                for (uint32_t idx = (uint32_t)t0; idx < nbits; idx += p)
                    lds_and(bits_a + 4u * (idx >> 5), ~(1u << (idx & 31u)));
            }
        };
        if (fast) large(std::true_type{}); else large(std::false_type{});
    }
    __syncthreads();

    if (SIEVE_ONLY) {
        // bitset dump: tile t owns output bits [T*t, T*t + cnt)
        const unsigned long long obase = (unsigned long long)a.tile_n * t / 32;
        for (uint32_t i = tid; i < cnt / 32; i += NT) a.sieve_out[obase + i] = L.bits[i];
        __syncthreads();
        return;
    }

    // ---- inverted-loop search, 64 even n per lane-block --------------------
    // Block bb of the tile holds n = N0 + 128 bb + 2j, 0 <= j < 64, as bit j
    // of a 64-bit mask.  Windows are planned with N0 a multiple of 128 (the
    // n below a window's first n are masked out), so j = (n/2) mod 64 and
    // floor(n/128) = N0/128 + bb for every n of the block.
    const uint32_t slot = W.slot;
    const uint32_t hrow = a.hist_per_slot ? slot : 0u;
    unsigned long long *hist = a.hist + (unsigned long long)hrow * GB_HIST_BINS_I;
    const uint32_t lead = t == 0 ? W.lead : 0u;
    // per-n output index of bit 0 of block 0 (wraps below zero when lead > 0)
    const unsigned long long outb = W.out_off - W.lead + (unsigned long long)a.tile_n * t;

    // valid n of the tile's first and last blocks
    const uint32_t first_lo = lead >= 32u ? 0u : ~0u << lead;
    const uint32_t first_hi = lead >= 32u ? ~0u << (lead - 32u) : ~0u;
    const uint32_t nv_last = cnt - 64u * (nblk - 1u);
    const uint32_t last_lo = nv_last >= 32 ? ~0u : ((1u << nv_last) - 1u);
    const uint32_t last_hi = nv_last >= 64 ? ~0u : (nv_last > 32 ? ((1u << (nv_last - 32)) - 1u) : 0u);
    const bool ragged = nv_last != 64u;
    // n = 4 = 2 + 2, the one even p_min, is settled apart from the search
    const bool has4 = N0 == 0ull && (first_lo & (nblk == 1u ? last_lo : ~0u) & 4u) != 0u;
    auto block_mask = [&](uint32_t bb, uint32_t &lo, uint32_t &hi) {
        lo = ~0u;
        hi = ~0u;
        if (bb == 0u) {
            lo &= first_lo;
            hi &= first_hi;
            if (N0 == 0ull) lo &= ~4u;
        }
        if (bb + 1u == nblk) {
            lo &= last_lo;
            hi &= last_hi;
        }
    };

    // Lane summaries.  A hit of the prime p = 2^17 - 1 - 2g on the mask h of
    // n is accumulated through g (the low half of the prime's packed word):
    //   sumg = sum of g * popcount(h), and accbg, the sum over the lane's
    //     blocks b of b times block b's part of sumg;
    //   s0, s1 = sum of g * (32-bit half c of h), exact in 64 bits.
    // At the tile's end these turn into the checksum of the n the search
    // resolved, with p = 2^17 - 1 - 2g, together with the n it did not
    // resolve (masked in front or behind, or left to the exhaustive phase):
    //   sum of floor(n/128), sum of 2^i per half (LDS atomics into red[4..6],
    //   a rare path, so they hold no registers in the search loop).
    // largest p_min of the lane and its first block, as the smallest key
    // (g << 16) | block over the blocks' last hits (g falls as p grows; the
    // key 0xFFFF << 16 stands for p = 2, and ~0 for no hit)
    uint32_t minkey = 0xFFFFFFFFu;
    // accbg telescopes: at the end of a block b followed by block b' it adds
    // (b - b') sumg, and after the last block b'' sumg, which sums b times
    // each block's part of sumg without a copy of sumg per block
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

    // n no fast-path prime resolves go to the exhaustive phase's list
    auto push_unresolved = [&](uint32_t blk, uint32_t ulo, uint32_t uhi) {
        deficit(blk, ulo, uhi);
        unsigned long long u = ((unsigned long long)uhi << 32) | ulo;
        atomicAdd(&L.red[1], (unsigned long long)__popcll(u));
        while (u) {
            const uint32_t j = (uint32_t)__builtin_ctzll(u);
            u &= u - 1ull;
            const unsigned long long e = atomicAdd(a.list_count, 1ull);
            if (e < a.list_cap) {
                GbExh x;
                x.n = N0 + 2ull * (64ull * blk + j);
                x.out_index = outb + 64ull * blk + j;
                x.slot = slot;
                x.start_k = nps;
                x.p = 0;
                a.list[e] = x;
            }
        }
    };

    // key (g << 16) of the last hit on block bb, found by searching it again
    // one prime at a time (bulk mode, for the rare blocks the fast path
    // leaves with unresolved n)
    auto last_hit_key = [&](uint32_t bb) -> uint32_t {
        uint32_t ulo, uhi;
        block_mask(bb, ulo, uhi);
        uint32_t key = (bb == 0u && has4) ? 0xFFFF0000u : 0xFFFFFFFFu;
        const uint32_t base = 64u * bb + HB;
        for (uint32_t kk = 0; kk < nps; ++kk) {
            const uint32_t g = L.pr[pr_px(kk)] & 0xFFFFu;
            const uint32_t s = base - (65536u - g);
            const uint32_t *wp = L.bits + (s >> 5);
            const uint32_t hlo = __builtin_amdgcn_alignbit(wp[1], wp[0], s) & ulo;
            const uint32_t hhi = __builtin_amdgcn_alignbit(wp[2], wp[1], s) & uhi;
            if (hlo | hhi) {
                key = g << 16;
                ulo ^= hlo;
                uhi ^= hhi;
            }
        }
        return key;
    };

    // block state: unresolved mask U, LDS byte address of the next group of
    // four primes (ka), LDS byte address of the block's base word minus
    // PX_BIAS (bw), g << 16 of the block's last hit (the last hit carries
    // the block's largest p_min)
    const uint32_t bits_addr = (uint32_t)(uintptr_t)(lds_u32 *)L.bits;
    const uint32_t pr_addr = (uint32_t)(uintptr_t)(lds_u32 *)L.pr;
    const uint32_t ka_end = pr_addr + 48u * ((nps + 3u) / 4u);
    uint32_t b = tid, ka = pr_addr, Ulo = 0, Uhi = 0, lastkey = 0xFFFFFFFFu;
    uint32_t bw = bits_addr + 8u * tid + HB / 8u - PX_BIAS;
    // Blocks are handed out in chunks of 64 that a wave holds in scalar
    // registers ([c_next, c_end)); its lanes start on blocks tid, and the
    // workgroup counter hands out the chunks from NT on.
    uint32_t c_next = 0, c_end = 0;
    if (b < nblk) {
        block_mask(b, Ulo, Uhi);
        if (b == 0u && has4) {
            lastkey = 0xFFFF0000u;    // p = 2
            if (!VERIFY) atomicAdd(&hist[0], 1ull);
            if (a.pmin) store_p<PB>(a.pmin, outb + 2u, 2u);
        }
    }
    while (b < nblk) {
        if (nps != 0u) {
            // twelve probes (three groups) per exit check, so that the
            // block-end work (hand-out and block set-up) runs a third as often
            // (four groups made the minimal-p form slower); the prime list is
            // padded with copies of its last prime, which cannot hit an n twice
            constexpr uint32_t kGroupsPerCheck = 3u;
#pragma unroll
            for (uint32_t gg = 0; gg < kGroupsPerCheck; ++gg) {
                // the group's twelve window words do not depend on the hits, so
                // they are all read before the first test
                const v4u32 xv = *reinterpret_cast<const lds_v4 *>(static_cast<uintptr_t>(ka));
                const uint32_t xs[4] = {xv.x, xv.y, xv.z, xv.w};
                uint32_t dw[4][3], pcs[4];
                if constexpr (GW) {
                    // the four windows lie in the four words from the base word
                    // of the group's last (largest) prime: two reads for the group
                    const lds_u32 *wp = probe_addr(xs[3], bw);
                    const uint32_t w0 = wp[0], w1 = wp[1], w2 = wp[2], w3 = wp[3];
#pragma unroll
                    for (uint32_t u = 0; u < 3; ++u) {
                        // all ones when the flag (bit 16) is set: one bit-field
                        // extract, then three bit-wise selects
                        const uint32_t m = sext_bit16(xs[u]);
                        dw[u][0] = bitsel(m, w1, w0);
                        dw[u][1] = bitsel(m, w2, w1);
                        dw[u][2] = bitsel(m, w3, w2);
                    }
                    dw[3][0] = w0;
                    dw[3][1] = w1;
                    dw[3][2] = w2;
                } else {
#pragma unroll
                    for (uint32_t u = 0; u < 4; ++u) {
                        const lds_u32 *wp = probe_addr(xs[u], bw);
                        dw[u][0] = wp[0];
                        dw[u][1] = wp[1];
                        dw[u][2] = wp[2];
                    }
                }
                // the group's four g with one 16-byte read up front (otherwise
                // the compiler sinks single reads into the hit branches)
                v4u32 gv = *reinterpret_cast<const lds_v4 *>(static_cast<uintptr_t>(ka + 16u));
                asm volatile("" : "+v"(gv.x), "+v"(gv.y), "+v"(gv.z), "+v"(gv.w));
                const uint32_t gs[4] = {gv.x, gv.y, gv.z, gv.w};
                if constexpr (VERIFY) {
                    // every n the prime resolves leaves U; the last probe that
                    // starts on a nonempty U is the one that empties it, i.e. the
                    // block's last hit (when the block resolves completely)
#pragma unroll
                    for (uint32_t u = 0; u < 4; ++u) {
                        const uint32_t x = xs[u];
                        const uint32_t wlo = __builtin_amdgcn_alignbit(dw[u][1], dw[u][0], x);
                        const uint32_t whi = __builtin_amdgcn_alignbit(dw[u][2], dw[u][1], x);
                        lastkey = (Ulo | Uhi) != 0u ? gs[u] : lastkey;
                        Ulo &= ~wlo;
                        Uhi &= ~whi;
                    }
                } else {
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) {
                    const uint32_t x = xs[u];
                    const uint32_t hlo = __builtin_amdgcn_alignbit(dw[u][1], dw[u][0], x) & Ulo;
                    const uint32_t hhi = __builtin_amdgcn_alignbit(dw[u][2], dw[u][1], x) & Uhi;
                    pcs[u] = __popc(hlo) + __popc(hhi);
                    if (pcs[u] != 0u) {
                        const uint32_t pc = pcs[u];
                        sumg = mad_lo16(x, pc, sumg);
                        s0 += (unsigned long long)gs[u] * hlo;
                        s1 += (unsigned long long)gs[u] * hhi;
                        lastkey = x << 16;
                        if constexpr (PB != 0) {
                            if (a.pmin) {
                                const uint32_t p = 131071u - 2u * (x & 0xFFFFu);
                                unsigned long long hb = ((unsigned long long)hhi << 32) | hlo;
                                const unsigned long long ob = outb + 64ull * b;
                                while (hb) {
                                    store_p<PB>(a.pmin, ob + (unsigned long long)__builtin_ctzll(hb), p);
                                    hb &= hb - 1ull;
                                }
                            }
                        }
                        Ulo ^= hlo;
                        Uhi ^= hhi;
                    }
                }
                // the group's hit counts, two primes per 64-bit LDS atomic
                lds_u64 *lh2 = reinterpret_cast<lds_u64 *>(static_cast<uintptr_t>(ka + 32u));
                const unsigned long long c01 = (unsigned long long)pcs[0] | ((unsigned long long)pcs[1] << 32);
                const unsigned long long c23 = (unsigned long long)pcs[2] | ((unsigned long long)pcs[3] << 32);
                if (c01 != 0ull) __hip_atomic_fetch_add(&lh2[0], c01, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (c23 != 0ull) __hip_atomic_fetch_add(&lh2[1], c23, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                ka += 48u;
            }
        }
        // Lanes that finish a block take the next blocks of their wave's
        // chunk, so that no lane idles while others still have long blocks;
        // a wave whose chunk runs short takes a new one with one LDS atomic.
        const unsigned long long dm =
            __builtin_amdgcn_uicmp(Ulo | Uhi, 0u, 32) | __builtin_amdgcn_uicmp(ka, ka_end, 35);  // ==, >=
        if (dm != 0ull) {
            const uint32_t cnt = (uint32_t)__popcll(dm);
            const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(dm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)dm, 0u));
            uint32_t nb = c_next + r;
            if (c_end - c_next >= cnt) {
                c_next += cnt;
            } else {
                const uint32_t rem = c_end - c_next;
                const uint32_t leader = (uint32_t)__builtin_ctzll(dm);
                uint32_t cn = 0;
                if (lane == leader) {
                    // the counter's address is made opaque so that the
                    // compiler does not wrap this one-lane atomic in its wave
                    // aggregation
                    uint32_t na = (uint32_t)(uintptr_t)(lds_u32 *)L.next;
                    asm volatile("" : "+v"(na));
                    cn = __hip_atomic_fetch_add(reinterpret_cast<lds_u32 *>(static_cast<uintptr_t>(na)), 64u,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                cn = __builtin_amdgcn_readlane(cn, leader);
                nb = r < rem ? nb : cn + (r - rem);
                c_next = cn + (cnt - rem);
                c_end = cn + 64u;
            }
            if ((Ulo | Uhi) == 0u || ka >= ka_end) {
                if constexpr (VERIFY) {
                    // a block left with unresolved n: the last probe was not
                    // necessarily a hit, so its last hit is found again
                    if (Ulo | Uhi) lastkey = last_hit_key(b);
                } else {
                    accbg += (unsigned long long)(long long)((int)b - (int)nb) * sumg;
                }
                minkey = min(minkey, lastkey | b);
                if (Ulo | Uhi) push_unresolved(b, Ulo, Uhi);
                b = nb;
                bw = bits_addr + 8u * b + HB / 8u - PX_BIAS;
                ka = pr_addr;
                Ulo = ~0u;
                Uhi = ~0u;
            // the tile's last block may be partial: a wave-level test keeps
            // the masking off the common path
                if (ragged && __builtin_amdgcn_ballot_w64(b + 1u == nblk) != 0ull) {
                    if (b + 1u == nblk) {
                        Ulo = last_lo;
                        Uhi = last_hi;
                    }
                }
            }
        }
    }

    // ---- tile summary ------------------------------------------------------
    // Lane part of the checksum of the resolved n, with p = 2^17 - 1 - 2g:
    //   sum of p floor(n/128)   = 131071 (sum of floor(n/128) over resolved n)
    //                             - 2 (sum over hits of floor(n/128) g popcount)
    //   sum of p (2c+1) 2^i     = sum over halves c of (2c+1) (131071 (sum of
    //                             2^i over resolved n of half c) - 2 s_c)
    // where the sums over resolved n are the sums over the whole tile minus
    // the deficits; thread 0 adds the whole-tile terms and the masked n.
    if (tid == 0u) {
        uint32_t lo, hi;
        block_mask(0u, lo, hi);
        deficit(0u, ~lo, ~hi);
        if (nblk > 1u) {
            block_mask(nblk - 1u, lo, hi);
            deficit(nblk - 1u, ~lo, ~hi);
        }
    }
    accbg += (unsigned long long)b * sumg;
    unsigned long long ysum = 0ull - 2ull * ((N0 >> 7) * sumg + accbg);
    unsigned long long zsum = (0ull - 2ull * s0) + 3ull * (0ull - 2ull * s1);
    if (tid == 0u) {
        // every block's floor(n/128) for its 64 n, and every half's 2^i sum
        const unsigned long long nb = nblk;
        const unsigned long long sum_b = nb * (N0 >> 7) + nb * (nb - 1ull) / 2ull;
        ysum += 131071ull * 64ull * sum_b;
        zsum += 4ull * 131071ull * (nb * 0xFFFFFFFFull);
        if (has4) zsum += 8ull;   // n = 4: p = 2 at i = 2 of half 0
    }
    const unsigned long long cs = VERIFY ? 0ull : (ysum << 33) + zsum;
    const uint32_t gmax = minkey >> 16, mblk = minkey & 0xFFFFu;
    const uint32_t maxp = minkey == 0xFFFFFFFFu ? 0u : (gmax == 0xFFFFu ? 2u : 131071u - 2u * gmax);
    const unsigned long long key = ((unsigned long long)maxp << 32) | (0xFFFFFFFFu - mblk);
    // LDS atomics instead of shuffles: nothing per lane stays live for them
    // across the tiles of a persistent workgroup
    if (cs) atomicAdd(&L.red[0], cs);
    if (maxp) atomicMax(&L.red[2], key);
    __syncthreads();
    if (wave == 0) {
        // the lanes' parts plus the deficit terms of the n not resolved here
        const unsigned long long csum =
            VERIFY ? 0ull
                   : L.red[0] + ((0ull - 131071ull * L.red[4]) << 33) + (0ull - 131071ull * L.red[5]) +
                         3ull * (0ull - 131071ull * L.red[6]);
        const unsigned long long xsum = L.red[1], kmax = L.red[2];
        const uint32_t mp = (uint32_t)(kmax >> 32);
        const uint32_t mb = 0xFFFFFFFFu - (uint32_t)(kmax & 0xFFFFFFFFu);
        // smallest n of block mb with p_min = mp: the n of the block that mp
        // hits and no smaller prime does
        uint32_t am = 0;
        if (mp == 2u) {
            am = 2u;  // n = 4
        } else if (mp != 0u) {
            uint32_t ulo, uhi;
            block_mask(mb, ulo, uhi);
            const uint32_t hmp = (mp + 1u) >> 1, mbase = 64u * mb + HB;
            uint32_t olo = 0, ohi = 0;
            for (uint32_t kk = lane; kk < nps; kk += 64u) {
                const uint32_t h = 65536u - (L.pr[pr_px(kk)] & 0xFFFFu);
                if (h < hmp) {
                    const uint32_t s = mbase - h;
                    const uint32_t *wp = L.bits + (s >> 5);
                    olo |= __builtin_amdgcn_alignbit(wp[1], wp[0], s);
                    ohi |= __builtin_amdgcn_alignbit(wp[2], wp[1], s);
                }
            }
            uint32_t *orw = reinterpret_cast<uint32_t *>(&L.red[3]);
            if (olo) atomicOr(&orw[0], olo);
            if (ohi) atomicOr(&orw[1], ohi);
            __builtin_amdgcn_wave_barrier();
            olo = orw[0];
            ohi = orw[1];
            const uint32_t s = mbase - hmp;
            const uint32_t *wp = L.bits + (s >> 5);
            const uint32_t hlo = __builtin_amdgcn_alignbit(wp[1], wp[0], s) & ulo & ~olo;
            const uint32_t hhi = __builtin_amdgcn_alignbit(wp[2], wp[1], s) & uhi & ~ohi;
            am = 64u * mb + (hlo ? (uint32_t)__builtin_ctz(hlo) : 32u + (uint32_t)__builtin_ctz(hhi));
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
            C[CY_EXH] += xsum;
            const unsigned long long an = N0 + 2ull * am;
            if (mp > C[CY_MAXP] || (mp != 0u && mp == C[CY_MAXP] && an < C[CY_ARGN])) {
                C[CY_MAXP] = mp;
                C[CY_ARGN] = an;
            }
        }
    }
    __syncthreads();
}

template <int NT, int PB, bool PERS, bool SIEVE_ONLY, bool GW>
__global__ __launch_bounds__(NT) void k_tile(GbTileArgs a)
{
    extern __shared__ uint32_t smem[];
    const TileLds L = carve(smem, a);
    HistCarry hc;
    if constexpr (!SIEVE_ONLY) {
        setup_primes<NT, PB == 1, GW>(a, L);   // behind the first barrier below
        if (threadIdx.x == 0) L.carry[CY_SLOT] = kNoSlot;
    }
    if constexpr (PERS) {
        for (;;) {
            if (threadIdx.x == 0) *L.tile = atomicAdd(a.queue, 1ull);
            __syncthreads();
            const unsigned long long g = *L.tile;
            if (g >= a.ntiles) break;
            process_tile<NT, PB, SIEVE_ONLY, GW>(a, g, L, hc);
        }
    } else {
        __syncthreads();
        process_tile<NT, PB, SIEVE_ONLY, GW>(a, a.tile0 + blockIdx.x, L, hc);
    }
    // process_tile ends with a barrier, so every count is in LDS
    if constexpr (!SIEVE_ONLY && PB != 1)
        if (hc.row != kNoRow) flush_hist(a, L, hc.row);
    if constexpr (!SIEVE_ONLY)
        if (threadIdx.x == 0) flush_slot(a, L.carry);
}


// ---------------------------------------------------------------------------
// 64-bit Montgomery arithmetic (Montgomery 1985) for the Miller-Rabin test.
// Residues are kept as x*R mod m with R = 2^64, m odd.
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long mont_inv(unsigned long long m)
{
    // Newton iteration for m^-1 mod 2^64: m*m = 1 mod 8 gives 3 correct bits
    unsigned long long x = m;
    for (int i = 0; i < 5; ++i) x *= 2ull - m * x;
    return 0ull - x;   // -m^-1
}

__device__ __forceinline__ unsigned long long mont_mul(unsigned long long a, unsigned long long b,
                                                       unsigned long long m, unsigned long long ni)
{
    const unsigned long long lo = a * b, hi = __umul64hi(a, b);
    const unsigned long long u = lo * ni;
    const unsigned long long mh = __umul64hi(u, m);
    // lo + u*m = 0 mod 2^64 and carries out exactly when lo != 0
    const unsigned long long t = hi + mh;
    const bool c1 = t < hi;
    const unsigned long long t2 = t + (lo != 0ull);
    const bool c2 = t2 < t;
    return (c1 || c2 || t2 >= m) ? t2 - m : t2;
}

__device__ __forceinline__ unsigned long long add_mod(unsigned long long x, unsigned long long y,
                                                      unsigned long long m)
{
    const unsigned long long s = x + y;
    return (s < x || s >= m) ? s - m : s;
}

// Strong probable-prime test of odd m > 37 to the small base a.
__device__ bool sprp(unsigned long long m, uint32_t a)
{
    const unsigned long long ni = mont_inv(m);
    const unsigned long long one = (0ull - m) % m;        // R mod m
    const unsigned long long mone = m - one;              // -1
    unsigned long long ar = 0;                            // a*R mod m
    for (int bit = 5; bit >= 0; --bit) {
        ar = add_mod(ar, ar, m);
        if ((a >> bit) & 1u) ar = add_mod(ar, one, m);
    }
    unsigned long long d = m - 1ull;
    const int s = __builtin_ctzll(d);
    d >>= s;
    unsigned long long x = one;
    for (int bit = 63 - __builtin_clzll(d); bit >= 0; --bit) {
        x = mont_mul(x, x, m, ni);
        if ((d >> bit) & 1ull) x = (a == 2u) ? add_mod(x, x, m) : mont_mul(x, ar, m, ni);
    }
    if (x == one || x == mone) return true;
    for (int r = 1; r < s; ++r) {
        x = mont_mul(x, x, m, ni);
        if (x == mone) return true;
        if (x == one) return false;
    }
    return false;
}

// Odd primes up to 37 as a bit mask over (v-1)/2.
__device__ __forceinline__ bool small_odd_prime(unsigned long long v)
{
    // 3,5,7,11,13,17,19,23,29,31,37 -> bits 1,2,3,5,6,8,9,11,14,15,18
    const uint32_t mask = (1u << 1) | (1u << 2) | (1u << 3) | (1u << 5) | (1u << 6) | (1u << 8) |
                          (1u << 9) | (1u << 11) | (1u << 14) | (1u << 15) | (1u << 18);
    return (mask >> ((uint32_t)(v - 1) >> 1)) & 1u;
}

// Base-2 screen of an odd v >= 3: exact for v <= 37, a strong base-2 test above.
__device__ __forceinline__ bool screen2(unsigned long long v)
{
    return v <= 37ull ? small_odd_prime(v) : sprp(v, 2u);
}

__constant__ uint32_t MR_BASES[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};

__global__ __launch_bounds__(256) void k_mr(GbMrArgs a)
{
    const uint32_t lane = threadIdx.x & 63u;
    const unsigned long long gw = (blockIdx.x * 256ull + threadIdx.x) >> 6;
    const unsigned long long nw = (gridDim.x * 256ull) >> 6;
    unsigned long long cnt = *a.list_count;
    if (cnt > a.list_cap) cnt = a.list_cap;
    const uint32_t ptop = a.primes[a.ntab - 1];
    for (unsigned long long e = gw; e < cnt; e += nw) {
        const GbExh E = a.list[e];
        const unsigned long long n = E.n;
        unsigned long long found = 0, kfound = ~0ull;
        if (n == 4ull) {
            found = 2;
        } else {
            unsigned long long bound = n >> 1;
            if (a.budget && a.budget < bound) bound = a.budget;
            for (unsigned long long kb = E.start_k;; kb += 64ull) {
                const unsigned long long k = kb + lane;
                const bool in_tab = k < a.ntab;
                const unsigned long long p =
                    in_tab ? (unsigned long long)a.primes[k] : (unsigned long long)ptop + 2ull * (k - a.ntab + 1ull);
                const bool valid = p <= bound;
                const unsigned long long q = n - p;
                const bool pass = valid && screen2(q) && (in_tab || screen2(p));
                unsigned long long m = __ballot(pass);
                while (m) {
                    const int c = __builtin_ctzll(m);
                    const unsigned long long qc = __shfl(q, c, 64);
                    const unsigned long long pc = __shfl(p, c, 64);
                    const bool tabc = (kb + (unsigned long long)c) < a.ntab;
                    bool ok = true;
                    if (lane < 11u) {
                        if (qc > 37ull) ok = sprp(qc, MR_BASES[lane + 1]);
                        if (ok && !tabc && pc > 37ull) ok = sprp(pc, MR_BASES[lane + 1]);
                    }
                    if (__ballot(!ok) == 0ull) {
                        found = pc;
                        kfound = kb + (unsigned long long)c;
                        break;
                    }
                    m &= m - 1ull;
                }
                if (found) break;
                if (__ballot(valid) == 0ull) break;  // every candidate is past the bound
            }
        }
        if (lane == 0) {
            a.list[e].p = found;
            if (a.pmin && E.out_index != ~0ull) {
                if (a.pmin_bits == 16)
                    static_cast<uint16_t *>(a.pmin)[E.out_index] = (uint16_t)(found < 65536ull ? found : 0ull);
                else
                    static_cast<uint32_t *>(a.pmin)[E.out_index] = (uint32_t)(found < 4294967296ull ? found : 0ull);
            }
            if (a.slots) {
                GbSlot *S = a.slots + E.slot;
                unsigned long long *hist = a.hist + (a.hist_per_slot ? (unsigned long long)E.slot : 0ull) * GB_HIST_BINS_I;
                if (found) {
                    const unsigned long long bin =
                        found == 2ull ? 0ull : (found < 65536ull ? kfound + 1ull : GB_HIST_BINS_I - 1ull);
                    atomicAdd(&hist[bin], 1ull);
                    atomicAdd(&S->checksum, checksum_weight(n) * found);
                    atomicMax(&S->max_p, found);
                } else {
                    atomicAdd(&S->n_failed, 1ull);
                    atomicMin(&S->first_failed_n, n);
                }
                if (a.count_exh && (found == 0ull || found > a.pmax_fast)) atomicAdd(&S->n_exhaustive, 1ull);
            }
        }
    }
}

// One block per probe record, its threads over the workgroup rows.  When
// every row names the same histogram row (a range or windows call without
// per-segment histograms) the block sums the record's counts and adds them
// with one 64-bit atomic; otherwise each thread adds its own partial sums.
__global__ __launch_bounds__(256) void k_hist_reduce(const uint32_t *wg_hist, uint32_t nwg, uint32_t stride,
                                                     uint32_t nrec, const uint32_t *rec_bin,
                                                     unsigned long long *hist)
{
    __shared__ unsigned long long part[4];
    __shared__ uint32_t lo_row, hi_row;
    const uint32_t r = blockIdx.x;
    if (r >= nrec) return;
    if (threadIdx.x == 0) {
        lo_row = 0xFFFFFFFFu;
        hi_row = 0u;
    }
    __syncthreads();
    const uint32_t bin = rec_bin[r];
    uint32_t mine = 0xFFFFFFFFu;
    unsigned long long sum = 0;
    for (uint32_t w = threadIdx.x; w < nwg; w += blockDim.x) {
        const uint32_t *row = wg_hist + (unsigned long long)w * stride;
        const uint32_t hr = row[0];
        if (hr == 0xFFFFFFFFu) continue;
        const uint32_t c = row[1u + r];
        if (mine != 0xFFFFFFFFu && hr != mine) {   // a second histogram row in this thread's share
            if (sum) atomicAdd(&hist[(unsigned long long)mine * GB_HIST_BINS_I + bin], sum);
            sum = 0;
            hi_row = 0xFFFFFFFEu;                   // forces the per-thread path below
        }
        mine = hr;
        sum += c;
    }
    if (mine != 0xFFFFFFFFu) {
        atomicMin(&lo_row, mine);
        atomicMax(&hi_row, mine);
    }
    __syncthreads();
    if (lo_row == 0xFFFFFFFFu) return;   // no row holds anything
    if (lo_row != hi_row) {
        if (sum) atomicAdd(&hist[(unsigned long long)mine * GB_HIST_BINS_I + bin], sum);
        return;
    }
    // one histogram row: wave sums, then the block's
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_down(sum, o, 64);
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (uint32_t k = 0; k < (blockDim.x + 63u) / 64u; ++k) t += part[k];
        if (t) atomicAdd(&hist[(unsigned long long)lo_row * GB_HIST_BINS_I + bin], t);
    }
}

__global__ void k_argmax(GbSlot *slots, const GbTileRec *recs, const unsigned long long *rec_count,
                         unsigned long long rec_cap, const GbExh *list,
                         const unsigned long long *list_count, unsigned long long cap)
{
    unsigned long long cnt = *list_count;
    if (cnt > cap) cnt = cap;
    unsigned long long nrecs = *rec_count;
    if (nrecs > rec_cap) nrecs = rec_cap;
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
         i < nrecs + cnt; i += stride) {
        if (i < nrecs) {
            const GbTileRec r = recs[i];
            if (r.max_p && r.max_p == slots[r.slot].max_p) atomicMin(&slots[r.slot].argmax_n, r.argmax_n);
        } else {
            const GbExh &x = list[i - nrecs];
            if (x.p && x.p == slots[x.slot].max_p) atomicMin(&slots[x.slot].argmax_n, x.n);
        }
    }
}

__global__ void k_init(GbSlot *slots, uint64_t nslots, unsigned long long *hist, uint64_t hist_words,
                       unsigned long long *counters, uint32_t ncounters)
{
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    const unsigned long long i0 = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
    for (unsigned long long i = i0; i < nslots; i += stride) {
        GbSlot s = {};
        s.argmax_n = ~0ull;
        s.first_failed_n = ~0ull;
        slots[i] = s;
    }
    for (unsigned long long i = i0; i < hist_words; i += stride) hist[i] = 0ull;
    if (i0 < ncounters) counters[i0] = 0ull;
}

__global__ void k_make_queries(GbExh *list, const unsigned long long *n, uint64_t k,
                               unsigned long long *list_count)
{
    const unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
    if (i < k) {
        GbExh x;
        x.n = n[i];
        x.out_index = ~0ull;
        x.slot = 0;
        x.start_k = 0;
        x.p = 0;
        list[i] = x;
    }
    if (i == 0) *list_count = k;
}

__global__ void k_finish_queries(const GbExh *list, uint64_t k, unsigned long long *p_out)
{
    const unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
    if (i < k) p_out[i] = list[i].p;
}

template <int NT, int PB, bool PERS, bool SO, bool GW>
hipError_t launch_one(const GbTileArgs &a, uint32_t grid, size_t lds, hipStream_t st)
{
    hipLaunchKernelGGL((k_tile<NT, PB, PERS, SO, GW>), dim3(grid), dim3(NT), lds, st, a);
    return hipGetLastError();
}

template <int NT, int PB, bool PERS, bool SO, bool GW>
hipError_t allow_lds(size_t lds)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_tile<NT, PB, PERS, SO, GW>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int NT, bool GW>
hipError_t allow_lds_search(size_t lds)
{
    hipError_t e = hipSuccess, r;
    if ((r = allow_lds<NT, 0, false, false, GW>(lds)) != hipSuccess) e = r;
    if ((r = allow_lds<NT, 1, true, false, GW>(lds)) != hipSuccess) e = r;
    if ((r = allow_lds<NT, 16, false, false, GW>(lds)) != hipSuccess) e = r;
    if ((r = allow_lds<NT, 32, false, false, GW>(lds)) != hipSuccess) e = r;
    if ((r = allow_lds<NT, 0, true, false, GW>(lds)) != hipSuccess) e = r;
    if ((r = allow_lds<NT, 16, true, false, GW>(lds)) != hipSuccess) e = r;
    if ((r = allow_lds<NT, 32, true, false, GW>(lds)) != hipSuccess) e = r;
    return e;
}

template <int NT>
hipError_t allow_lds_nt(size_t lds)
{
    hipError_t e = hipSuccess, r;
    if ((r = allow_lds<NT, 0, false, true, false>(lds)) != hipSuccess) e = r;
    if ((r = allow_lds_search<NT, false>(lds)) != hipSuccess) e = r;
    if ((r = allow_lds_search<NT, true>(lds)) != hipSuccess) e = r;
    return e;
}

template <int NT, bool GW>
hipError_t launch_search(const GbTileArgs &a, uint32_t grid, size_t lds, int pb, bool pers, hipStream_t st)
{
    if (pers) {
        if (pb == 1) return launch_one<NT, 1, true, false, GW>(a, grid, lds, st);
        if (pb == 16) return launch_one<NT, 16, true, false, GW>(a, grid, lds, st);
        if (pb == 32) return launch_one<NT, 32, true, false, GW>(a, grid, lds, st);
        return launch_one<NT, 0, true, false, GW>(a, grid, lds, st);
    }
    if (pb == 16) return launch_one<NT, 16, false, false, GW>(a, grid, lds, st);
    if (pb == 32) return launch_one<NT, 32, false, false, GW>(a, grid, lds, st);
    return launch_one<NT, 0, false, false, GW>(a, grid, lds, st);
}

template <int NT>
hipError_t launch_nt(const GbTileArgs &a, uint32_t grid, size_t lds, int pb, bool pers, bool so, bool gw,
                     hipStream_t st)
{
    if (so) return launch_one<NT, 0, false, true, false>(a, grid, lds, st);
    return gw ? launch_search<NT, true>(a, grid, lds, pb, pers, st) : launch_search<NT, false>(a, grid, lds, pb, pers, st);
}

}  // namespace

size_t gb_tile_lds_bytes(uint32_t tile_n, uint32_t halo_bits, uint32_t np_search, uint32_t n_off)
{
    // the same carve-up as carve()
    size_t words = ((tile_n + halo_bits) / 32 + 3) & ~(size_t)3;
    words += 12 * (((size_t)np_search + 3) / 4 + 2);          // prime groups
    words += n_off;                                       // first strikes
    words = (words + 1) & ~(size_t)1;
    words += 2 * 7;                                       // tile reductions
    words += 2 * 6;                                       // the slot carry
    words = (words + 1) & ~(size_t)1;
    words += 2;                                           // the persistent tile index
    words += 2;                                           // the block counter (and padding)
    return words * 4;
}

hipError_t gb_prepare_tiles(uint32_t threads, size_t lds_bytes)
{
    switch (threads) {
    case 256: return allow_lds_nt<256>(lds_bytes);
    case 512: return allow_lds_nt<512>(lds_bytes);
    case 1024: return allow_lds_nt<1024>(lds_bytes);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gb_tile_occupancy(uint32_t threads, size_t lds_bytes, bool group_window, int *blocks_per_cu)
{
#define GB_OCC(NT)                                                                                        \
    (group_window                                                                                         \
         ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_tile<NT, 0, true, false, true>, NT,  \
                                                        lds_bytes)                                        \
         : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_tile<NT, 0, true, false, false>, NT, \
                                                        lds_bytes))
    switch (threads) {
    case 256: return GB_OCC(256);
    case 512: return GB_OCC(512);
    case 1024: return GB_OCC(1024);
    default: return hipErrorInvalidValue;
    }
#undef GB_OCC
}

hipError_t gb_launch_tiles(const GbTileArgs &a, uint32_t grid, uint32_t threads, size_t lds_bytes, int pmin_bits,
                           bool persistent, bool sieve_only, bool group_window, hipStream_t st)
{
    if (grid == 0) return hipSuccess;
    switch (threads) {
    case 256: return launch_nt<256>(a, grid, lds_bytes, pmin_bits, persistent, sieve_only, group_window, st);
    case 512: return launch_nt<512>(a, grid, lds_bytes, pmin_bits, persistent, sieve_only, group_window, st);
    case 1024: return launch_nt<1024>(a, grid, lds_bytes, pmin_bits, persistent, sieve_only, group_window, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gb_launch_mr(const GbMrArgs &a, uint32_t grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_mr, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t gb_launch_hist_reduce(const uint32_t *wg_hist, uint32_t nwg, uint32_t stride, uint32_t nrec,
                                 const uint32_t *rec_bin, unsigned long long *hist, hipStream_t st)
{
    if (nrec == 0 || nwg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hist_reduce, dim3(nrec), dim3(256), 0, st, wg_hist, nwg, stride, nrec, rec_bin, hist);
    return hipGetLastError();
}

hipError_t gb_launch_argmax(GbSlot *slots, const GbTileRec *recs, const unsigned long long *rec_count,
                            unsigned long long rec_cap, const GbExh *list,
                            const unsigned long long *list_count, unsigned long long list_cap,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_argmax, dim3(1024), dim3(256), 0, st, slots, recs, rec_count, rec_cap, list,
                       list_count, list_cap);
    return hipGetLastError();
}

hipError_t gb_launch_init(GbSlot *slots, uint64_t nslots, unsigned long long *hist, uint64_t hist_words,
                          unsigned long long *counters, uint32_t ncounters, hipStream_t st)
{
    hipLaunchKernelGGL(k_init, dim3(512), dim3(256), 0, st, slots, nslots, hist, hist_words, counters,
                       ncounters);
    return hipGetLastError();
}

hipError_t gb_launch_make_queries(GbExh *list, const unsigned long long *n, uint64_t k,
                                  unsigned long long *list_count, hipStream_t st)
{
    const uint32_t grid = (uint32_t)((k + 255) / 256) + 1;
    hipLaunchKernelGGL(k_make_queries, dim3(grid), dim3(256), 0, st, list, n, k, list_count);
    return hipGetLastError();
}

hipError_t gb_launch_finish_queries(const GbExh *list, uint64_t k, unsigned long long *p_out,
                                    hipStream_t st)
{
    const uint32_t grid = (uint32_t)((k + 255) / 256) + 1;
    hipLaunchKernelGGL(k_finish_queries, dim3(grid), dim3(256), 0, st, list, k, p_out);
    return hipGetLastError();
}
