// gb_kernels.hip -- HIP kernels (gfx950, wave64) of the segmented Goldbach
// verifier besides the search (gb_class.hip).
//
// k_tile: the sieve of one tile of consecutive odd numbers, dumped to device
// memory (gb_sieve_window, for parity tests of the paper's segmented Sieve of
// Eratosthenes, subsection "Correct segmentation").  One workgroup sieves the
// odd numbers w0 + 2i, w0 = N0 + 1 - 2*HB, 0 <= i < T + HB, into an LDS bitset
// (bit = 1 for a prime): a rotated wheel pattern for the multiples of 3 ..
// wheel_max, then the odd multiples m p >= p^2 of every sieving prime above
// it, the small primes striding with the whole workgroup, the medium ones
// with one wave, the large ones with one lane each.
//
// k_mr: one wavefront per listed n (the exhaustive phase, the paper's Phase
// 2, here on the GPU; and the single-n queries).  Lane l takes the l-th next
// candidate prime p, screens q = n - p with a base-2 strong probable-prime
// test in Montgomery arithmetic, and the lowest passing lane (ballot + first
// set bit) is confirmed with the other eleven bases of the deterministic
// 64-bit test (bases 2..37), one base per lane.
//
// k_hist_reduce, k_argmax, k_init and the query helpers complete a call.
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

// Clear the bits of m's zeros in the LDS word at byte address addr.
__device__ __forceinline__ void lds_and(uint32_t addr, uint32_t m)
{
    __hip_atomic_fetch_and(reinterpret_cast<lds_u32 *>(static_cast<uintptr_t>(addr)), m, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

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

// LDS carve-up of one sieve workgroup (offsets in 32-bit words).
struct TileLds {
    uint32_t *bits;   // (T + HB)/32 words: the tile's window, 1 = prime
    uint32_t *offs;   // first bit index (or ~0) of each small/medium sieving prime
};

__device__ __forceinline__ TileLds carve(uint32_t *smem, const GbTileArgs &a)
{
    TileLds L;
    L.bits = smem;
    L.offs = smem + (a.tile_n + a.halo_bits) / 32;
    return L;
}

// The sieve of tile g of the window table, dumped to a.sieve_out.
template <int NT>
__device__ void sieve_tile(const GbTileArgs &a, unsigned long long g, const TileLds &L)
{
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
    const bool small_w0 = w0 < (1ll << 53);   // exact as a double
    const double w0d = (double)w0;

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

    // bitset dump: tile t owns output bits [T*t, T*t + cnt)
    const unsigned long long obase = (unsigned long long)a.tile_n * t / 32;
    for (uint32_t i = tid; i < cnt / 32; i += NT) a.sieve_out[obase + i] = L.bits[i];
}

template <int NT>
__global__ __launch_bounds__(NT) void k_tile(GbTileArgs a)
{
    extern __shared__ uint32_t smem[];
    const TileLds L = carve(smem, a);
    sieve_tile<NT>(a, a.tile0 + blockIdx.x, L);
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

template <int NT>
hipError_t launch_tile(const GbTileArgs &a, uint32_t grid, size_t lds, hipStream_t st)
{
    hipLaunchKernelGGL((k_tile<NT>), dim3(grid), dim3(NT), lds, st, a);
    return hipGetLastError();
}

template <int NT>
hipError_t allow_tile(size_t lds)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_tile<NT>), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

}  // namespace

size_t gb_tile_lds_bytes(uint32_t tile_n, uint32_t halo_bits, uint32_t n_off)
{
    // the same carve-up as carve()
    return 4 * ((size_t)(tile_n + halo_bits) / 32 + n_off);
}

hipError_t gb_prepare_tiles(uint32_t threads, size_t lds_bytes)
{
    switch (threads) {
    case 256: return allow_tile<256>(lds_bytes);
    case 512: return allow_tile<512>(lds_bytes);
    case 1024: return allow_tile<1024>(lds_bytes);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gb_launch_tiles(const GbTileArgs &a, uint32_t grid, uint32_t threads, size_t lds_bytes, hipStream_t st)
{
    if (grid == 0) return hipSuccess;
    switch (threads) {
    case 256: return launch_tile<256>(a, grid, lds_bytes, st);
    case 512: return launch_tile<512>(a, grid, lds_bytes, st);
    case 1024: return launch_tile<1024>(a, grid, lds_bytes, st);
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
