// gb_bignum28.h -- fixed-width multi-limb integers with 28-bit limbs (K
// little-endian limbs, each held in the low 28 bits of a 32-bit word) and the
// strong probable-prime test on them, for the minimal Goldbach prime of even
// n beyond 64 bits (paper section "Arbitrary Precision Checker", which tests
// q = n - p with Miller-Rabin).
//
// Arithmetic mod an odd m with 2^(28(K - E) + 24) <= m < 2^(28K - 2),
// R = 2^(28K), where E = est_limbs(K) is 3 up to K = 16 and 5 above:
//
// - Montgomery squaring (Montgomery 1985) in the finely integrated
//   product-scanning order (Koc, Acar and Kaliski 1996), each cross product
//   taken once and doubled.  With 28-bit limbs a column of at most 2K + 1
//   products plus the carry stays below 2^62, so a column sums in one 64-bit
//   accumulator: one 64-bit multiply-add per limb product, no carry handling.
// - Lazy reduction: operands and results lie in [0, 2m), not [0, m).  As
//   4m < R, a squaring of a value below 2m ends below 2m without the final
//   conditional subtraction; values are brought into [0, m) only where they
//   are compared.
// - Multiplication by a small integer f <= 2^20: x f - h m, with the quotient
//   h estimated from the top E limbs of x and of m in double precision,
//   rounded down so that h never exceeds the true quotient; the result is
//   below 1.2 m (the bound is worked out at mul_small).
//
// Host and device: the same code runs in a lane or on the CPU.
#pragma once
#include <cstdint>

namespace gbbig28 {

constexpr uint32_t kBits = 28;
constexpr uint32_t kMask = (1u << kBits) - 1u;

template <int K> struct Num {
    uint32_t w[K];
};

// Limbs in the quotient estimate of mul_small
template <int K> constexpr int est_limbs() { return K <= 16 ? 3 : 5; }

// -m^(-1) mod 2^28 for odd m, by Newton's iteration x <- x (2 - m x)
__host__ __device__ inline uint32_t neg_inv28(uint32_t m)
{
    uint32_t x = m;
    for (int i = 0; i < 4; ++i) x *= 2u - m * x;
    return (0u - x) & kMask;
}

template <int K> __host__ __device__ inline bool equal(const Num<K> &a, const Num<K> &b)
{
    uint32_t d = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) d |= a.w[i] ^ b.w[i];
    return d == 0;
}

// r = a - b, returns the borrow
template <int K> __host__ __device__ inline uint32_t sub(Num<K> &r, const Num<K> &a, const Num<K> &b)
{
    uint32_t br = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const uint32_t t = a.w[i] - b.w[i] - br;
        r.w[i] = t & kMask;
        br = t >> 31;
    }
    return br;
}

// a mod m for a < 2m
template <int K> __host__ __device__ inline void reduce_once(Num<K> &a, const Num<K> &m)
{
    Num<K> d;
    const uint32_t br = sub(d, a, m);
#pragma unroll
    for (int i = 0; i < K; ++i) a.w[i] = br ? a.w[i] : d.w[i];
}

// a^2 R^(-1) mod m, lazily: for a < 2m the result is below 2m (4m < R).
// Column i collects every a_j a_(i-j) (the pairs j < i - j once, doubled,
// and a_(i/2)^2) and u_j m_(i-j); the low columns choose
// u_i = t ninv mod 2^28 so that the column's low 28 bits become zero, the
// high columns are the result.  Fully unrolled, so every limb stays in a
// register.
template <int K>
__host__ __device__ inline void mont_sqr(Num<K> &r, const Num<K> &a, const Num<K> &m, uint32_t ninv)
{
    // column: below K/2 + 1 cross products doubled, a square and K
    // products u_j m_(i-j), each below 2^56, plus a carry below 2^36
    static_assert(K >= 4 && K <= 40, "a column must stay below 2^64");
    uint64_t t = 0;
    uint32_t u[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        uint64_t c = 0;
#pragma unroll
        for (int j = 0; j < i - j; ++j) c += (uint64_t)a.w[j] * a.w[i - j];
        t += c << 1;
        if ((i & 1) == 0) t += (uint64_t)a.w[i / 2] * a.w[i / 2];
#pragma unroll
        for (int j = 0; j < i; ++j) t += (uint64_t)u[j] * m.w[i - j];
        u[i] = ((uint32_t)t * ninv) & kMask;
        t += (uint64_t)u[i] * m.w[0];                // the low 28 bits are now zero
        t >>= kBits;
    }
#pragma unroll
    for (int i = K; i < 2 * K; ++i) {
        uint64_t c = 0;
#pragma unroll
        for (int j = i - K + 1; j < i - j; ++j) c += (uint64_t)a.w[j] * a.w[i - j];
        t += c << 1;
        if ((i & 1) == 0 && i / 2 < K) t += (uint64_t)a.w[i / 2] * a.w[i / 2];
#pragma unroll
        for (int j = i - K + 1; j < K; ++j) t += (uint64_t)u[j] * m.w[i - j];
        r.w[i - K] = (uint32_t)t & kMask;
        t >>= kBits;
    }
    // (a^2 + U m) / R < (4 m^2 + R m) / R < 2m < R: nothing is left in t
}

// The top E limbs of x as a double: x / 2^(28(K-E)) rounded down, then
// rounded to double (Horner's rule, one rounding per step)
template <int K> __host__ __device__ inline double top_limbs(const Num<K> &x)
{
    constexpr int E = est_limbs<K>();
    double v = (double)x.w[K - 1];
#pragma unroll
    for (int i = 2; i <= E; ++i) v = v * 268435456.0 + (double)x.w[K - i];
    return v;
}

// The quotient estimate's scale for m: (1 - 2^-40) / (M' + 1), with M' m's
// top E limbs (m / 2^(28(K-E)) rounded down) in double precision.
template <int K> __host__ __device__ inline double est_recip(const Num<K> &m)
{
    return (1.0 - 0x1p-40) / (top_limbs(m) + 1.0);
}

// x <- x f mod m, lazily, for x < 2m and 1 <= f <= 2^20 (rq = est_recip(m)).
// With X = x f, M' = m / 2^(28(K-E)) >= 2^24 and x' = x / 2^(28(K-E)) < 2M',
// the estimate h = floor(f X' rq) (X': x's top E limbs) never exceeds X / m:
// each of the few roundings moves a value by at most 2^-53 of itself, less
// than 2^-48 in all, and the factor 1 - 2^-40 in rq covers them.  It falls
// short of X / m by less than 1 + f (3 / M' + 2^-37) < 1.19, so X - h m lies
// in [0, 1.19 m).  One pass over the limbs forms x_i f - h m_i plus the
// signed carry.
template <int K> __host__ __device__ inline void mul_small(Num<K> &x, uint32_t f, const Num<K> &m, double rq)
{
    const double xd = top_limbs(x);
    const int32_t nh = -(int32_t)(uint32_t)(xd * (double)f * rq);   // h < 2^21
    int64_t c = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        int64_t t = (int64_t)(int32_t)x.w[i] * (int32_t)f + c;
        t += (int64_t)nh * (int32_t)m.w[i];
        x.w[i] = (uint32_t)t & kMask;
        c = t >> kBits;                              // arithmetic: the carry may be negative
    }
}

template <int K> __host__ __device__ inline int bit_length(const Num<K> &a)
{
    for (int i = K - 1; i >= 0; --i)
        if (a.w[i]) return (int)kBits * i + 32 - __builtin_clz(a.w[i]);
    return 0;
}

// Limb j of a for a j known only at run time, by a chain of selects (an
// indexed read would move the number out of registers).
template <int K> __host__ __device__ inline uint32_t limb_at(const Num<K> &a, int j)
{
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) r = (i == j) ? a.w[i] : r;
    return r;
}

// R mod m, m odd with nb bits: 2^(nb-1) < m multiplied by 2^(28K - nb + 1)
// in steps of at most 2^20, then brought below m.
template <int K> __host__ __device__ inline void mont_one(Num<K> &one, const Num<K> &m, int nb, double rq)
{
    const int top = (nb - 1) / (int)kBits;
#pragma unroll
    for (int i = 0; i < K; ++i) one.w[i] = (i == top) ? 1u << (nb - 1 - top * (int)kBits) : 0u;
    for (int e = (int)kBits * K - nb + 1; e > 0; e -= 20) mul_small(one, 1u << (e < 20 ? e : 20), m, rq);
    reduce_once(one, m);
}

// Strong probable prime to base a: q odd with 2^(28(K - E) + 24) <= q < 2^(28K - 2),
// 2 <= a <= 101 (so that a^3 <= 2^20).  With q - 1 = d 2^s, d odd: true when
// a^d = 1 or -1 mod q, or a^(d 2^r) = -1 for some 0 < r < s.
//
// a^d is taken left to right over 2-bit windows of d, in Montgomery form:
// two squarings, then one multiplication by a^v <= 2^20 for the window's
// value v (by 1 when v = 0, so that every lane does the same work).  d is
// first shifted so that its lowest window ends at an even bit position e and
// its top bit lies in the top window (bits 28K - 2, 28K - 1), so the windows
// of every q sit at the same positions and a window never straddles two
// limbs; only where the windows end (e) differs from q to q.
template <int K> __host__ __device__ inline bool strong_prp(const Num<K> &q, uint32_t a)
{
    const uint32_t ninv = neg_inv28(q.w[0]);
    const double rq = est_recip(q);
    const int nb = bit_length(q);
    // s: the lowest set bit of q - 1 (q odd: bit 0 is the one cleared)
    int s = 0;
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        const uint32_t w = i == 0 ? q.w[0] & ~1u : q.w[i];
        if (w) s = (int)kBits * i + __builtin_ctz(w);
    }
    if (s == 0) return false;                        // q = 1
    // dd = (q - 1) << t: d's bits at [e, 28K), zeros below; t <= 28E - 25
    // (q has at least 28 (K - E) + 25 bits), so t / 28 < E
    const int e = ((int)kBits * K - nb + s) & ~1;
    const int t = e - s;
    const int L = t / (int)kBits, b = t - L * (int)kBits;
    constexpr int E = est_limbs<K>();
    Num<K> dd;
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        // limbs i - L and i - L - 1 of q - 1 (w0 .. w5: limbs i .. i - 5)
        const uint32_t w0 = i == 0 ? q.w[0] & ~1u : q.w[i];
        const uint32_t w1 = i < 1 ? 0u : i == 1 ? q.w[0] & ~1u : q.w[i - 1];
        const uint32_t w2 = i < 2 ? 0u : i == 2 ? q.w[0] & ~1u : q.w[i - 2];
        const uint32_t w3 = i < 3 ? 0u : i == 3 ? q.w[0] & ~1u : q.w[i - 3];
        uint32_t hi = L == 0 ? w0 : L == 1 ? w1 : w2;
        uint32_t lo = L == 0 ? w1 : L == 1 ? w2 : w3;
        if constexpr (E > 3) {
            const uint32_t w4 = i < 4 ? 0u : i == 4 ? q.w[0] & ~1u : q.w[i - 4];
            const uint32_t w5 = i < 5 ? 0u : i == 5 ? q.w[0] & ~1u : q.w[i - 5];
            hi = L == 3 ? w3 : L == 4 ? w4 : hi;
            lo = L == 3 ? w4 : L == 4 ? w5 : lo;
        }
        dd.w[i] = ((hi << b) | (b ? lo >> (kBits - b) : 0u)) & kMask;
    }
    const uint32_t f1 = a, f2 = a * a, f3 = a * a * a;
    Num<K> x;
    mont_one(x, q, nb, rq);
    {
        const uint32_t v = dd.w[K - 1] >> (kBits - 2);
        mul_small(x, v == 1 ? f1 : v == 2 ? f2 : f3, q, rq);   // v != 0: the top bit of d is here
    }
    uint32_t wl = dd.w[K - 1];
    for (int pos = (int)kBits * K - 4; pos >= e; pos -= 2) {
        const int li = pos / (int)kBits, off = pos - li * (int)kBits;
        if (off == (int)kBits - 2) wl = limb_at(dd, li);
        const uint32_t v = (wl >> off) & 3u;
        mont_sqr(x, x, q, ninv);
        mont_sqr(x, x, q, ninv);
        mul_small(x, v == 0 ? 1u : v == 1 ? f1 : v == 2 ? f2 : f3, q, rq);
    }
    reduce_once(x, q);                               // a^d R mod q
    Num<K> one, mone;
    mont_one(one, q, nb, rq);
    sub(mone, q, one);
    if (equal(x, one) || equal(x, mone)) return true;
    for (int r = 1; r < s; ++r) {
        mont_sqr(x, x, q, ninv);
        reduce_once(x, q);
        if (equal(x, mone)) return true;
        if (equal(x, one)) return false;
    }
    return false;
}

}  // namespace gbbig28
