// gb_bignum28.h -- fixed-width multi-limb integers with 28-bit limbs (K
// little-endian limbs, each held in the low 28 bits of a 32-bit word) and the
// strong probable-prime test on them, for the minimal Goldbach prime of even
// n beyond 64 bits (paper section "Arbitrary Precision Checker", which tests
// q = n - p with Miller-Rabin).
//
// Montgomery multiplication (Montgomery 1985) with R = 2^(28K) in the finely
// integrated product-scanning order (Koc, Acar and Kaliski 1996).  With
// 28-bit limbs a product is below 2^56 and a column of at most 2K + 1 <= 33
// products plus the carry from the column before stays below 2^62, so a
// column sums in one 64-bit accumulator: one 64-bit multiply-add per limb
// product and no carry handling.  Host and device: the same code runs in a
// lane or on the CPU.
#pragma once
#include <cstdint>

namespace gbbig28 {

constexpr uint32_t kBits = 28;
constexpr uint32_t kMask = (1u << kBits) - 1u;

template <int K> struct Num {
    uint32_t w[K];
};

// -m^(-1) mod 2^28 for odd m, by Newton's iteration x <- x (2 - m x)
__host__ __device__ inline uint32_t neg_inv28(uint32_t m)
{
    uint32_t x = m;
    for (int i = 0; i < 4; ++i) x *= 2u - m * x;
    return (0u - x) & kMask;
}

template <int K> __host__ __device__ inline bool geq(const Num<K> &a, const Num<K> &b)
{
    for (int i = K - 1; i >= 0; --i)
        if (a.w[i] != b.w[i]) return a.w[i] > b.w[i];
    return true;
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

// (2a) mod m for a < m
template <int K> __host__ __device__ inline void dbl_mod(Num<K> &a, const Num<K> &m)
{
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const uint32_t t = (a.w[i] << 1) | c;
        c = t >> kBits;
        a.w[i] = t & kMask;
    }
    if (c || geq(a, m)) sub(a, a, m);
}

// (a + b) mod m for a, b < m
template <int K> __host__ __device__ inline void add_mod(Num<K> &a, const Num<K> &b, const Num<K> &m)
{
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const uint32_t t = a.w[i] + b.w[i] + c;
        c = t >> kBits;
        a.w[i] = t & kMask;
    }
    if (c || geq(a, m)) sub(a, a, m);
}

// a b R^(-1) mod m for a, b < m < R, m odd: column i collects every
// a_j b_(i-j) and u_j m_(i-j); the low columns choose u_i = t ninv mod 2^28 so
// that the column's low 28 bits become zero, the high columns are the result.
// Fully unrolled, so every limb stays in a register.
template <int K>
__host__ __device__ inline void mont_mul(Num<K> &r, const Num<K> &a, const Num<K> &b, const Num<K> &m, uint32_t ninv)
{
    static_assert(K <= 16, "a column of 2K + 1 products must stay below 2^64");
    uint64_t t = 0;
    uint32_t u[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
#pragma unroll
        for (int j = 0; j < i; ++j) {
            t += (uint64_t)a.w[j] * b.w[i - j];
            t += (uint64_t)u[j] * m.w[i - j];
        }
        t += (uint64_t)a.w[i] * b.w[0];
        u[i] = ((uint32_t)t * ninv) & kMask;
        t += (uint64_t)u[i] * m.w[0];                // the low 28 bits are now zero
        t >>= kBits;
    }
    Num<K> s;
#pragma unroll
    for (int i = K; i < 2 * K; ++i) {
#pragma unroll
        for (int j = i - K + 1; j < K; ++j) {
            t += (uint64_t)a.w[j] * b.w[i - j];
            t += (uint64_t)u[j] * m.w[i - j];
        }
        s.w[i - K] = (uint32_t)t & kMask;
        t >>= kBits;
    }
    // (t, s) < 2m: one conditional subtraction
    Num<K> d;
    const uint32_t br = sub(d, s, m);
    const bool keep = (uint32_t)t == 0u && br != 0u;   // below m
#pragma unroll
    for (int i = 0; i < K; ++i) r.w[i] = keep ? s.w[i] : d.w[i];
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

template <int K> __host__ __device__ inline uint32_t bit(const Num<K> &a, int i)
{
    const int j = i / (int)kBits;
    return (limb_at(a, j) >> (i - j * (int)kBits)) & 1u;
}

// R mod q, q odd with nb bits: 2^(nb-1) < q doubled 28K - nb + 1 times
template <int K> __host__ __device__ inline void mont_one(Num<K> &one, const Num<K> &q, int nb)
{
    const int top = (nb - 1) / (int)kBits;
#pragma unroll
    for (int i = 0; i < K; ++i) one.w[i] = (i == top) ? 1u << (nb - 1 - top * (int)kBits) : 0u;
    for (int i = nb - 1; i < (int)kBits * K; ++i) dbl_mod(one, q);
}

// The end of the strong test: with x = a^d R mod q, true when a^d = 1 or -1,
// or a^(d 2^r) = -1 for some 0 < r < s.  R mod q and q - R mod q are formed
// here, after the exponentiation, so that they hold no registers during it.
template <int K> __host__ __device__ inline bool strong_tail(Num<K> &x, const Num<K> &q, uint32_t ninv, int nb, int s)
{
    Num<K> one, mone;
    mont_one(one, q, nb);
    sub(mone, q, one);
    if (equal(x, one) || equal(x, mone)) return true;
    for (int r = 1; r < s; ++r) {
        mont_mul(x, x, x, q, ninv);
        if (equal(x, mone)) return true;
        if (equal(x, one)) return false;
    }
    return false;
}

// Strong probable prime to base 2, q odd, 2 < q < R: with q - 1 = d 2^s (d
// odd), 2^d = 1 or 2^(d 2^r) = -1 mod q for an r < s.  Left to right in
// Montgomery form; each multiplication by the base is a modular doubling
// (2 x R mod q from x R mod q), so one squaring per exponent bit.
template <int K> __host__ __device__ inline bool strong_prp2(const Num<K> &q)
{
    const uint32_t ninv = neg_inv28(q.w[0]);
    const int nb = bit_length(q);
    int s = 1;
    while (s < (int)kBits * K && bit(q, s) == 0u) ++s;   // q odd: ends below nb
    if (s >= (int)kBits * K) return false;
    const int db = nb - s;                           // bit i of d is bit i + s of q
    Num<K> x;
    mont_one(x, q, nb);
    dbl_mod(x, q);                                   // 2R: the top bit of d
    for (int i = db - 2; i >= 0; --i) {
        mont_mul(x, x, x, q, ninv);
        if (bit(q, i + s)) dbl_mod(x, q);
    }
    return strong_tail(x, q, ninv, nb, s);
}

// Strong probable prime to a small base a (2 <= a < 2^28, a < q).  The
// exponentiation has one Montgomery product call site (the multiplier
// selected), so the code stays small.
template <int K> __host__ __device__ inline bool strong_prp(const Num<K> &q, uint32_t a)
{
    const uint32_t ninv = neg_inv28(q.w[0]);
    const int nb = bit_length(q);
    int s = 1;
    while (s < (int)kBits * K && bit(q, s) == 0u) ++s;
    if (s >= (int)kBits * K) return false;
    const int db = nb - s;
    // am = a R mod q, by doubling and adding R mod q
    Num<K> am;
    {
        Num<K> one;
        mont_one(one, q, nb);
#pragma unroll
        for (int i = 0; i < K; ++i) am.w[i] = 0;
        for (int i = (int)kBits - 1; i >= 0; --i) {
            dbl_mod(am, q);
            if ((a >> i) & 1u) add_mod(am, one, q);
        }
    }
    Num<K> x = am;
    int i = db - 2;
    bool mul_next = false;
    while (i >= 0 || mul_next) {
        Num<K> y;
#pragma unroll
        for (int j = 0; j < K; ++j) y.w[j] = mul_next ? am.w[j] : x.w[j];
        mont_mul(x, x, y, q, ninv);
        if (mul_next) {
            mul_next = false;
            --i;
        } else if (bit(q, i + s)) {
            mul_next = true;
        } else {
            --i;
        }
    }
    return strong_tail(x, q, ninv, nb, s);
}

}  // namespace gbbig28
