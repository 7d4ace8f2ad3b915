// gb_bignum.h -- fixed-width multi-limb integers (K little-endian 32-bit
// limbs) and the strong probable-prime test on them, for the minimal Goldbach
// prime of even n beyond 64 bits (paper section "Arbitrary Precision
// Checker", which tests q = n - p with Miller-Rabin), used for n of 449 bits
// and more (32 limbs).  Montgomery multiplication (Montgomery 1985) with
// R = 2^(32K) in the coarsely integrated operand-scanning order (Koc, Acar
// and Kaliski 1996).  Host and device: the same code runs in a lane or on the
// CPU.
#pragma once
#include <cstdint>

namespace gbbig {

template <int K> struct Num {
    uint32_t w[K];
};

// -m^(-1) mod 2^32 for odd m, by Newton's iteration x <- x (2 - m x)
// (each step doubles the number of correct low bits; m is correct to 3).
__host__ __device__ inline uint32_t neg_inv32(uint32_t m)
{
    uint32_t x = m;
    for (int i = 0; i < 4; ++i) x *= 2u - m * x;
    return 0u - x;
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
    for (int i = 0; i < K; ++i) d |= a.w[i] ^ b.w[i];
    return d == 0;
}

// a - b, returns the borrow
template <int K> __host__ __device__ inline uint32_t sub(Num<K> &r, const Num<K> &a, const Num<K> &b)
{
    uint64_t br = 0;
    for (int i = 0; i < K; ++i) {
        const uint64_t t = (uint64_t)a.w[i] - b.w[i] - br;
        r.w[i] = (uint32_t)t;
        br = (t >> 63) & 1u;
    }
    return (uint32_t)br;
}

// (2a) mod m for a < m
template <int K> __host__ __device__ inline void dbl_mod(Num<K> &a, const Num<K> &m)
{
    uint32_t top = a.w[K - 1] >> 31;
    for (int i = K - 1; i > 0; --i) a.w[i] = (a.w[i] << 1) | (a.w[i - 1] >> 31);
    a.w[0] <<= 1;
    if (top || geq(a, m)) sub(a, a, m);
}

// (a + b) mod m for a, b < m
template <int K> __host__ __device__ inline void add_mod(Num<K> &a, const Num<K> &b, const Num<K> &m)
{
    uint64_t c = 0;
    for (int i = 0; i < K; ++i) {
        c += (uint64_t)a.w[i] + b.w[i];
        a.w[i] = (uint32_t)c;
        c >>= 32;
    }
    if (c || geq(a, m)) sub(a, a, m);
}

// a b R^(-1) mod m for a, b < m < R, m odd, in the coarsely integrated
// operand-scanning order: one row of K multiply-adds per limb of b.
template <int K>
__host__ __device__ inline void mont_mul(Num<K> &r, const Num<K> &a, const Num<K> &b, const Num<K> &m, uint32_t ninv)
{
    // fully unrolled, so that every limb stays in a register
    uint32_t t[K + 2];
#pragma unroll
    for (int i = 0; i < K + 2; ++i) t[i] = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        uint64_t c = 0;
        const uint32_t bi = b.w[i];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            c = (uint64_t)a.w[j] * bi + t[j] + (c >> 32);
            t[j] = (uint32_t)c;
        }
        c = (uint64_t)t[K] + (c >> 32);
        t[K] = (uint32_t)c;
        t[K + 1] = (uint32_t)(c >> 32);
        const uint32_t q = t[0] * ninv;
        c = (uint64_t)q * m.w[0] + t[0];
#pragma unroll
        for (int j = 1; j < K; ++j) {
            c = (uint64_t)q * m.w[j] + t[j] + (c >> 32);
            t[j - 1] = (uint32_t)c;
        }
        c = (uint64_t)t[K] + (c >> 32);
        t[K - 1] = (uint32_t)c;
        t[K] = t[K + 1] + (uint32_t)(c >> 32);
    }
    // t < 2m: one conditional subtraction
    Num<K> s;
    uint64_t br = 0;
    for (int i = 0; i < K; ++i) {
        const uint64_t d = (uint64_t)t[i] - m.w[i] - br;
        s.w[i] = (uint32_t)d;
        br = (d >> 63) & 1u;
    }
    const bool keep = t[K] == 0u && br != 0u;   // t < m
    for (int i = 0; i < K; ++i) r.w[i] = keep ? t[i] : s.w[i];
}

template <int K> __host__ __device__ inline int bit_length(const Num<K> &a)
{
    for (int i = K - 1; i >= 0; --i)
        if (a.w[i]) return 32 * i + 32 - __builtin_clz(a.w[i]);
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
    return (limb_at(a, i >> 5) >> (i & 31)) & 1u;
}

// Strong probable prime to base a (2 <= a < q), q odd, q < R = 2^(32K):
// with q - 1 = d 2^s (d odd), a^d = 1 or a^(d 2^r) = -1 mod q for an r < s.
// Exponentiation in Montgomery form, left to right.
template <int K> __host__ __device__ inline bool strong_prp(const Num<K> &q, uint32_t a)
{
    const uint32_t ninv = neg_inv32(q.w[0]);
    const int nb = bit_length(q);
    // one = R mod q: 2^(nb-1) < q doubled 32K - nb + 1 times
    Num<K> one;
#pragma unroll
    for (int i = 0; i < K; ++i) one.w[i] = (i == ((nb - 1) >> 5)) ? 1u << ((nb - 1) & 31) : 0u;
    for (int i = nb - 1; i < 32 * K; ++i) dbl_mod(one, q);
    // am = a R mod q (a < 2^7 in use; any 32-bit a works), by doubling and adding
    Num<K> am;
    for (int i = 0; i < K; ++i) am.w[i] = 0;
    for (int i = 31; i >= 0; --i) {
        dbl_mod(am, q);
        if ((a >> i) & 1u) add_mod(am, one, q);
    }
    Num<K> mone;                      // (q - 1) R mod q = q - one
    sub(mone, q, one);
    // s = number of trailing zeros of q - 1; d = (q - 1) >> s: bit i of d is
    // bit i + s of q (q odd, so q - 1 differs from q only in bit 0)
    int s = 1;
    while (s < 32 * K && bit(q, s) == 0u) ++s;   // q odd: ends below nb
    if (s >= 32 * K) return false;
    const int db = nb - s;            // bit length of d
    // x = a^d: start from the top bit of d (= aR), then for bits db-2 .. 0
    // one squaring each and one multiplication for each set bit; then up to
    // s - 1 more squarings.  One Montgomery product per step, with its second
    // operand selected, so the product is inlined once.
    Num<K> x = am;
    int i = db - 2;
    bool mul_next = false;
    int r = 0;                        // squarings after the exponentiation
    for (;;) {
        const bool expo = i >= 0 || mul_next;
        if (!expo) {
            if (r == 0) {
                if (equal(x, one) || equal(x, mone)) return true;
            } else {
                if (equal(x, mone)) return true;
                if (equal(x, one)) return false;
            }
            if (++r >= s) return false;
        }
        Num<K> y;
#pragma unroll
        for (int j = 0; j < K; ++j) y.w[j] = mul_next ? am.w[j] : x.w[j];
        mont_mul(x, x, y, q, ninv);
        if (expo) {
            if (mul_next) {
                mul_next = false;
                --i;
            } else if (bit(q, i + s)) {
                mul_next = true;
            } else {
                --i;
            }
        }
    }
}

}  // namespace gbbig
