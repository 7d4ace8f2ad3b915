// gb_bignum.h -- fixed-width multi-limb integers (K little-endian 32-bit
// limbs) and the strong probable-prime test on them, for the minimal Goldbach
// prime of even n beyond 64 bits (paper section "Arbitrary Precision
// Checker", which tests q = n - p with Miller-Rabin).  Montgomery
// multiplication (Montgomery 1985) with R = 2^(32K), in the finely integrated
// product-scanning order and, for the 32-limb kernel, the coarsely integrated
// operand-scanning order (Koc, Acar and Kaliski 1996).  Host and device: the
// same code runs in a lane or on the CPU (the multiply-add with carry is one
// instruction pair on the GPU, plain 64-bit arithmetic on the host).
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

// Column accumulator of the product-scanning form: 96 bits, (hi, lo).
struct Acc {
    uint64_t lo;
    uint32_t hi;
};

// t += x y.  On the GPU one 64-bit multiply-add whose carry-out feeds one
// add-with-carry into the top word.
__host__ __device__ inline void mac(Acc &t, uint32_t x, uint32_t y)
{
#if defined(__HIP_DEVICE_COMPILE__)
    uint64_t cc;
    asm("v_mad_u64_u32 %0, %2, %3, %4, %0\n\tv_addc_co_u32_e64 %1, %2, %1, 0, %2"
        : "+v"(t.lo), "+v"(t.hi), "=&s"(cc)
        : "v"(x), "v"(y));
#else
    const uint64_t p = (uint64_t)x * y + t.lo;
    t.hi += p < t.lo ? 1u : 0u;
    t.lo = p;
#endif
}

// a b R^(-1) mod m for a, b < m < R, m odd.  Montgomery multiplication in
// the finely integrated product-scanning order (Koc, Acar and Kaliski 1996):
// column i collects every a_j b_(i-j) and u_j m_(i-j) in one accumulator, the
// low columns choose u_i = t ninv mod 2^32 so that the column becomes zero,
// and the high columns are the result.  Fully unrolled, so every limb stays
// in a register; two instructions per multiply-add on the GPU.
template <int K>
__host__ __device__ inline void mont_mul(Num<K> &r, const Num<K> &a, const Num<K> &b, const Num<K> &m, uint32_t ninv)
{
    Acc t = {0, 0};
    uint32_t u[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
#pragma unroll
        for (int j = 0; j < i; ++j) {
            mac(t, a.w[j], b.w[i - j]);
            mac(t, u[j], m.w[i - j]);
        }
        mac(t, a.w[i], b.w[0]);
        u[i] = (uint32_t)t.lo * ninv;
        mac(t, u[i], m.w[0]);                        // the low word is now zero
        t.lo = (t.lo >> 32) | ((uint64_t)t.hi << 32);
        t.hi = 0;
    }
    Num<K> s;
#pragma unroll
    for (int i = K; i < 2 * K; ++i) {
#pragma unroll
        for (int j = i - K + 1; j < K; ++j) {
            mac(t, a.w[j], b.w[i - j]);
            mac(t, u[j], m.w[i - j]);
        }
        s.w[i - K] = (uint32_t)t.lo;
        t.lo = (t.lo >> 32) | ((uint64_t)t.hi << 32);
        t.hi = 0;
    }
    // (t.lo, s) < 2m: one conditional subtraction
    Num<K> d;
    uint64_t br = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const uint64_t x = (uint64_t)s.w[i] - m.w[i] - br;
        d.w[i] = (uint32_t)x;
        br = (x >> 63) & 1u;
    }
    const bool keep = (uint32_t)t.lo == 0u && br != 0u;   // below m
#pragma unroll
    for (int i = 0; i < K; ++i) r.w[i] = keep ? s.w[i] : d.w[i];
}

// The same product in the coarsely integrated operand-scanning order
// (Montgomery 1985; Koc, Acar and Kaliski 1996), one row of K multiply-adds
// per limb of b; kept for the 32-limb kernel, whose device code was checked
// in this form.
template <int K>
__host__ __device__ inline void mont_mul_cios(Num<K> &r, const Num<K> &a, const Num<K> &b, const Num<K> &m, uint32_t ninv)
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
template <int K, bool CIOS = false> __host__ __device__ inline bool strong_prp(const Num<K> &q, uint32_t a)
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
        if constexpr (CIOS)
            mont_mul_cios(x, x, y, q, ninv);
        else
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

// Strong probable prime to base 2, as strong_prp, with each multiplication
// by the base done as a modular doubling (2 x R mod q from x R mod q): one
// Montgomery squaring per exponent bit and no general product.  R mod q and
// q - R mod q are formed only after the exponentiation, so that they hold no
// registers during it.
template <int K> __host__ __device__ inline bool strong_prp2(const Num<K> &q)
{
    const uint32_t ninv = neg_inv32(q.w[0]);
    const int nb = bit_length(q);
    int s = 1;
    while (s < 32 * K && bit(q, s) == 0u) ++s;   // q odd: ends below nb
    if (s >= 32 * K) return false;
    const int db = nb - s;
    // x = 2^d R: the top bit of d gives 2R; each lower bit one squaring, then
    // a doubling for a set bit
    Num<K> x;
#pragma unroll
    for (int i = 0; i < K; ++i) x.w[i] = (i == ((nb - 1) >> 5)) ? 1u << ((nb - 1) & 31) : 0u;
    for (int i = nb - 1; i <= 32 * K; ++i) dbl_mod(x, q);
    for (int i = db - 2; i >= 0; --i) {
        mont_mul(x, x, x, q, ninv);
        if (bit(q, i + s)) dbl_mod(x, q);
    }
    Num<K> one, mone;
#pragma unroll
    for (int i = 0; i < K; ++i) one.w[i] = (i == ((nb - 1) >> 5)) ? 1u << ((nb - 1) & 31) : 0u;
    for (int i = nb - 1; i < 32 * K; ++i) dbl_mod(one, q);
    sub(mone, q, one);
    if (equal(x, one) || equal(x, mone)) return true;
    for (int r = 1; r < s; ++r) {
        mont_mul(x, x, x, q, ninv);
        if (equal(x, mone)) return true;
        if (equal(x, one)) return false;
    }
    return false;
}

}  // namespace gbbig
