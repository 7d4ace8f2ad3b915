// bignum_host.cpp -- host build of the GPU's multi-limb header
// (gb_bignum28.h: 28-bit limbs) for the CPU tests.  The header is written
// for both sides; compiled here with g++ (and the sanitizers), the same
// Montgomery squarings, small multiplications and strong tests run on the
// CPU, so their arithmetic can be checked against Python integers and the
// big-n oracle without a GPU.
//
// Commands on stdin, one per line, answers on stdout (K: limbs of 28 bits,
// R = 2^(28 K)):
//   sqr  K m a          -> "r rn": r = the lazy a^2 R^-1 mod m (a < 2m;
//                          r < 2m), rn = r mod m
//   mulsmall K m x f    -> "r rn": r = the lazy x f mod m (x < 2m,
//                          f <= 2^20; r < 1.19 m), rn = r mod m
//   one  K m            -> R mod m
//   sprp K q a          -> 1 if q is a strong probable prime to base a, else 0
//   pmin K n            -> "p groups tests": the minimal p the GPU search
//                          returns for n (odd primes p ascending, p = n mod r
//                          dropped for the 24 odd bases r, q = n - p tested to
//                          base 2, then to the other 24 bases), the groups of
//                          64 table entries the filter read and the base-2
//                          tests it ran
//   pmin_nobase2 K n    -> the same search when every base-2 test fails (the
//                          trip counts of a search that never finds a
//                          candidate: the whole table)
// Numbers are hexadecimal without a prefix.
#define __host__
#define __device__
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <iostream>
#include <sstream>
#include <string>
#include <type_traits>
#include <vector>

#include "../paper_2603_02621_amd/csrc/gb_bignum28.h"

namespace {

const uint32_t kBases[25] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41,
                             43, 47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97};

// little-endian bits of a hexadecimal string
std::vector<uint8_t> hex_bits(const std::string &h)
{
    std::vector<uint8_t> b;
    for (size_t i = h.size(); i-- > 0;) {
        const char ch = h[i];
        const int v = ch <= '9' ? ch - '0' : (ch | 32) - 'a' + 10;
        for (int k = 0; k < 4; ++k) b.push_back((uint8_t)((v >> k) & 1));
    }
    return b;
}

template <int K, int F, class N> N from_hex(const std::string &h)
{
    N x;
    for (int i = 0; i < K; ++i) x.w[i] = 0;
    const std::vector<uint8_t> b = hex_bits(h);
    for (size_t i = 0; i < b.size(); ++i)
        if (b[i]) {
            if (i >= (size_t)F * K) {
                std::fprintf(stderr, "number wider than %d limbs of %d bits\n", K, F);
                std::exit(2);
            }
            x.w[i / F] |= 1u << (i % F);
        }
    return x;
}

template <int K, int F, class N> std::string to_hex(const N &x)
{
    std::vector<uint8_t> b((size_t)F * K);
    for (int i = 0; i < F * K; ++i) b[i] = (x.w[i / F] >> (i % F)) & 1u;
    std::string s;
    for (int i = F * K - 4; i >= 0; i -= 4) {
        const int v = b[i] | b[i + 1] << 1 | b[i + 2] << 2 | b[i + 3] << 3;
        if (s.empty() && v == 0) continue;
        s += "0123456789abcdef"[v];
    }
    return s.empty() ? "0" : s;
}

std::vector<uint32_t> odd_primes(uint32_t limit)
{
    std::vector<uint8_t> comp(limit + 1, 0);
    std::vector<uint32_t> out;
    for (uint64_t i = 3; i <= limit; i += 2) {
        if (comp[i]) continue;
        out.push_back((uint32_t)i);
        for (uint64_t j = i * i; j <= limit; j += 2 * i) comp[j] = 1;
    }
    return out;
}

// n mod r from the limbs, most significant first
template <int K, int F, class N> uint32_t mod_small(const N &n, uint32_t r)
{
    const uint32_t t = (uint32_t)((1ull << F) % r);
    uint32_t acc = 0;
    for (int i = K - 1; i >= 0; --i) acc = (acc * t + n.w[i] % r) % r;
    return acc;
}

template <int K, int F, class N> N sub_p(const N &n, uint32_t p)
{
    // schoolbook subtraction of a 32-bit p
    N q;
    const uint64_t mask = F == 32 ? 0xFFFFFFFFull : (1ull << F) - 1;
    uint64_t borrow = 0, pp = p;
    for (int i = 0; i < K; ++i) {
        const uint64_t pi = pp & mask;
        pp >>= F;
        const int64_t d = (int64_t)n.w[i] - (int64_t)pi - (int64_t)borrow;
        borrow = d < 0;
        q.w[i] = (uint32_t)((uint64_t)d & mask);
    }
    return q;
}

template <int K> void run(const std::string &cmd, std::istringstream &in)
{
    constexpr int F = 28;
    using N = gbbig28::Num<K>;
    if (cmd == "sqr" || cmd == "mulsmall" || cmd == "one") {
        std::string m, a;
        uint32_t f = 0;
        in >> m;
        if (cmd != "one") in >> a;
        if (cmd == "mulsmall") in >> f;
        const N M = from_hex<K, F, N>(m);
        N r = cmd == "one" ? M : from_hex<K, F, N>(a);
        if (cmd == "sqr") {
            gbbig28::mont_sqr<K>(r, r, M, gbbig28::neg_inv28(M.w[0]));
        } else if (cmd == "mulsmall") {
            gbbig28::mul_small<K>(r, f, M, gbbig28::est_recip<K>(M));
        } else {
            gbbig28::mont_one<K>(r, M, gbbig28::bit_length<K>(M), gbbig28::est_recip<K>(M));
            std::cout << to_hex<K, F, N>(r) << "\n";
            return;
        }
        N rn = r;
        // r < 2m is part of the contract; rn is r reduced once
        gbbig28::reduce_once<K>(rn, M);
        std::cout << to_hex<K, F, N>(r) << " " << to_hex<K, F, N>(rn) << "\n";
    } else if (cmd == "sprp") {
        std::string q;
        uint32_t a;
        in >> q >> a;
        const N Q = from_hex<K, F, N>(q);
        std::cout << (gbbig28::strong_prp<K>(Q, a) ? 1 : 0) << "\n";
    } else if (cmd == "pmin" || cmd == "pmin_nobase2") {
        static const std::vector<uint32_t> primes = odd_primes(1u << 22);
        std::string h;
        in >> h;
        const N n = from_hex<K, F, N>(h);
        uint32_t res[24];
        for (int j = 0; j < 24; ++j) res[j] = mod_small<K, F, N>(n, kBases[j + 1]);
        const bool nob2 = cmd == "pmin_nobase2";
        uint64_t groups = 0, tests = 0;
        uint32_t ans = 0;
        for (size_t c = 0; c < primes.size() && !ans; ++c) {
            if (c % 64 == 0) ++groups;
            const uint32_t p = primes[c];
            bool drop = false;
            for (int j = 0; j < 24; ++j) drop = drop || p % kBases[j + 1] == res[j];
            if (drop) continue;
            const N q = sub_p<K, F, N>(n, p);
            ++tests;
            if (nob2 || !gbbig28::strong_prp<K>(q, 2u)) continue;
            bool ok = true;
            for (int j = 1; j < 25 && ok; ++j) ok = gbbig28::strong_prp<K>(q, kBases[j]);
            if (ok) ans = p;
        }
        std::cout << ans << " " << groups << " " << tests << "\n";
    } else {
        std::fprintf(stderr, "unknown command %s\n", cmd.c_str());
        std::exit(2);
    }
}

}  // namespace

int main()
{
    std::string line;
    while (std::getline(std::cin, line)) {
        std::istringstream in(line);
        std::string cmd;
        int K = 0;
        in >> cmd >> K;
        switch (K) {
        case 4: run<4>(cmd, in); break;
        case 6: run<6>(cmd, in); break;
        case 8: run<8>(cmd, in); break;
        case 10: run<10>(cmd, in); break;
        case 12: run<12>(cmd, in); break;
        case 14: run<14>(cmd, in); break;
        case 16: run<16>(cmd, in); break;
        case 20: run<20>(cmd, in); break;
        case 24: run<24>(cmd, in); break;
        case 28: run<28>(cmd, in); break;
        case 32: run<32>(cmd, in); break;
        case 36: run<36>(cmd, in); break;
        case 37: run<37>(cmd, in); break;
        default: std::fprintf(stderr, "no form with %d limbs\n", K); return 2;
        }
        std::cout.flush();
    }
    return 0;
}
