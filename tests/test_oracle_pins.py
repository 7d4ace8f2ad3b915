"""Pins for the CPU oracle: every check compares it with something that is
not the oracle -- trial division written here, SymPy's primality routines,
prime counts from the literature, the counts the paper prints, and strong
pseudoprimes published in the Miller-Rabin literature.

A plausible mistake anywhere in the oracle (a dropped prime, a window off by
one, a wrong MR base, a mis-ordered scan, a summary with a wrong weight or a
wrong tie-break) fails at least one of these.
"""
import os
import random

import numpy as np
import pytest
import sympy
from sympy.ntheory.primetest import mr as sympy_mr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.txt")


def _golden():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                kind, arg, val, _src = line.split()
                rows.append((kind, int(arg), int(val)))
    return rows


# --------------------------------------------------------------------------
# independent brute force: trial division only
# --------------------------------------------------------------------------

def _td_prime_table(limit):
    """is_prime[x] for 0 <= x <= limit by trial division of each x."""
    tab = [False] * (limit + 1)
    for x in range(2, limit + 1):
        d, ok = 2, True
        while d * d <= x:
            if x % d == 0:
                ok = False
                break
            d += 1
        tab[x] = ok
    return tab


def _td_pmin(n, tab):
    for p in range(2, n // 2 + 1):
        if tab[p] and tab[n - p]:
            return p
    return 0


@pytest.fixture(scope="module")
def td_table():
    return _td_prime_table(100_000)


# --------------------------------------------------------------------------
# prime counts
# --------------------------------------------------------------------------

def test_pi_paper_value(orc):
    for kind, arg, val in _golden():
        if kind == "pi":
            assert orc.prime_count(arg) == val


@pytest.mark.parametrize("x,pi", [
    (10**7, 664_579), (10**8, 5_761_455),
    (2**10, 172), (2**13, 1028), (2**16, 6542), (31_622, 3401), (1, 0), (2, 1), (3, 2),
])
def test_pi_known(orc, x, pi):
    # classical prime counts; the small ones re-derived with SymPy below
    assert orc.prime_count(x) == pi
    if x <= 10**7:
        assert sympy.primepi(x) == pi


@pytest.mark.slow
def test_pi_1e9(orc):
    assert orc.prime_count(10**9) == 50_847_534


# --------------------------------------------------------------------------
# primality predicates
# --------------------------------------------------------------------------

def test_trial_division_vs_sympy(orc):
    for q in list(range(0, 3000)) + [10**12 - 11, 10**12 + 39, 999_999_999_989]:
        assert orc.trial_is_prime(q) == sympy.isprime(q), q


STRONG_PSP = [
    # (n, bases it passes, base that exposes it) -- Pomerance, Selfridge and
    # Wagstaff (1980); Jaeschke (1993); Zhang and Tang (2003).
    (2047, [2], 3),
    (1373653, [2, 3], 5),
    (25326001, [2, 3, 5], 7),
    (3215031751, [2, 3, 5, 7], 11),
    (2152302898747, [2, 3, 5, 7, 11], 13),
    (3474749660383, [2, 3, 5, 7, 11, 13], 17),
    (341550071728321, [2, 3, 5, 7, 11, 13, 17, 19], 23),
    (3825123056546413051, [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31], 37),
]


@pytest.mark.parametrize("n,passes,fails", STRONG_PSP)
def test_strong_pseudoprimes(orc, n, passes, fails):
    assert not sympy.isprime(n)
    for a in passes:
        assert orc.mr_base(n, a), (n, a)
    assert not orc.mr_base(n, fails)
    assert not orc.mr(n)
    # each single-base verdict also agrees with SymPy's strong test
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        assert orc.mr_base(n, a) == sympy_mr(n, [a]), (n, a)


@pytest.mark.parametrize("p", [2**61 - 1, 2**63 - 25, 2**64 - 59, 2**31 - 1,
                               1_000_000_000_039, 999_999_999_989])
def test_mr_known_primes(orc, p):
    assert sympy.isprime(p)
    assert orc.mr(p)
    assert orc.is_prime(p)


@pytest.mark.parametrize("c", [2**64 - 1, 2**63 - 1, 561, 1105, 1729, 2465, 2821, 6601,
                               8911, 4, 9, 25, 49, 121, 1, 0])
def test_mr_known_composites(orc, c):
    assert not orc.mr(c)


def test_mr_vs_sympy_random(orc):
    rng = random.Random(12345)
    for _ in range(20_000):
        q = rng.getrandbits(64) | 1
        assert orc.mr(q) == sympy.isprime(q), q
    for _ in range(300):
        p = sympy.randprime(2**40, 2**64)
        assert orc.mr(p)


def test_mr_vs_trial_small(orc, td_table):
    for q in range(0, 100_001):
        assert orc.mr(q) == td_table[q], q


# --------------------------------------------------------------------------
# p_min per n
# --------------------------------------------------------------------------

def test_pmin_bruteforce_1e5(orc, td_table):
    out, hist, s = orc.verify_range(4, 100_000, per_n_bits=32)
    ref = np.array([_td_pmin(n, td_table) for n in range(4, 100_001, 2)], dtype=np.uint32)
    assert np.array_equal(out, ref)
    assert s["count"] == len(ref)
    assert s["n_failed"] == 0


def _weight(n):
    """Checksum weight of n: 2^33 b + (2c+1) 2^i with b = 3 floor(n/384) +
    (n mod 6)/2 and j = floor(n/6) mod 64 = 32c + i."""
    b = 3 * (n // 384) + (n % 6) // 2
    c, i = divmod((n // 6) % 64, 32)
    return ((b << 33) + ((2 * c + 1) << i)) % 2**64


def _summaries_by_hand(ns, ps, pmax):
    """Summary definitions written out directly over (n, p) pairs."""
    hist = np.zeros(6543, dtype=np.uint64)
    cs, mx, arg, nex = 0, 0, 0, 0
    for n, p in zip(ns, ps):
        b = sympy.primepi(p) - 1 if p < 65536 else 6542
        hist[b] += 1
        cs = (cs + _weight(n) * p) % 2**64
        if p > mx:
            mx, arg = p, n
        if p > pmax:
            nex += 1
    return hist, dict(count=len(ns), checksum=cs, max_p=mx, argmax_n=arg, n_exhaustive=nex)


@pytest.mark.parametrize("lo,hi,pmax", [(4, 20_000, 8192), (1_001, 19_999, 7), (4, 4, 8192),
                                        (6, 6, 3), (5_000, 9_000, 13)])
def test_summaries_bruteforce(orc, td_table, lo, hi, pmax):
    out, hist, s = orc.verify_range(lo, hi, pmax=pmax, per_n_bits=32)
    a = max(lo, 4) + (max(lo, 4) & 1)
    ns = list(range(a, hi - (hi & 1) + 1, 2))
    ps = [_td_pmin(n, td_table) for n in ns]
    h, ref = _summaries_by_hand(ns, ps, pmax)
    assert np.array_equal(hist, h)
    for k, v in ref.items():
        assert s[k] == v, k
    # consistency identities
    assert int(hist.sum()) == s["count"]


def _v2(x):
    x %= 2**64
    return 64 if x == 0 else (x & -x).bit_length() - 1


def test_checksum_weight_definition(orc):
    rng = np.random.default_rng(11)
    ns = [4, 6, 8, 126, 128, 130, 254, 256, 382, 384, 386, 388, 2**63, 2**63 - 2] + \
        [int(x) * 2 for x in rng.integers(2, 2**62, size=2000)]
    for n in ns:
        assert orc.checksum_weight(n) == _weight(n), n


def test_checksum_detects_single_and_swapped_errors():
    # a wrong p_min changes p by an even delta with |delta| < 2^16, i.e. at
    # most 15 factors of 2: the change delta * w(n) is nonzero mod 2^64
    # because w(n) has exactly floor(n/6) mod 32 <= 31 of them
    rng = np.random.default_rng(12)
    for n in [int(x) * 2 for x in rng.integers(2, 2**62, size=4000)] + list(range(4, 1 << 14, 2)):
        assert _v2(_weight(n)) == (n // 6) % 32, n
    # two n exchanging their p change the sum by (p1 - p2) (w1 - w2), and
    # p1 - p2 has at most 15 factors of 2.  Within 16 stretches of 384 (16
    # sets of 64 n of each class) w1 - w2 has at most 38 of them (the same
    # place j in sets whose b differ by 32)...
    worst = 0
    for base in (0, 10**12 - 2**36, 2**62, 2**63 - 6144):
        base -= base % 384
        ws = [_weight(base + 2 * k) for k in range(3072)]
        for a in range(0, 3072, 11):
            for b in range(a + 1, 3072):
                worst = max(worst, _v2(ws[a] - ws[b]))
    assert worst == 38
    # ...and for n closer than 8 million the b differ by less than 2^16, so
    # w1 - w2 has at most 33 + 15 factors of 2: every such exchange is seen
    for _ in range(20000):
        n1 = int(rng.integers(2, 2**62)) * 2
        n2 = n1 + 2 * int(rng.integers(1, 4_000_000))
        if n2 >= 2**64:
            continue
        b1 = 3 * (n1 // 384) + (n1 % 6) // 2
        b2 = 3 * (n2 // 384) + (n2 % 6) // 2
        assert abs(b1 - b2) < 2**16
        assert _v2(_weight(n1) - _weight(n2)) <= 48


def test_config1_summary(orc):
    # every even n in [4, 10^6]: 499,999 of them; maximum p_min is 523,
    # first reached at n = 503,222 -- re-checked with SymPy here
    out, hist, s = orc.verify_range(4, 10**6, per_n_bits=32)
    assert s["count"] == 499_999 and s["n_failed"] == 0
    n = s["argmax_n"]
    p = s["max_p"]
    assert sympy.isprime(p) and sympy.isprime(n - p)
    assert all(not sympy.isprime(n - r) for r in sympy.primerange(2, p))
    assert int(out.max()) == p and 4 + 2 * int(np.argmax(out)) == n


def _check_minimal(n, p):
    assert p >= 2 and sympy.isprime(p) and sympy.isprime(n - p), (n, p)
    for r in sympy.primerange(2, p):
        assert not sympy.isprime(n - r), (n, p, r)


@pytest.mark.parametrize("n", [10**6, 10**9, 10**12, 10**15, 2**62, 2**63, 2**63 - 2,
                               10**12 - 2**36, 4, 6, 8, 2**64 - 2])
def test_verify_one_minimal(orc, n):
    p = orc.verify_one(n)
    _check_minimal(n, p)


def test_verify_one_random(orc):
    rng = np.random.default_rng(7)
    ns = [2 * int(x) for x in rng.integers(2, 2**62, size=200, endpoint=True)]
    ps = orc.verify_many(ns, threads=4)
    for n, p in zip(ns, ps):
        _check_minimal(n, int(p))


def test_verify_one_limit_reports_failure(orc):
    # 98 = 19 + 79 and no smaller prime works, so a scan bounded by 17 fails
    assert orc.verify_one(98) == 19
    assert orc.verify_one(98, limit=17) == 0
    assert orc.verify_one(7) == 0 and orc.verify_one(2) == 0


def test_window_near_1e12_matches_single_n(orc):
    lo, hi = 10**12 - 2**17, 10**12
    out, hist, s = orc.verify_range(lo, hi, per_n_bits=16)
    rng = np.random.default_rng(3)
    idx = rng.integers(0, len(out), size=300)
    for i in idx:
        n = lo + 2 * int(i)
        p = int(out[i])
        assert p == orc.verify_one(n)
        _check_minimal(n, p)
    assert s["count"] == 2**16 + 1


def test_multithread_equals_single(orc):
    lo, hi = 10**9 - 2**23, 10**9 + 2**22
    o1, h1, s1 = orc.verify_range(lo, hi, per_n_bits=16)
    o2, h2, s2 = orc.verify_range(lo, hi, per_n_bits=16, threads=5)
    assert np.array_equal(o1, o2) and np.array_equal(h1, h2) and s1 == s2


@pytest.mark.parametrize("w0", [10**12 - 1001, 1000003**2 - 2000, 2**53 - 2001, 1, 99_991])
def test_odd_primality_vs_sympy(orc, w0):
    # the byte sieve the GPU sieve is compared with, pinned directly: every
    # odd number of windows near 10^12, across 1000003^2 (the first square
    # of a sieving prime above 10^6) and across 2^53, against SymPy
    count = 2000
    got = orc.odd_primality(w0, count)
    want = [int(sympy.isprime(w0 + 2 * i)) for i in range(count)]
    assert got.tolist() == want


def test_windows_bruteforce_and_single_n(orc, td_table):
    # overlapping and ragged windows below 10^5 against trial division, and
    # windows near 10^12 and 10^15 (the serving workload's range starts)
    # against the Miller-Rabin scan of single n with SymPy minimality
    wins = [(4, 1), (4, 500), (98, 3), (1000, 777), (1002, 100), (99_000, 500), (50_000, 1)]
    out, sums = orc.verify_windows(wins, threads=3)
    o = 0
    for (start, ln), sm in zip(wins, sums):
        ref = [_td_pmin(start + 2 * i, td_table) for i in range(ln)]
        assert out[o:o + ln].tolist() == ref, start
        assert sm["count"] == ln and sm["n_failed"] == 0
        assert sm["max_p"] == max(ref)
        assert sm["argmax_n"] == start + 2 * ref.index(max(ref))
        assert sm["checksum"] == sum(_weight(start + 2 * i) * p for i, p in enumerate(ref)) % 2**64
        o += ln
    big = [(10**15 + 2 * 12345, 300), (10**12 - 2**17, 200), (2 * 10**14 + 6, 1)]
    out, sums = orc.verify_windows(big, threads=2)
    o = 0
    rng = np.random.default_rng(11)
    for (start, ln), sm in zip(big, sums):
        for i in rng.integers(0, ln, size=min(ln, 20)):
            n = start + 2 * int(i)
            assert int(out[o + int(i)]) == orc.verify_one(n)
        _check_minimal(start, int(out[o]))
        o += ln
    with pytest.raises(ValueError):
        orc.verify_windows([(7, 10)])


def test_paper_counts_small(orc):
    for kind, arg, val in _golden():
        if kind == "count" and arg <= 10**8:
            _, _, s = orc.verify_range(4, arg, per_n_bits=None, hist=False, threads=4)
            assert s["count"] == val
            assert s["n_failed"] == 0
        elif kind == "count":
            assert orc.n_even(4, arg) == val


@pytest.mark.slow
def test_paper_no_failures_1e9(orc):
    for kind, arg, val in _golden():
        if kind == "nofail":
            _, hist, s = orc.verify_range(4, arg, pmax=10**6, per_n_bits=None, threads=8)
            assert s["n_failed"] == val
            assert s["n_exhaustive"] == 0
            assert s["count"] == 499_999_999
            assert int(hist.sum()) == s["count"]


# --------------------------------------------------------------------------
# Goldbach partition counts c(n) (n = p + q, primes p <= q)
# --------------------------------------------------------------------------

# Worked by hand: the partitions of each n.  4 = 2+2; 6 = 3+3; 8 = 3+5;
# 10 = 3+7 = 5+5; 12 = 5+7; 14 = 3+11 = 7+7; 16 = 3+13 = 5+11;
# 18 = 5+13 = 7+11; 20 = 3+17 = 7+13; 22 = 3+19 = 5+17 = 11+11;
# 24 = 5+19 = 7+17 = 11+13; 26 = 3+23 = 7+19 = 13+13; 28 = 5+23 = 11+17;
# 30 = 7+23 = 11+19 = 13+17.
_PC_BY_HAND = {4: 1, 6: 1, 8: 1, 10: 2, 12: 1, 14: 2, 16: 2, 18: 2, 20: 2,
               22: 3, 24: 3, 26: 3, 28: 2, 30: 3}


def test_partition_counts_by_hand(orc):
    c, s = orc.partition_counts_range(4, 30)
    assert [int(x) for x in c] == [_PC_BY_HAND[n] for n in range(4, 31, 2)]
    # summaries of this list: sum, the first n with the fewest (4) and the
    # first with the most (22)
    assert s == {"count": 14, "sum": sum(_PC_BY_HAND.values()), "min_c": 1,
                 "argmin_n": 4, "max_c": 3, "argmax_n": 22}


def test_partition_counts_trial_division(orc, td_table):
    ns = list(range(4, 6001, 2))
    c, _ = orc.partition_counts(ns, threads=4)
    for n, got in zip(ns, c):
        want = sum(1 for p in range(2, n // 2 + 1) if td_table[p] and td_table[n - p])
        assert int(got) == want, n


def _np_odd_sieve(top):
    """is_prime for the odd numbers 1, 3, ..., top (numpy, written here)."""
    m = (top - 1) // 2 + 1
    isp = np.ones(m, dtype=bool)
    isp[0] = False
    for k in range(1, (int(top ** 0.5) - 1) // 2 + 1):
        if isp[k]:
            p = 2 * k + 1
            isp[(p * p - 1) // 2::p] = False
    return isp


def test_partition_counts_vs_vector_sieve(orc):
    # a different computation: for each n, AND the odd-prime flags of p and
    # of n - p as whole vectors
    top = 2_000_000
    isp = _np_odd_sieve(top)
    ns = [10**6, 10**6 - 2, 999_000, 1_999_998, 2_000_000, 1_234_568, 65_536]
    c, _ = orc.partition_counts(ns, threads=4)
    for n, got in zip(ns, c):
        k = np.arange(1, (n // 2 - 1) // 2 + 1)          # odd p = 2k+1 <= n/2
        want = int(np.count_nonzero(isp[k] & isp[(n - 2 * k - 2) // 2]))
        assert int(got) == want, n


def test_partition_count_total_identity(orc):
    # sum over even n <= N of c(n) counts the pairs of primes p <= q with
    # p + q <= N: for each prime p <= N/2, the primes q in [p, N - p]
    N = 40_000
    isp = _np_odd_sieve(N)
    odd_primes = 2 * np.nonzero(isp)[0] + 1
    pi_odd = np.cumsum(isp)                               # odd primes <= 2i+1
    pairs = 1                                             # 2 + 2
    for p in odd_primes[odd_primes <= N // 2]:
        q_hi = N - p
        q_hi -= 1 - (q_hi & 1)                            # largest odd <= N - p
        pairs += int(pi_odd[(q_hi - 1) // 2] - pi_odd[(p - 1) // 2] + 1)
    _, s = orc.partition_counts_range(4, N, threads=4)
    assert s["sum"] == pairs
    assert s["count"] == N // 2 - 1


def test_partition_counts_rejects_odd(orc):
    with pytest.raises(ValueError):
        orc.partition_counts([4, 7])
