"""Pins for the big-n oracle (oracle/big.py): the paper's Table 5, the 64-bit
oracle (independent C code with the deterministic twelve-base test) below
2^63, SymPy's primality test, and the smallest strong pseudoprimes to the
first 12 and 13 prime bases (Sorenson and Webster), which a test with fewer
bases would call prime."""
import os
import random

import pytest
import sympy

from oracle import big

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_big.txt")


def _table5():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                e, p = line.split()
                rows.append((int(e), int(p)))
    return rows


def test_table5_values():
    rows = _table5()
    assert rows
    for e, p in rows:
        n = 10**e
        assert big.pmin_big(n) == p
        # minimality with a different primality test
        assert sympy.isprime(n - p)
        assert not any(sympy.isprime(n - q) for q in sympy.primerange(3, p))


def test_table5_row_10e200_is_not_a_partition():
    # the reading recorded in the fixture: 10^200 - 113 has the factor 13
    assert (10**200 - 113) % 13 == 0


def test_equals_64bit_oracle(orc):
    rng = random.Random(11)
    ns = [2 * rng.randrange(2, 2**62) for _ in range(300)] + [10**12, 2**63, 2**63 - 2, 98]
    for n in ns:
        assert big.pmin_big(n) == orc.verify_one(n), n


@pytest.mark.parametrize("psi,k", [(318665857834031151167461, 12), (3317044064679887385961981, 13)])
def test_strong_pseudoprimes_need_more_bases(psi, k):
    assert not sympy.isprime(psi)
    assert all(big.strong_probable_prime(psi, a) for a in big.BASES[:k])
    assert not big.probable_prime(psi)


def test_agrees_with_sympy_on_random_big_numbers():
    rng = random.Random(5)
    for bits in (70, 100, 128, 200, 400):
        for _ in range(60):
            q = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
            assert big.probable_prime(q) == sympy.isprime(q), q
    for e in (89, 107, 127, 521):
        assert big.probable_prime(2**e - 1)
    assert not big.probable_prime(2**128 + 1)


def test_random_big_n_minimal():
    rng = random.Random(3)
    for bits in (80, 128, 256):
        for _ in range(5):
            n = 2 * rng.getrandbits(bits - 1) + 4
            p = big.pmin_big(n)
            assert p and sympy.isprime(p) and sympy.isprime(n - p)
            assert not any(sympy.isprime(n - q) for q in sympy.primerange(3, p))


def test_small_factor_fails_its_own_base():
    # q with an odd prime factor r <= 97 fails the strong test to base r: every
    # power of r mod q is a multiple of r, never 1 or q - 1.  The GPU scan drops
    # p = n (mod r) on this ground before exponentiating, so its answer equals
    # the full 25-base scan's.
    rng = random.Random(11)
    for r in big.BASES[1:]:
        for bits in (70, 200, 500):
            for _ in range(4):
                q = r * (rng.getrandbits(bits) | 1)
                assert not big.strong_probable_prime(q, r), (q, r)
                assert not big.probable_prime(q)
