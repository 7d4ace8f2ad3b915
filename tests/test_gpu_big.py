"""Minimal Goldbach prime of even n beyond 64 bits on the GPU against the
big-n oracle (GPU): the paper's Table 5 values, random n in every limb-count
class (up to 1024 bits) and at each class's edges, n just above 2^64, a
batch, base-2 pseudoprime candidates, one call over every class, and the
argument checks."""
import random

import pytest

from oracle import big

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_02621_amd import Verifier
    v = Verifier(0)
    yield v
    v.close()


def test_table5(V):
    assert V.verify_big([10**50, 10**100]) == [383, 797]


@pytest.mark.parametrize("bits", [65, 96, 127, 128, 200, 256, 333, 500, 512, 520, 600, 700, 768, 1020])
def test_random_vs_oracle(V, bits):
    rng = random.Random(bits)
    ns = [2 * rng.getrandbits(bits - 1) | (1 << (bits - 1)) for _ in range(6)]
    ns = [n - (n & 1) for n in ns]
    assert V.verify_big(ns) == [big.pmin_big(n) for n in ns]


def test_just_above_2p64(V):
    ns = [2**64, 2**64 + 2, 2**64 + 10**6, 2**96 - 2, 2**128 - 2]
    assert V.verify_big(ns) == [big.pmin_big(n) for n in ns]


def test_batch(V):
    ns = [10**30 + 2 * i for i in range(300)]
    assert V.verify_big(ns) == [big.pmin_big(n) for n in ns]


def test_many_open_n_share_wavefronts(V):
    # 300 n of 440 bits: many need more than the first 32 candidates the
    # small-base filter leaves, so the later passes give each open n several
    # groups of 32 (up to 16) that all start from one resume point
    ns = [2**439 + 2 * 10**6 * i + 2 * i * i for i in range(300)]
    assert V.verify_big(ns) == [big.pmin_big(n) for n in ns]


def test_argument_checks(V):
    from paper_2603_02621_amd import GoldbachError
    with pytest.raises(GoldbachError):
        V.verify_big([10**30 + 1])           # odd
    with pytest.raises(GoldbachError):
        V.verify_big([2**64 - 2])            # below 2^64
    with pytest.raises(ValueError):
        V.verify_big([2**1024])              # beyond 1024 bits
    assert V.verify_big([]) == []


@pytest.mark.parametrize("psi", [318665857834031151167461, 3317044064679887385961981])
def test_base2_pseudoprime_candidate_is_rejected(V, psi):
    # q = psi is a strong pseudoprime to 2, 3, ..., 37 (and 41 for the second):
    # for n = psi + 3 the base-2 search stops at p = 3, the confirmation over
    # the other bases rejects it, and the search resumes after it
    ns = [psi + 3, psi + 5, psi + 3 + 2 * 10**6]
    assert big.strong_probable_prime(psi, 2) and not big.probable_prime(psi)
    got = V.verify_big(ns)
    assert got == [big.pmin_big(n) for n in ns]
    assert got[0] > 3


@pytest.mark.parametrize("bits", [110, 111, 166, 167, 222, 223, 278, 279, 334, 335, 390, 391, 446, 447,
                                  558, 559, 670, 671, 782, 783, 894, 895, 1006, 1007, 1024])
def test_limb_class_edges(V, bits):
    # n of exactly `bits` bits: the largest and smallest of each class of
    # 28-bit limbs (K = 4, 6, ..., 16, 20, 24, ..., 36, 37 limbs hold n up to
    # 28K - 2 bits), up to the largest n the call takes
    rng = random.Random(1000 + bits)
    top = (1 << bits) - 2                              # all ones but the last bit
    low = 1 << (bits - 1)
    mid = (rng.getrandbits(bits - 1) | (1 << (bits - 1))) & ~1
    ns = [top, low, mid]
    assert all(n.bit_length() == bits and n % 2 == 0 for n in ns)
    assert V.verify_big(ns) == [big.pmin_big(n) for n in ns]
    # mixed with a smaller n, which runs in its own form
    assert V.verify_big([2**64 + 2, top]) == [big.pmin_big(2**64 + 2), big.pmin_big(top)]


def test_one_call_over_every_form(V):
    # n of every limb class in one call, interleaved: the call splits them by
    # form and puts each answer back at its n's position
    rng = random.Random(77)
    sizes = [70, 130, 180, 240, 300, 333, 380, 430, 460, 600]
    ns = []
    for i in range(30):
        b = sizes[(7 * i) % len(sizes)]
        ns.append((rng.getrandbits(b - 1) | (1 << (b - 1))) & ~1)
    assert V.verify_big(ns) == [big.pmin_big(n) for n in ns]
