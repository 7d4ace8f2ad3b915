"""The GPU's multi-limb header (gb_bignum28.h, 28-bit limbs) built for the
CPU with g++ under the address and undefined-behaviour sanitizers, and
checked against Python integers and the big-n oracle: the lazy Montgomery
squaring, the multiplication by a small integer (quotient estimated in
double precision from the top limbs), R mod m, strong probable-prime tests
to all 25 bases, and the minimal-p search in the kernels' order (odd bases
filter, base 2, then the other 24 bases), at every limb count the library
compiles (K = 4, 6, ..., 16, 20, 24, ..., 36, 37) and at the bounds of the
moduli each takes.

The last test models the search's trip counts: a base-2 test that never
passes (what a wrong device build of it does) sends a search through the
whole prime table instead of a few groups of 64."""
import os
import random
import shutil
import subprocess

import pytest

from oracle import big

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bignum_host.cpp")
LIMIT = 1 << 22                       # the driver's prime table: odd primes below 2^22
FORMS = (4, 6, 8, 10, 12, 14, 16, 20, 24, 28, 32, 36, 37)

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def drv(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("bignum") / "bignum_host")
    subprocess.check_call(["g++", "-O3", "-std=c++17", "-fsanitize=undefined,address",
                           "-fno-sanitize-recover=all", "-Wall", "-Wno-unknown-pragmas", "-o", exe, SRC])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    p = subprocess.Popen([exe], stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True, env=env)

    def ask(line):
        p.stdin.write(line + "\n")
        p.stdin.flush()
        out = p.stdout.readline().strip()
        assert out, f"driver gave no answer to {line!r} (exit {p.poll()})"
        return out

    yield ask
    p.stdin.close()
    assert p.wait(timeout=30) == 0


def _widths(K):
    """Modulus widths a form takes: 2^(28(K-E)+24) <= m < 2^(28K-2), with E the
    limbs of the quotient estimate (3 up to K = 16, 5 above)."""
    E = 3 if K <= 16 else 5
    return 28 * (K - E) + 25, 28 * K - 2


def _form(bits):
    """The form the library picks for an n of this many bits."""
    return next(K for K in FORMS if 28 * K - 2 >= bits)


@pytest.mark.parametrize("K", FORMS)
def test_lazy_squaring_small_multiplier_and_one(drv, K):
    # operands anywhere in [0, 2m), the lazy range; results must stay in
    # [0, 2m) for the squaring and [0, 1.19 m) for the small multiplier, and
    # agree with Python integers mod m
    rng = random.Random(K)
    R = 1 << (28 * K)
    lo, hi = _widths(K)
    for t in range(60):
        w = (lo, hi)[t % 2] if t < 4 else rng.randrange(lo, hi + 1)
        m = rng.getrandbits(w) | 1 | (1 << (w - 1))
        a = (2 * m - 1, 0, m, 1)[t % 4] if t < 8 else rng.randrange(2 * m)
        r, rn = (int(x, 16) for x in drv(f"sqr {K} {m:x} {a:x}").split())
        want = a * a * pow(R, -1, m) % m
        assert r < 2 * m and r % m == want and rn == want, (K, hex(m), hex(a))
        f = (1 << 20, 1, 97 ** 3, 2)[t % 4] if t < 8 else rng.randrange(1, (1 << 20) + 1)
        r, rn = (int(x, 16) for x in drv(f"mulsmall {K} {m:x} {a:x} {f}").split())
        assert 100 * r < 119 * m and r % m == a * f % m and rn == a * f % m, (K, hex(m), hex(a), f)
        assert int(drv(f"one {K} {m:x}"), 16) == R % m


@pytest.mark.parametrize("K", FORMS)
def test_strong_tests_match_the_oracle(drv, K):
    rng = random.Random(7 * K + 28)
    lo, hi = _widths(K)
    lo = max(lo, 66)
    qs = []
    for t in range(6 if K <= 16 else 3):
        w = (lo, hi)[t % 2] if t < 2 else rng.randrange(lo, hi + 1)
        q = rng.getrandbits(w) | 1 | (1 << (w - 1))
        while not big.probable_prime(q):
            q += 2
        qs += [q, q + 2, q + 4]
    # q - 1 with many trailing zero bits (long squaring tails)
    for s in (20, 45):
        w = rng.randrange(lo, hi + 1)
        qs.append(((rng.getrandbits(w - s) | (1 << (w - s - 1))) << s) + 1)
    # strong pseudoprimes to the first 12 and 13 prime bases
    qs += [318665857834031151167461, 3317044064679887385961981]
    for q in qs:
        if not (lo <= q.bit_length() <= hi):
            continue
        for a in big.BASES:
            want = big.strong_probable_prime(q, a)
            assert int(drv(f"sprp {K} {q:x} {a}")) == int(want), (K, hex(q), a)


def _random_even(bits, rng):
    n = 2 * rng.getrandbits(bits - 1) | (1 << (bits - 1))
    return n - (n & 1)


@pytest.mark.parametrize("bits", [100, 160, 200, 250, 280, 333, 390, 440, 447, 520, 600, 700, 1020, 1024])
def test_minimal_p_search_matches_the_oracle(drv, bits):
    # the inputs of the GPU tests at these sizes (random.Random(bits)), in
    # the form the library picks for them
    rng = random.Random(bits)
    ns = [_random_even(bits, rng) for _ in range(6)]
    K = _form(bits)
    for n in ns[:3 if bits < 600 else 1]:
        p, groups, tests = (int(x) for x in drv(f"pmin {K} {n:x}").split())
        assert p == big.pmin_big(n, limit=LIMIT), (bits, K)
        assert p > 0 and tests >= 1 and groups >= 1


def test_search_without_base2_passes_reads_the_whole_table(drv):
    # A search stops at its first candidate; with a base-2 test that never
    # passes it filters every table entry instead.  At 520 bits the real
    # search reads a handful of groups of 64 entries; the failing one reads
    # all of them (here 2^22 / ln-density ~ 4.6k groups, in the library's
    # 2.07M-prime table about 32k groups and 4.4e5 base-2 tests per n).
    rng = random.Random(520)
    n = _random_even(520, rng)
    p, g_ok, t_ok = (int(x) for x in drv(f"pmin 20 {n:x}").split())
    z, g_all, t_all = (int(x) for x in drv(f"pmin_nobase2 20 {n:x}").split())
    nprimes = sum(1 for _ in big._odd_primes(LIMIT))
    assert p > 0 and z == 0
    assert g_all == (nprimes + 63) // 64
    assert g_ok <= 64 and g_all > 50 * g_ok
    assert t_all > 100 * t_ok
