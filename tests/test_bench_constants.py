"""The per-n algorithmic work the benchmark divides by (bench.ALG_OPS_PER_N)
recomputed from its ingredients: the sieve's bit clears from the sum of 1/p
over the sieving primes, and the probes and hit events per 64-n block from
the oracle's p_min on the last 2^20 even n up to 10^12."""
import math

import numpy as np

import bench


def _odd_primes(limit):
    s = np.ones(limit + 1, dtype=bool)
    s[:2] = False
    for i in range(2, int(limit ** 0.5) + 1):
        if s[i]:
            s[i * i::i] = False
    return np.nonzero(s)[0][1:]          # odd primes


def test_sieve_clears_per_odd_number():
    ps = _odd_primes(10**6)
    assert len(ps) == 78497
    clears = float(np.sum(1.0 / ps[ps >= 11]))
    assert math.isclose(clears, bench.CLEARS_PER_N, rel_tol=2e-3)
    assert math.isclose(len(ps) / 2**20, bench.STRIKES_PER_N, rel_tol=1e-9)


def test_probes_and_hits_per_block(orc):
    blocks = 1 << 14
    hi = 10**12
    lo = hi - 2 * (64 * blocks - 1)
    lo -= 2 * ((lo // 2) % 64)                 # blocks start where (n/2) mod 64 = 0
    out, _, _ = orc.verify_range(lo, lo + 2 * (64 * blocks - 1), per_n_bits=32, hist=False)
    P = out.reshape(-1, 64)
    ps = _odd_primes(70000)
    index = {int(p): i + 1 for i, p in enumerate(ps)}          # 3 -> 1, 5 -> 2, ...
    largest = np.array([index[int(r.max())] for r in P])
    distinct = np.array([len(set(r.tolist())) for r in P])
    assert math.isclose(largest.mean() / 64, bench.PROBES_PER_N, rel_tol=0.01)
    assert math.isclose(distinct.mean() / 64, bench.HITS_PER_N, rel_tol=0.01)
    ops = (bench.CLEARS_PER_N * 3 + 5 / 32 + bench.STRIKES_PER_N * 10 + bench.PROBES_PER_N * 7
           + bench.HITS_PER_N * 8)
    assert math.isclose(ops, bench.ALG_OPS_PER_N)
    # 157.3 TFLOP/s of fp32 vector FMA is 78.6e12 lane slots per second
    assert math.isclose(bench.ALU_PEAK_OPS, 157.3e12 / 2, rel_tol=1e-3)
