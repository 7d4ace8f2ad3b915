"""Seeded generators: reproducible, and inside the stated ranges."""
import numpy as np

from paper_2603_02621_amd import workloads as W


def test_config3_reproducible_and_in_range():
    a = W.config3_windows(0, 4096)
    b = W.config3_windows(0, 4096)
    assert a == b and len(a) == 4096
    s = np.array([x for x, _ in a])
    n = np.array([y for _, y in a])
    assert (s % 2 == 0).all() and s.min() >= 10**9 and s.max() <= 10**12
    assert n.min() >= 2**10 and n.max() <= 2**24
    # log-uniform lengths: about half below the geometric midpoint 2^17
    assert 0.4 < np.mean(n < 2**17) < 0.6
    assert 6e9 < n.sum() < 8e9


def test_config5_mix_and_rates():
    r = W.config5_requests(1, 5000, qps=1000.0)
    assert r == W.config5_requests(1, 5000, qps=1000.0)
    kinds = np.array([q["kind"] == "one" for q in r])
    assert 0.77 < kinds.mean() < 0.83
    t = np.array([q["t"] for q in r])
    assert (np.diff(t) > 0).all() and 4.5 < t[-1] < 5.5
    for q in r:
        assert q["n"] % 2 == 0
        if q["kind"] == "one":
            assert 4 <= q["n"] <= 2**63
        else:
            assert 10**12 <= q["n"] <= 10**15 and 2**12 <= q["len"] <= 2**22


def test_fixed_configs():
    assert W.CONFIG4[1] - W.CONFIG4[0] == 2**36
    lo, hi = W.CONFIG4_SLICE
    assert (hi - lo) // 2 + 1 == 2**26 and hi == 10**12
