"""Seeded synthetic workloads: integers only, no arithmetic of the method.

Both the GPU path and the oracle take their inputs from here, so this module
holds nothing but the draws.  numpy's default_rng (PCG64) fixes the streams.
"""
from __future__ import annotations

import numpy as np

# every even n in [4, 10^6]
CONFIG1 = (4, 10**6)
# every even n in [4, 10^9], segments of 2^24 even n, fast path up to 2^13
CONFIG2 = (4, 10**9)
CONFIG2_PARAMS = {"seg_log2": 24, "pmax": 2**13}
# the last 2^36 integers up to 10^12: 2^35 + 1 even n
CONFIG4 = (10**12 - 2**36, 10**12)
# its oracle sub-slice: 2^26 consecutive even n ending at 10^12
CONFIG4_SLICE = (10**12 - 2 * (2**26 - 1), 10**12)


def config3_windows(seed: int = 0, k: int = 4096):
    """k windows of even n: start even, uniform in [10^9, 10^12]; length
    log-uniform in [2^10, 2^24] even numbers.  Returns [(start, len)]."""
    rng = np.random.default_rng(seed)
    start = 2 * rng.integers(5 * 10**8, 5 * 10**11, size=k, endpoint=True)
    u = rng.random(k)
    length = np.clip(np.floor(2.0 ** (10 + 14 * u)).astype(np.int64), 2**10, 2**24)
    return [(int(s), int(n)) for s, n in zip(start, length)]


def config5_requests(seed: int = 1, count: int = 10_000, qps: float = 1000.0):
    """A Poisson request stream at rate `qps`.  Each request, in order:
    exponential gap; with probability 0.8 one even n uniform in [4, 2^63];
    otherwise a range with start even, uniform in [10^12, 10^15], and
    length log-uniform in [2^12, 2^22] even numbers.

    Returns a list of dicts: {"t": arrival seconds, "kind": "one"|"range",
    "n": int, "len": int}.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += float(rng.exponential(1.0 / qps))
        if rng.random() < 0.8:
            n = 2 * int(rng.integers(2, 2**62, endpoint=True))
            out.append({"t": t, "kind": "one", "n": n, "len": 1})
        else:
            start = 2 * int(rng.integers(5 * 10**11, 5 * 10**14, endpoint=True))
            ln = int(np.floor(2.0 ** (12 + 10 * rng.random())))
            out.append({"t": t, "kind": "range", "n": start, "len": ln})
    return out
