"""CPU oracle for minimal Goldbach partitions -- TEST INFRASTRUCTURE ONLY.

Plain, slow and obviously correct: a segmented byte-per-odd-number Sieve of
Eratosthenes plus a scan of primes p upward from 2 for every even n (the
paper's CPU baseline, section "Methods"), with a deterministic twelve-base
Miller-Rabin test for single 64-bit n (section "GPU Single-Number Checker"),
and Goldbach partition counts c(n) by their definition (section "Future
work").
Only tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package.  The product library never does.

Every function here is pinned by ``tests/test_oracle_pins.py`` against
results that do not come from the oracle itself (trial division, SymPy's
primality routines, prime counts, the paper's printed counts, strong
pseudoprimes from the literature).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gb_oracle.c")
_LIB = os.path.join(_HERE, "libgb_oracle.so")

HIST_BINS = 6543


class PcSummary(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "count", "sum", "min_c", "argmin_n", "max_c", "argmax_n")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class Summary(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "count", "max_p", "argmax_n", "checksum", "n_exhaustive", "n_failed",
        "first_failed_n")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into a shared library next to its source."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-shared", "-fPIC",
                               "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u64, u32, vp, ip = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
        L.orc_isqrt.argtypes, L.orc_isqrt.restype = [u64], u64
        L.orc_trial_is_prime.argtypes, L.orc_trial_is_prime.restype = [u64], ip
        L.orc_mr_base.argtypes, L.orc_mr_base.restype = [u64, u64], ip
        L.orc_mr.argtypes, L.orc_mr.restype = [u64], ip
        L.orc_is_prime.argtypes, L.orc_is_prime.restype = [u64], ip
        L.orc_prime_count.argtypes, L.orc_prime_count.restype = [u64], u64
        L.orc_verify_range.argtypes = [u64, u64, u32, vp, ip, vp, ctypes.POINTER(Summary)]
        L.orc_verify_range.restype = ip
        L.orc_verify_range_mt.argtypes = [u64, u64, u32, vp, ip, vp,
                                          ctypes.POINTER(Summary), ip]
        L.orc_verify_range_mt.restype = ip
        L.orc_verify_one.argtypes, L.orc_verify_one.restype = [u64, u64], u64
        L.orc_verify_many.argtypes = [vp, vp, u64, u64, ip]
        L.orc_verify_many.restype = None
        L.orc_hist_bins.argtypes, L.orc_hist_bins.restype = [], u32
        L.orc_checksum_weight.argtypes, L.orc_checksum_weight.restype = [u64], u64
        L.orc_odd_primality.argtypes, L.orc_odd_primality.restype = [u64, u64, vp], ip
        L.orc_verify_windows.argtypes = [vp, vp, u64, u32, vp, ctypes.POINTER(Summary), ip]
        L.orc_verify_windows.restype = ip
        L.orc_partition_counts.argtypes = [vp, vp, u64, ctypes.POINTER(PcSummary), ip]
        L.orc_partition_counts.restype = ip
        _lib = L
    return _lib


def isqrt(x: int) -> int:
    return int(lib().orc_isqrt(x))


def trial_is_prime(q: int) -> bool:
    return bool(lib().orc_trial_is_prime(q))


def mr_base(q: int, a: int) -> bool:
    return bool(lib().orc_mr_base(q, a))


def checksum_weight(n: int) -> int:
    """Weight of even n in the checksum (sum of weight * p_min, mod 2^64)."""
    return int(lib().orc_checksum_weight(n))


def mr(q: int) -> bool:
    return bool(lib().orc_mr(q))


def is_prime(q: int) -> bool:
    return bool(lib().orc_is_prime(q))


def prime_count(x: int) -> int:
    return int(lib().orc_prime_count(x))


def n_even(lo: int, hi: int) -> int:
    lo = max(lo, 4)
    lo += lo & 1
    hi -= hi & 1
    return 0 if lo > hi else (hi - lo) // 2 + 1


def verify_range(lo: int, hi: int, pmax: int = 8192, per_n_bits: int | None = 32,
                 hist: bool = True, threads: int = 1):
    """p_min for every even n in [max(lo,4), hi].

    Returns (pmin array or None, hist array or None, summary dict).  With
    ``per_n_bits=16`` the array is uint16 and holds 0 for p_min >= 2^16.
    """
    L = lib()
    cnt = n_even(lo, hi)
    out = None
    if per_n_bits:
        out = np.zeros(cnt, dtype=np.uint32 if per_n_bits == 32 else np.uint16)
    h = np.zeros(HIST_BINS, dtype=np.uint64) if hist else None
    s = Summary()
    optr = out.ctypes.data if out is not None and cnt else None
    hptr = h.ctypes.data if h is not None else None
    if threads > 1:
        rc = L.orc_verify_range_mt(lo, hi, pmax, optr, per_n_bits or 32, hptr,
                                   ctypes.byref(s), threads)
    else:
        rc = L.orc_verify_range(lo, hi, pmax, optr, per_n_bits or 32, hptr,
                                ctypes.byref(s))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return out, h, s.as_dict()


def verify_windows(windows, pmax: int = 8192, per_n: bool = True, threads: int = 1):
    """p_min for the even n of each window (start, len): start, start + 2,
    ..., start + 2 (len - 1), start even and >= 4.  Returns (uint16 array of
    every window's n concatenated in order, or None; list of summary dicts,
    one per window)."""
    k = len(windows)
    st = np.ascontiguousarray(np.array([w[0] for w in windows], dtype=np.uint64))
    ln = np.ascontiguousarray(np.array([w[1] for w in windows], dtype=np.uint64))
    out = np.zeros(int(ln.sum()), dtype=np.uint16) if per_n else None
    sums = (Summary * max(k, 1))()
    if k:
        rc = lib().orc_verify_windows(st.ctypes.data, ln.ctypes.data, k, pmax,
                                      out.ctypes.data if out is not None and out.size else None,
                                      sums, threads)
        if rc == -2:
            raise ValueError("every window needs an even start >= 4 and a positive length")
        if rc != 0:
            raise MemoryError("oracle allocation failed")
    return out, [sums[i].as_dict() for i in range(k)]


def odd_primality(w0: int, count: int) -> np.ndarray:
    """uint8 array: 1 where w0 + 2i (w0 odd) is prime, for 0 <= i < count."""
    out = np.zeros(count, dtype=np.uint8)
    if count and lib().orc_odd_primality(w0, count, out.ctypes.data) != 0:
        raise MemoryError("oracle allocation failed")
    return out


def verify_one(n: int, limit: int = 0) -> int:
    return int(lib().orc_verify_one(n, limit))


def verify_many(ns, limit: int = 0, threads: int = 1) -> np.ndarray:
    arr = np.ascontiguousarray(np.asarray(ns, dtype=np.uint64))
    out = np.zeros_like(arr)
    if arr.size:
        lib().orc_verify_many(arr.ctypes.data, out.ctypes.data, arr.size, limit, threads)
    return out


def partition_counts(ns, threads: int = 1):
    """Goldbach partition counts c(n) (n = p + q, primes p <= q) for each even
    n >= 4 of ``ns``.  Returns (uint64 array, summary dict)."""
    arr = np.ascontiguousarray(np.asarray(ns, dtype=np.uint64))
    out = np.zeros_like(arr)
    s = PcSummary()
    rc = lib().orc_partition_counts(arr.ctypes.data if arr.size else None,
                                    out.ctypes.data if arr.size else None,
                                    arr.size, ctypes.byref(s), threads)
    if rc == -2:
        raise ValueError("every n must be even and at least 4")
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return out, s.as_dict()


def partition_counts_range(lo: int, hi: int, threads: int = 1):
    """c(n) for every even n in [max(lo, 4), hi]."""
    cnt = n_even(lo, hi)
    first = max(lo, 4)
    first += first & 1
    return partition_counts(first + 2 * np.arange(cnt, dtype=np.uint64), threads)
