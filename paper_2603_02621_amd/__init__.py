"""MI355X-native segmented Goldbach verifier (GoldbachGPU, arXiv 2603.02621).

Python face of the C ABI in ``include/goldbach.h``.  Every step of the
computation runs in the HIP library ``libgoldbach.so``; PyTorch only provides
device buffers and the current stream.  There is no CPU fallback: using the
verifier without the built library raises.
"""
from __future__ import annotations

import ctypes

from ._binding import (HIST_BINS, MAX_N, GoldbachError, Params, PcResult, Peaks, Result,
                       Summary, Window, lib)

__all__ = ["Verifier", "GoldbachError", "HIST_BINS", "MAX_N"]


def _stream_ptr(stream):
    if stream is None:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Verifier:
    """One library context on one GPU (resident prime table, buffers, graphs)."""

    def __init__(self, device: int = 0, **params):
        self._lib = lib()
        p = Params()
        p.device = device
        for k, v in params.items():
            if not hasattr(p, k):
                raise TypeError(f"unknown parameter {k}")
            setattr(p, k, int(v))
        h = ctypes.c_void_p()
        st = self._lib.gb_create(ctypes.byref(h), ctypes.byref(p))
        if st != 0:
            raise GoldbachError(st, "gb_create failed")
        self._h = h

    # -- plumbing -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.gb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st, allow=()):
        if st != 0 and st not in allow:
            raise GoldbachError(st, self._lib.gb_last_error(self._h).decode())
        return st

    @property
    def params(self) -> dict:
        p = Params()
        self._check(self._lib.gb_get_params(self._h, ctypes.byref(p)))
        return p.as_dict()

    @property
    def geometry(self) -> dict:
        """Tile geometry the parameters resolve to (see gb_tile_geometry)."""
        v = [ctypes.c_uint64() for _ in range(4)]
        self._check(self._lib.gb_tile_geometry(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("cls_tile_n", "cls_lds_bytes", "cls_list_primes", "bulk_tile_n"),
                        (int(x.value) for x in v)))

    @property
    def last_error(self) -> str:
        return self._lib.gb_last_error(self._h).decode()

    # -- calls ----------------------------------------------------------------
    def verify_range(self, lo: int, hi: int, pmin=None, hist=True, seg_hist_rows=0,
                     batched=False, stream=None, allow_unresolved=False):
        """Minimal p for every even n in [max(lo,4), hi].

        ``pmin``: None, or a torch tensor (uint16/int32 on the GPU, or a numpy
        array on the host) with one entry per even n.  Returns a dict with the
        summaries, ``hist`` (numpy uint64), ``seg_hist`` and ``status``.
        """
        import numpy as np
        r = Result()
        keep = []
        if pmin is not None:
            r.pmin, r.pmin_bits, r.pmin_on_device = _buffer(pmin)
            keep.append(pmin)
        h = np.zeros(HIST_BINS, dtype=np.uint64) if hist else None
        if h is not None:
            r.hist = h.ctypes.data
        sh = None
        if seg_hist_rows:
            sh = np.zeros((seg_hist_rows, HIST_BINS), dtype=np.uint64)
            r.seg_hist = sh.ctypes.data
            r.seg_hist_rows = seg_hist_rows
        fn = self._lib.gb_verify_range_batched if batched else self._lib.gb_verify_range
        st = fn(self._h, lo, hi, ctypes.byref(r), _stream_ptr(stream))
        self._check(st, allow=(5,) if allow_unresolved else ())
        out = r.summary()
        out.update(status=st, hist=h, seg_hist=sh, n_segments=int(r.n_segments),
                   device_ms=float(r.device_ms), tile_ms=float(r.tile_ms),
                   tile_launches=int(r.tile_launches))
        return out

    def verify_range_bulk(self, lo: int, hi: int, stream=None, allow_unresolved=False):
        """Bulk verification of every even n in [max(lo,4), hi]: every n gets a
        partition, without recording each minimal p.  Returns count, max_p,
        argmax_n, n_exhaustive, n_failed, first_failed_n (checksum is 0) and
        the timings."""
        r = Result()
        st = self._lib.gb_verify_range_bulk(self._h, lo, hi, ctypes.byref(r), _stream_ptr(stream))
        self._check(st, allow=(5,) if allow_unresolved else ())
        out = r.summary()
        out.update(status=st, n_segments=int(r.n_segments), device_ms=float(r.device_ms),
                   tile_ms=float(r.tile_ms), tile_launches=int(r.tile_launches))
        return out

    def partition_counts(self, lo: int, hi: int, counts=None, stream=None):
        """Goldbach partition counts c(n) (n = p + q, primes p <= q) of every
        even n in [max(lo,4), hi].  ``counts`` (optional) is a contiguous
        int64 tensor on the GPU with one entry per n, overwritten.  Returns
        count, sum, min_c, argmin_n, max_c, argmax_n and the timings."""
        ptr = None
        if counts is not None:
            import torch
            if not (hasattr(counts, "data_ptr") and counts.is_cuda and counts.is_contiguous()
                    and counts.dtype in (torch.int64, torch.uint64)):
                raise ValueError("counts must be a contiguous 64-bit integer tensor on the GPU")
            ptr = counts.data_ptr()
        r = PcResult()
        st = self._lib.gb_partition_counts(self._h, lo, hi, ptr, ctypes.byref(r), _stream_ptr(stream))
        self._check(st)
        out = r.summary()
        out.update(device_ms=float(r.device_ms), kernel_ms=float(r.kernel_ms))
        return out

    def verify_big(self, ns, stream=None, allow_unresolved=False):
        """Minimal p (25-base probable-prime q) of each even n with
        2^64 <= n < 2^1024 (Python integers).  Returns a list of ints (0 for
        none in the prime table)."""
        import numpy as np
        ns = list(map(int, ns))
        if not ns:
            return []
        if min(ns) < 0:
            raise ValueError("n must be positive")
        nl = max(3, (max(ns).bit_length() + 31) // 32)
        if nl > 32:
            raise ValueError("n must be below 2^1024")
        nb = 4 * nl
        words = np.frombuffer(b"".join([x.to_bytes(nb, "little") for x in ns]),
                              dtype="<u4").reshape(len(ns), nl)
        return self.verify_big_words(words, stream, allow_unresolved).tolist()

    def verify_big_words(self, words, stream=None, allow_unresolved=False):
        """The same for n already laid out as the C call takes them: a C-ordered
        uint32 array of shape (k, nlimbs), little-endian limbs, 3 <= nlimbs
        <= 32.  Returns a uint64 array of k entries."""
        import numpy as np
        w = np.ascontiguousarray(words, dtype=np.uint32)
        if w.ndim != 2:
            raise ValueError("words must have shape (k, nlimbs)")
        k, nl = w.shape
        out = np.zeros(k, dtype=np.uint64)
        if k == 0:
            return out
        st = self._lib.gb_verify_big(self._h, w.ctypes.data, nl, k, out.ctypes.data, _stream_ptr(stream))
        self._check(st, allow=(5,) if allow_unresolved else ())
        return out

    def measure_peaks(self, stream=None):
        """Measured device throughput ceilings (see gb_measure_peaks)."""
        r = Peaks()
        self._check(self._lib.gb_measure_peaks(self._h, ctypes.byref(r), _stream_ptr(stream)))
        return r.as_dict()

    def verify_windows(self, windows, pmin=None, sums=True, hist=True, stream=None,
                       allow_unresolved=False):
        """Batched windows: ``windows`` is a sequence of (start, len)."""
        import numpy as np
        k = len(windows)
        W = (Window * max(k, 1))()
        for i, (s, ln) in enumerate(windows):
            W[i].start, W[i].len = int(s), int(ln)
        S = (Summary * max(k, 1))() if sums else None
        h = np.zeros(HIST_BINS, dtype=np.uint64) if hist else None
        ptr = None
        if pmin is not None:
            ptr, bits, on_dev = _buffer(pmin)
            if bits != 16 or not on_dev:
                raise ValueError("windows output must be a uint16 tensor on the GPU")
        st = self._lib.gb_verify_windows(self._h, W, k, ptr, S,
                                         h.ctypes.data if h is not None else None,
                                         _stream_ptr(stream))
        self._check(st, allow=(5,) if allow_unresolved else ())
        return {"status": st, "hist": h,
                "sums": [S[i].as_dict() for i in range(k)] if S is not None else None}

    def verify_one(self, n: int, stream=None, allow_unresolved=False) -> int:
        p = ctypes.c_uint64()
        st = self._lib.gb_verify_one(self._h, n, ctypes.byref(p), _stream_ptr(stream))
        self._check(st, allow=(5,) if allow_unresolved else ())
        return int(p.value)

    def verify_many(self, ns, stream=None, allow_unresolved=False):
        """Minimal p for each even n of a numpy uint64 array (host) or a
        torch int64/uint64 tensor on the GPU (result has the same kind)."""
        import numpy as np
        if hasattr(ns, "data_ptr"):
            import torch
            out = torch.empty_like(ns)
            st = self._lib.gb_verify_many(self._h, ns.data_ptr(), out.data_ptr(), ns.numel(), 1,
                                          _stream_ptr(stream))
        else:
            arr = np.ascontiguousarray(np.asarray(ns, dtype=np.uint64))
            out = np.zeros_like(arr)
            st = self._lib.gb_verify_many(self._h, arr.ctypes.data, out.ctypes.data, arr.size, 0,
                                          _stream_ptr(stream))
        self._check(st, allow=(5,) if allow_unresolved else ())
        return out

    def verify_many_noalloc(self, ns, out=None, stream=None, allow_unresolved=False):
        """verify_many for a torch int64/uint64 tensor on the GPU with no
        device allocation inside the library (at most 65536 n; `out`, a
        tensor like `ns`, receives the p)."""
        import torch
        if out is None:
            out = torch.empty_like(ns)
        st = self._lib.gb_verify_many_noalloc(self._h, ns.data_ptr(), out.data_ptr(), ns.numel(),
                                              _stream_ptr(stream))
        self._check(st, allow=(5,) if allow_unresolved else ())
        return out

    def sieve_window(self, w0: int, nbits: int, out, stream=None):
        """Sieve bits of the odd numbers w0, w0+2, ... into ``out`` (a torch
        int32 tensor of nbits/32 words on the GPU)."""
        self._check(self._lib.gb_sieve_window(self._h, w0, nbits, out.data_ptr(),
                                              _stream_ptr(stream)))
        return out

    def sieve_planes(self, k0: int, nk: int, out, stream=None):
        """The minimal-p search's sieve planes: row i of ``out`` (a torch int32
        tensor of 2 x nk/32 words on the GPU) holds bit k = [6(k0+k) + c_i is
        prime], c = (1, 5)."""
        self._check(self._lib.gb_sieve_planes(self._h, k0, nk, out.data_ptr(), _stream_ptr(stream)))
        return out

    def exhaustive_list(self):
        import numpy as np
        cnt = ctypes.c_size_t()
        self._check(self._lib.gb_exhaustive_list(self._h, None, None, 0, ctypes.byref(cnt)))
        n = np.zeros(cnt.value, dtype=np.uint64)
        p = np.zeros(cnt.value, dtype=np.uint64)
        if cnt.value:
            self._check(self._lib.gb_exhaustive_list(self._h, n.ctypes.data, p.ctypes.data,
                                                      cnt.value, ctypes.byref(cnt)))
        return n, p

    def autotune(self, windows, cache_path=None):
        k = len(windows)
        W = (Window * max(k, 1))()
        for i, (s, ln) in enumerate(windows):
            W[i].start, W[i].len = int(s), int(ln)
        best = Params()
        self._check(self._lib.gb_autotune(self._h, W, k,
                                          cache_path.encode() if cache_path else None,
                                          ctypes.byref(best)))
        return best.as_dict()


def _buffer(x):
    """(pointer, bits, on_device) of a torch tensor or numpy array."""
    import numpy as np
    if hasattr(x, "data_ptr"):
        import torch
        bits = {torch.uint16: 16, torch.int16: 16, torch.int32: 32, torch.uint32: 32}.get(x.dtype)
        if bits is None or not x.is_contiguous():
            raise ValueError("pmin tensor must be contiguous 16- or 32-bit integers")
        return x.data_ptr(), bits, 1 if x.is_cuda else 0
    a = x
    if not isinstance(a, np.ndarray) or not a.flags.c_contiguous:
        raise ValueError("pmin array must be a contiguous numpy array")
    bits = {np.dtype(np.uint16): 16, np.dtype(np.uint32): 32}.get(a.dtype)
    if bits is None:
        raise ValueError("pmin array must be uint16 or uint32")
    return a.ctypes.data, bits, 0
