"""ctypes declarations of the C ABI in ``include/goldbach.h``.

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly when ``libgoldbach.so`` has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgoldbach.so")

HIST_BINS = 6543
MAX_N = 1 << 63

STATUS = {0: "GB_OK", 1: "GB_EINVAL", 2: "GB_ERANGE", 3: "GB_ENOMEM", 4: "GB_EDEVICE",
          5: "GB_EUNRESOLVED"}

u64, u32, i32, vp, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double


class Params(ctypes.Structure):
    _fields_ = [("device", i32), ("pmax", u32), ("seg_log2", u32), ("tile_log2", u32),
                ("wg_threads", u32), ("wheel_max", u32), ("search_mode", u32), ("reserved", u32),
                ("max_hi", u64),
                ("exhaustive_budget_p", u64), ("max_unresolved", u64), ("mem_budget", u64)]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class Result(ctypes.Structure):
    _fields_ = [("pmin", vp), ("pmin_bits", u32), ("pmin_on_device", u32),
                ("hist", vp), ("seg_hist", vp), ("seg_hist_rows", u64),
                ("count", u64), ("max_p", u64), ("argmax_n", u64), ("checksum", u64),
                ("n_exhaustive", u64), ("n_failed", u64), ("first_failed_n", u64),
                ("n_segments", u64), ("device_ms", dbl), ("tile_ms", dbl),
                ("tile_launches", u64)]

    SUMMARY = ("count", "max_p", "argmax_n", "checksum", "n_exhaustive", "n_failed",
               "first_failed_n")

    def summary(self):
        return {k: int(getattr(self, k)) for k in self.SUMMARY}


class Window(ctypes.Structure):
    _fields_ = [("start", u64), ("len", u64)]


class Summary(ctypes.Structure):
    _fields_ = [(k, u64) for k in Result.SUMMARY]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k in Result.SUMMARY}


class Request(ctypes.Structure):
    _fields_ = [("kind", u32), ("flags", u32), ("n", u64), ("len", u64), ("pmin", vp), ("tag", u64)]


class Completion(ctypes.Structure):
    _fields_ = [("id", u64), ("tag", u64), ("status", i32), ("kind", u32), ("p", u64),
                ("summary", Summary), ("submit_ns", u64), ("launch_ns", u64), ("done_ns", u64),
                ("batch_requests", u32), ("stream", u32)]


class PcResult(ctypes.Structure):
    _fields_ = [(k, u64) for k in ("count", "sum", "min_c", "argmin_n", "max_c", "argmax_n")] + \
               [("device_ms", dbl), ("kernel_ms", dbl)]

    SUMMARY = ("count", "sum", "min_c", "argmin_n", "max_c", "argmax_n")

    def summary(self):
        return {k: int(getattr(self, k)) for k in self.SUMMARY}


class Peaks(ctypes.Structure):
    _fields_ = [(k, dbl) for k in ("valu_vop2_ops", "valu_vop3_ops", "lds_read_bytes",
                                   "lds_atomic_ops", "hbm_copy_bytes")]

    def as_dict(self):
        return {name: float(getattr(self, name)) for name, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [(k, u64) for k in ("submitted", "completed", "rejected", "queued", "inflight",
                                   "bytes_inflight", "peak_bytes_inflight", "launches",
                                   "peak_concurrent_launches")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


# exported name -> (argtypes, restype)
SIGNATURES = {
    "gb_create": ([ctypes.POINTER(vp), ctypes.POINTER(Params)], i32),
    "gb_destroy": ([vp], None),
    "gb_get_params": ([vp, ctypes.POINTER(Params)], i32),
    "gb_tile_geometry": ([vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                          ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)], i32),
    "gb_verify_range": ([vp, u64, u64, ctypes.POINTER(Result), vp], i32),
    "gb_verify_range_batched": ([vp, u64, u64, ctypes.POINTER(Result), vp], i32),
    "gb_verify_range_bulk": ([vp, u64, u64, ctypes.POINTER(Result), vp], i32),
    "gb_verify_windows": ([vp, ctypes.POINTER(Window), ctypes.c_size_t, vp,
                           ctypes.POINTER(Summary), vp, vp], i32),
    "gb_verify_one": ([vp, u64, ctypes.POINTER(u64), vp], i32),
    "gb_verify_many": ([vp, vp, vp, ctypes.c_size_t, ctypes.c_int, vp], i32),
    "gb_verify_many_noalloc": ([vp, vp, vp, ctypes.c_size_t, vp], i32),
    "gb_sieve_window": ([vp, u64, u64, vp, vp], i32),
    "gb_sieve_planes": ([vp, u64, u64, vp, vp], i32),
    "gb_partition_counts": ([vp, u64, u64, vp, ctypes.POINTER(PcResult), vp], i32),
    "gb_measure_peaks": ([vp, ctypes.POINTER(Peaks), vp], i32),
    "gb_verify_big": ([vp, vp, u32, ctypes.c_size_t, vp, vp], i32),
    "gb_exhaustive_list": ([vp, vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)], i32),
    "gb_autotune": ([vp, ctypes.POINTER(Window), ctypes.c_size_t, ctypes.c_char_p,
                     ctypes.POINTER(Params)], i32),
    "gb_server_start": ([ctypes.POINTER(vp), ctypes.POINTER(Params), u32, u32], i32),
    "gb_server_submit": ([vp, ctypes.POINTER(Request), ctypes.POINTER(u64)], i32),
    "gb_server_poll": ([vp, ctypes.POINTER(Completion), ctypes.c_size_t,
                        ctypes.POINTER(ctypes.c_size_t), i32], i32),
    "gb_server_replay": ([vp, ctypes.POINTER(Request), ctypes.POINTER(u64), ctypes.c_size_t,
                          ctypes.POINTER(Completion), u32], i32),
    "gb_server_stats_get": ([vp, ctypes.POINTER(ServerStats)], i32),
    "gb_server_stop": ([vp], i32),
    "gb_server_last_error": ([vp], ctypes.c_char_p),
    "gb_status_str": ([i32], ctypes.c_char_p),
    "gb_last_error": ([vp], ctypes.c_char_p),
}

_lib = None


def lib():
    """Load the HIP library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2603_02621_amd.build`; "
                "there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


class GoldbachError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message
