"""Serving front end: a ctypes face of the gb_server_* C ABI and a Poisson
load driver that reports p50/p99 latency beside throughput.

All batching, admission and device work happens in the library's scheduler
thread; this module only submits requests at their arrival times and
collects completions.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from ._binding import Completion, GoldbachError, Params, Request, ServerStats, lib

REQ_ONE, REQ_RANGE = 0, 1


class Server:
    def __init__(self, device: int = 0, streams: int = 2, max_batch: int = 4096, **params):
        self._lib = lib()
        p = Params()
        p.device = device
        for k, v in params.items():
            setattr(p, k, int(v))
        h = ctypes.c_void_p()
        st = self._lib.gb_server_start(ctypes.byref(h), ctypes.byref(p), streams, max_batch)
        if st != 0:
            raise GoldbachError(st, "gb_server_start failed")
        self._h = h
        self._keep = {}          # request id -> host buffers kept alive until completion
        self._buf = (Completion * 4096)()

    def submit_one(self, n: int, tag: int = 0) -> int:
        r = Request(kind=REQ_ONE, flags=0, n=n, len=1, pmin=None, tag=tag)
        return self._submit(r, None)

    def submit_range(self, start: int, length: int, pmin: np.ndarray | None = None,
                     tag: int = 0) -> int:
        ptr = None
        if pmin is not None:
            assert pmin.dtype == np.uint16 and pmin.size >= length and pmin.flags.c_contiguous
            ptr = pmin.ctypes.data
        r = Request(kind=REQ_RANGE, flags=0, n=start, len=length, pmin=ptr, tag=tag)
        return self._submit(r, pmin)

    def _submit(self, r, keep):
        rid = ctypes.c_uint64()
        st = self._lib.gb_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid))
        if st != 0:
            raise GoldbachError(st, "gb_server_submit rejected the request")
        if keep is not None:
            self._keep[rid.value] = keep
        return int(rid.value)

    def poll(self, wait_ms: int = 0):
        cnt = ctypes.c_size_t()
        st = self._lib.gb_server_poll(self._h, self._buf, len(self._buf), ctypes.byref(cnt), wait_ms)
        if st != 0:
            raise GoldbachError(st, "gb_server_poll failed")
        out = []
        for i in range(cnt.value):
            c = self._buf[i]
            self._keep.pop(int(c.id), None)
            out.append({"id": int(c.id), "tag": int(c.tag), "status": int(c.status),
                        "kind": "one" if c.kind == REQ_ONE else "range", "p": int(c.p),
                        "summary": c.summary.as_dict(), "submit_ns": int(c.submit_ns),
                        "launch_ns": int(c.launch_ns), "done_ns": int(c.done_ns),
                        "batch": int(c.batch_requests), "stream": int(c.stream)})
        return out

    def stats(self):
        s = ServerStats()
        self._lib.gb_server_stats_get(self._h, ctypes.byref(s))
        return s.as_dict()

    def stop(self):
        if getattr(self, "_h", None):
            self._lib.gb_server_stop(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()


def run_stream(server: Server, requests, want_pmin: bool = False, timeout_s: float = 120.0):
    """Submit each request at its arrival time (relative to now) and gather
    every completion.  Returns (completions by request index, wall seconds)."""
    t0 = time.perf_counter()
    pending = {}
    done = {}
    bufs = {}
    i = 0
    n = len(requests)
    while len(done) < n:
        now = time.perf_counter() - t0
        while i < n and requests[i]["t"] <= now:
            q = requests[i]
            if q["kind"] == "one":
                rid = server.submit_one(q["n"], tag=i)
            else:
                buf = np.zeros(q["len"], dtype=np.uint16) if want_pmin else None
                rid = server.submit_range(q["n"], q["len"], buf, tag=i)
                if buf is not None:
                    bufs[i] = buf
            pending[rid] = i
            i += 1
        for c in server.poll(wait_ms=0 if i < n else 1):
            idx = pending.pop(c["id"])
            if idx in bufs:
                c["pmin"] = bufs.pop(idx)
            done[idx] = c
        if time.perf_counter() - t0 > timeout_s:
            raise TimeoutError(f"{n - len(done)} requests still pending after {timeout_s} s")
        if i < n and not done and requests[i]["t"] > now + 1e-4:
            time.sleep(min(requests[i]["t"] - now, 1e-4))
    return done, time.perf_counter() - t0


def summarize(requests, done, wall_s):
    lat = {"one": [], "range": []}
    n_verified = 0
    for i, q in enumerate(requests):
        c = done[i]
        lat[q["kind"]].append((c["done_ns"] - c["submit_ns"]) / 1e6)
        n_verified += q["len"]
    out = {"requests": len(requests), "wall_s": wall_s, "req_per_s": len(requests) / wall_s,
           "even_n_per_s": n_verified / wall_s}
    allv = lat["one"] + lat["range"]
    for name, v in (("all", allv), ("one", lat["one"]), ("range", lat["range"])):
        if v:
            a = np.asarray(v)
            out[f"p50_ms_{name}"] = float(np.percentile(a, 50))
            out[f"p99_ms_{name}"] = float(np.percentile(a, 99))
    return out


def quick_latency(v=None, qps: float = 2000.0, count: int = 2000, streams: int = 2):
    """A short Poisson run (the benchmark's serving line)."""
    from .workloads import config5_requests
    reqs = config5_requests(seed=1, count=count, qps=qps)
    with Server(0, streams=streams) as srv:
        # warm the kernels once
        srv.submit_one(10**12)
        while not srv.poll(wait_ms=100):
            pass
        done, wall = run_stream(srv, reqs)
        stats = srv.stats()
    res = summarize(reqs, done, wall)
    res.update(qps_offered=qps, streams=streams, launches=stats["launches"],
               peak_concurrent_launches=stats["peak_concurrent_launches"],
               failures=sum(1 for c in done.values() if c["status"] != 0))
    return res
