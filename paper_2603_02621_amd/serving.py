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
REQ_PMIN_DEVICE = 1


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

    def submit_range_device(self, start: int, length: int, pmin, tag: int = 0) -> int:
        """A range whose per-n p_min the kernels write into `pmin`, a device
        tensor of at least `length` 16-bit entries (kept alive by the caller
        until the completion)."""
        assert pmin.element_size() == 2 and pmin.numel() >= length and pmin.is_contiguous()
        r = Request(kind=REQ_RANGE, flags=REQ_PMIN_DEVICE, n=start, len=length, pmin=pmin.data_ptr(), tag=tag)
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


def replay(server: Server, requests, pmin_arena=None, timeout_s: float = 600.0):
    """Replay a request trace inside the library (gb_server_replay): request
    i is submitted requests[i]["t"] seconds after the start, and each
    completion's submit time is that scheduled arrival.  With `pmin_arena`
    (a device tensor of 16-bit entries, one per n of every range, ranges
    concatenated in request order) the ranges' per-n p_min are written there
    on the device.  Returns the completions in request order."""
    k = len(requests)
    R = (Request * max(k, 1))()
    arr = (ctypes.c_uint64 * max(k, 1))()
    out = (Completion * max(k, 1))()
    base = pmin_arena.data_ptr() if pmin_arena is not None else None
    off = 0
    for i, q in enumerate(requests):
        r = R[i]
        r.n = q["n"]
        r.tag = i
        if q["kind"] == "one":
            r.kind, r.len = REQ_ONE, 1
        else:
            r.kind, r.len = REQ_RANGE, q["len"]
            if base is not None:
                r.pmin = base + 2 * off
                r.flags = REQ_PMIN_DEVICE
                off += q["len"]
        arr[i] = int(round(q["t"] * 1e9))
    if pmin_arena is not None and off > pmin_arena.numel():
        raise ValueError("pmin_arena holds fewer entries than the ranges' n")
    st = server._lib.gb_server_replay(server._h, R, arr, k, out, int(timeout_s * 1000))
    if st != 0:
        raise GoldbachError(st, server._lib.gb_server_last_error(server._h).decode() or "gb_server_replay failed")
    return [{"status": int(c.status), "kind": "one" if c.kind == REQ_ONE else "range", "p": int(c.p),
             "summary": c.summary.as_dict(), "submit_ns": int(c.submit_ns), "launch_ns": int(c.launch_ns),
             "done_ns": int(c.done_ns), "batch": int(c.batch_requests), "stream": int(c.stream)}
            for c in out[:k]]


def latency_stats(requests, done):
    """Latency percentiles per class (single n, range, all) from scheduled
    arrival to completion, the queueing and device parts of it, and the
    achieved rates."""
    out = {"requests": len(requests)}
    t0 = min(c["submit_ns"] for c in done)
    t1 = max(c["done_ns"] for c in done)
    wall = (t1 - t0) / 1e9
    out["wall_s"] = wall
    out["req_per_s"] = len(requests) / wall
    out["even_n_per_s"] = sum(q["len"] for q in requests) / wall
    for name in ("all", "one", "range"):
        sel = [c for q, c in zip(requests, done) if name == "all" or q["kind"] == name]
        if not sel:
            continue
        lat = np.array([(c["done_ns"] - c["submit_ns"]) / 1e6 for c in sel])
        wait = np.array([(c["launch_ns"] - c["submit_ns"]) / 1e6 for c in sel])
        out[f"n_{name}"] = len(sel)
        out[f"p50_ms_{name}"] = float(np.percentile(lat, 50))
        out[f"p99_ms_{name}"] = float(np.percentile(lat, 99))
        out[f"max_ms_{name}"] = float(lat.max())
        out[f"p50_wait_ms_{name}"] = float(np.percentile(wait, 50))
        out[f"p99_wait_ms_{name}"] = float(np.percentile(wait, 99))
    out["failures"] = sum(1 for c in done if c["status"] != 0)
    out["mean_batch"] = float(np.mean([c["batch"] for c in done]))
    return out


def sweep(qps_list=(1e2, 3e2, 1e3, 3e3, 1e4, 3e4, 1e5), count: int = 10_000, streams: int = 4,
          seed: int = 1, per_n: bool = True, stop_factor: float = 10.0, log=None, **params):
    """Serving sweep over offered loads: the seeded request stream of the
    serving workload (the same requests at every rate, only the arrival
    times scale) replayed at each rate in `qps_list`, ranges with per-n
    output on the device.  Stops after the first rate whose overall p99
    exceeds `stop_factor` times the first rate's.  Returns one dict per rate
    with "stats" (latency_stats plus the offered rate), "done" (the
    completions), "pmin" (the device arena of per-n output, or None) and the
    requests of the stream under "requests"."""
    import torch
    from .workloads import config5_requests
    points = []
    with Server(0, streams=streams, **params) as srv:
        base = None
        for qps in qps_list:
            reqs = config5_requests(seed=seed, count=count, qps=qps)
            nr = sum(q["len"] for q in reqs if q["kind"] == "range")
            arena = torch.zeros(nr, dtype=torch.int16, device="cuda") if per_n else None
            torch.cuda.synchronize()
            done = replay(srv, reqs, arena)
            st = latency_stats(reqs, done)
            st["qps_offered"] = qps
            st["streams"] = streams
            points.append({"stats": st, "done": done, "pmin": arena, "requests": reqs})
            if log:
                log(f"# serving {qps:g} req/s offered: {st['req_per_s']:.0f} achieved, p50/p99 one "
                    f"{st.get('p50_ms_one', 0):.3f}/{st.get('p99_ms_one', 0):.3f} ms, range "
                    f"{st.get('p50_ms_range', 0):.3f}/{st.get('p99_ms_range', 0):.3f} ms")
            if base is None:
                base = st["p99_ms_all"]
            elif st["p99_ms_all"] > stop_factor * base:
                st["stop"] = f"p99 above {stop_factor:g} x the first rate's"
                break
        points[-1]["stats"]["server"] = srv.stats()
    return points


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
