"""Benchmark: even n verified per second at N ~ 10^12 on one MI355X.

Workload: every even n in [10^12 - 2^36, 10^12] (2^35 + 1 of them), summaries
only (count, histogram, max p and its n, checksum), sieving primes up to
sqrt(10^12 + ...) resident.  One step is one complete verification of that
range.  The timed form is the batched one (one persistent tile launch in a
replayed HIP graph); the plain form (one launch per segment of S even n) is
timed beside it.  Prints one JSON line.

Beside it: the bulk form, the batched windows, partition counts, even n
beyond 64 bits, and a serving sweep (the seeded request stream replayed at
increasing offered rates, p50/p99 per request class), every request of which
the CPU leg re-verifies with the oracle.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-serve]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

# The plain form runs as many segments side by side as the process has
# hardware queues (the library reads GPU_MAX_HW_QUEUES, HIP's default 4);
# eight fill the device with its tiles.  Raised before HIP starts.
if int(os.environ.get("GPU_MAX_HW_QUEUES") or 4) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LO, HI = 10**12 - 2**36, 10**12
METRIC = "even n verified/s at N~1e12 on 1 MI355X (batched form)"

# Per-n algorithmic work of the sieve-and-search kernel at this workload
# (every even n of [1e12 - 2^36, 1e12], fast path P_max = 4096, tiles of
# T = 2^20 even n), counted in int32 lane operations and fixed here:
#  - sieve bit clears: the sum of 1/p over the sieving primes 11 <= p <= 10^6
#    is 1.711 clears per odd number, 3 ops each (next index, word, mask);
#  - wheel pattern: one 32-bit word store per 32 odd numbers, 5 ops each;
#  - first strikes: pi(10^6) - 1 = 78,497 odd sieving primes per tile, one
#    64-bit remainder (10 ops) each, per 2^20 n;
#  - window probes: 1.01 64-bit probes per n (the mean over 64-n blocks of
#    the largest prime index the block needs, 64.68, divided by 64), 7 ops
#    each (offset, word, two funnel shifts, two ANDs, test);
#  - hit bookkeeping: 29.9 distinct p_min per 64-n block, 0.467 hit events
#    per n, 8 ops each (clear the resolved n from the block mask: 2, popcount
#    for the histogram: 2, count add: 1, checksum multiply-adds: 3).
# This is the work of the method as the paper states it (a sieve of the odd
# numbers, every odd prime probed for every n), kept as the fixed unit: the
# kernel that runs (k_cls) splits n and q by residue mod 6 and does less of
# it (2/3 of the odd numbers sieved, 0.55 probes per n), so its rate in
# these units can exceed what the same kernel would reach counting its own
# operations.
CLEARS_PER_N = 1.711
PROBES_PER_N = 1.01
HITS_PER_N = 29.9 / 64
STRIKES_PER_N = 78497 / 2**20
ALG_OPS_PER_N = (CLEARS_PER_N * 3 + 5 / 32 + STRIKES_PER_N * 10 + PROBES_PER_N * 7
                 + HITS_PER_N * 8)
# Integer VALU peak: 157.3 TFLOP/s fp32 vector = 78.6e12 FMA lane-slots per
# second (256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz); one int32 op per slot.
ALU_PEAK_OPS = 256 * 4 * 32 * 2.4e9
PC_N, PC_HI = 1 << 16, 10**9        # partition-count workload: 2^16 even n ending at 1e9
BIG_N = 4096                        # beyond-64-bit workload: even n from 10^100 upward

# HBM bytes per launch of the tile kernel on this workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB copy's readings (factors 2.000
# and 1.000), valid only for the kernel sources and compiler flags they were
# taken with.
TRAFFIC = {"kernel_sha256_prefix": "d4250e8d76ca0699", "tile_log2": 20, "wg_threads": 1024,
           "bytes_per_launch": 18.733e6 + 1.293e6}
KERNEL_SOURCES = ("gb_class.hip", "gb_device.h", "gb_internal.h")


def _load_tuned():
    path = os.path.join(ROOT, "paper_2603_02621_amd", "tuned.json")
    if os.path.exists(path):
        with open(path) as f:
            d = json.load(f)
        return {k: int(d[k]) for k in ("pmax", "seg_log2", "tile_log2", "wg_threads", "wheel_max", "search_mode")
                if k in d}
    return {}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(threads: int, log2n: int = 30, serving_points=None):
    """The oracle as it stands, timed on the host cores: a bounded sample of
    the bench range on every core; the paper's CPU-baseline workloads
    (every even n up to 10^6 and up to 10^9) on one core and on every core;
    and the re-verification of every request of the serving sweep, whose
    mismatches are written into each sweep point."""
    import oracle
    oracle.build(force=False)
    lo = HI - 2 * ((1 << log2n) - 1)
    t0 = time.perf_counter()
    _, _, s = oracle.verify_range(lo, HI, per_n_bits=None, hist=True, threads=threads)
    dt = time.perf_counter() - t0
    out = {"value": s["count"] / dt, "unit": "even n/s", "cores": threads, "kind": "oracle",
           "sample": f"2^{log2n} even n ending at 1e12 ({s['count']} n, {dt:.2f} s wall)",
           "cpu_model": _cpu_model()}
    table = []
    for hi, th in ((10**6, 1), (10**9, 1), (10**9, threads)):
        t0 = time.perf_counter()
        _, _, r = oracle.verify_range(4, hi, per_n_bits=None, hist=True, threads=th)
        dt = time.perf_counter() - t0
        table.append({"workload": f"every even n in [4, {hi:.0e}]", "threads": th, "seconds": dt,
                      "even_n_per_s": r["count"] / dt, "n_failed": r["n_failed"]})
        print(f"# oracle [4, {hi:.0e}] on {th} thread(s): {dt:.2f} s", file=sys.stderr, flush=True)
    out["paper_workloads"] = table
    if serving_points:
        out["serving_reverify"] = reverify_serving(serving_points, threads)
    return out


def reverify_serving(points, threads: int):
    """Every request of the serving sweep checked against the oracle: p of
    each single n, and the summary and every per-n p_min of each range.  The
    stream's requests are the same at every rate, so the oracle runs once."""
    import numpy as np
    import oracle
    reqs = points[0]["requests"]
    ones = [(i, q["n"]) for i, q in enumerate(reqs) if q["kind"] == "one"]
    rngs = [(i, (q["n"], q["len"])) for i, q in enumerate(reqs) if q["kind"] == "range"]
    t0 = time.perf_counter()
    ref_p = oracle.verify_many([n for _, n in ones], threads=threads)
    t1 = time.perf_counter()
    ref_out, ref_sums = oracle.verify_windows([w for _, w in rngs], threads=threads)
    t2 = time.perf_counter()
    keys = ("count", "max_p", "argmax_n", "checksum", "n_failed")
    for pt in points:
        done = pt["done"]
        bad_one = sum(1 for (i, _), p in zip(ones, ref_p) if done[i]["p"] != int(p))
        bad_sum = sum(1 for (i, _), r in zip(rngs, ref_sums)
                      if any(done[i]["summary"][k] != r[k] for k in keys))
        bad_n = None
        if pt["pmin"] is not None:
            got = pt["pmin"].cpu().numpy().view(np.uint16)
            bad_n = int(np.count_nonzero(got != ref_out))
            pt["pmin"] = None
        pt["stats"]["oracle_mismatches"] = {"one": bad_one, "range_summary": bad_sum, "range_per_n": bad_n}
    n_range = int(sum(w[1] for _, w in rngs))
    print(f"# oracle re-verification of the serving stream: {t1 - t0:.2f} s for {len(ones)} single n, "
          f"{t2 - t1:.2f} s for {len(rngs)} ranges ({n_range} n)", file=sys.stderr, flush=True)
    return {"single_n": len(ones), "single_s": t1 - t0, "ranges": len(rngs), "range_n": n_range,
            "range_s": t2 - t1, "range_even_n_per_s": n_range / (t2 - t1), "threads": threads}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--no-windows", action="store_true")
    ap.add_argument("--params", default="", help="JSON object of gb_params fields overriding the tuned ones")
    ap.add_argument("--no-bulk", action="store_true", help="skip the bulk-verification line")
    ap.add_argument("--no-pcount", action="store_true", help="skip the partition-count line")
    ap.add_argument("--no-big", action="store_true", help="skip the beyond-64-bit line")
    ap.add_argument("--serve-count", type=int, default=10_000,
                    help="requests per offered rate of the serving sweep")
    ap.add_argument("--serve-qps", default="1e2,3e2,1e3,3e3,1e4,3e4,1e5,3e5,1e6",
                    help="offered rates of the serving sweep, comma-separated")
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of this many MiB (a reference "
                         "kernel of known traffic for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the verifier shards segments across GPUs by "
              "design, but this build runs and reports a single MI355X (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_02621_amd import Verifier

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    params = _load_tuned()
    if args.params:
        params.update({k: int(v) for k, v in json.loads(args.params).items()})
    v = Verifier(0, **params)
    p = v.params
    geo = v.geometry
    print(f"# params {p} geometry {geo}", file=sys.stderr, flush=True)

    # ---- batched (timed) --------------------------------------------------
    for _ in range(args.warmup):
        w = v.verify_range(LO, HI, batched=True)
        print(f"# warmup batched {w['device_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tile_ms, dev_ms = [], []
    ref = None
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = v.verify_range(LO, HI, batched=True)
        tile_ms.append(r["tile_ms"])
        dev_ms.append(r["device_ms"])
        if ref is None:
            ref = r
        assert r["checksum"] == ref["checksum"] and r["count"] == ref["count"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    count = ref["count"]
    ms_per_step = 1e3 * wall / args.steps
    value = count * args.steps / wall
    print(f"# batched: {ms_per_step:.1f} ms/step, tile kernel {sum(tile_ms)/len(tile_ms):.1f} ms",
          file=sys.stderr, flush=True)

    # ---- plain (beside it) ------------------------------------------------
    # The paper's segment loop: one tile launch per segment of S even n,
    # consecutive segments on four streams; at the tuned S (2^20 .. 2^26)
    # and at S = 2^24 with tiles of 2^18 n (64 tiles per segment: the tile
    # size at which four segments in flight cover the device).
    plain = []
    if args.plain_steps > 0:
        forms = [("tuned", {}), ("s24", {"seg_log2": 24, "tile_log2": 18, "wg_threads": 1024})]
        for name, over in forms:
            if name == "tuned" and p["seg_log2"] > 26:
                over = {"seg_log2": 26}
            vp = v if not over else Verifier(0, **{**params, **over})
            pp = vp.params
            vp.verify_range(LO, LO + 2 * ((1 << 28) - 1), batched=False)    # code and buffers warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plain_tile = []
            for _ in range(args.plain_steps):
                rp = vp.verify_range(LO, HI, batched=False)
                plain_tile.append(rp["tile_ms"])
            torch.cuda.synchronize()
            plain_wall = (time.perf_counter() - t0) / args.plain_steps
            for k in ("count", "checksum", "max_p", "argmax_n", "n_exhaustive", "n_failed"):
                assert rp[k] == ref[k], k
            t_tiles = sum(plain_tile) / len(plain_tile) / 1e3
            ach = ALG_OPS_PER_N * count / t_tiles
            print(f"# plain S=2^{pp['seg_log2']} T=2^{pp['tile_log2']}: {1e3*plain_wall:.1f} ms/step over "
                  f"{rp['n_segments']} segment launches", file=sys.stderr, flush=True)
            plain.append({"form": name, "seg_log2": pp["seg_log2"], "tile_log2": pp["tile_log2"],
                          "wg_threads": pp["wg_threads"], "value": count / plain_wall,
                          "ms_per_step": 1e3 * plain_wall, "segments": rp["n_segments"],
                          "streams": 4, "tile_phase_ms": 1e3 * t_tiles,
                          "vs_batched": value / (count / plain_wall),
                          "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": ALU_PEAK_OPS / 1e12,
                                       "unit": "Tops/s (int32 lane ops)", "frac": ach / ALU_PEAK_OPS,
                                       "alg_ops_per_n": round(ALG_OPS_PER_N, 3)}})
            if vp is not v:
                vp.close()

    # ---- bulk verification of the same range (no per-n minimal p) --------
    bulk = None
    if not args.no_bulk:
        v.verify_range_bulk(LO, HI)                  # graph capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bulk_tile = []
        for _ in range(2):
            rb = v.verify_range_bulk(LO, HI)
            bulk_tile.append(rb["tile_ms"])
        torch.cuda.synchronize()
        bulk_wall = (time.perf_counter() - t0) / 2
        for k in ("count", "max_p", "argmax_n", "n_exhaustive", "n_failed"):
            assert rb[k] == ref[k], k
        print(f"# bulk: {1e3*bulk_wall:.1f} ms/step, tile kernel {sum(bulk_tile)/2:.1f} ms",
              file=sys.stderr, flush=True)
        bulk = {"value": count / bulk_wall, "ms_per_step": 1e3 * bulk_wall,
                "tile_launch_ms": sum(bulk_tile) / 2,
                "reports": "count, max p_min and its n, n_exhaustive, n_failed (no per-n p, histogram or checksum)"}

    # ---- batched windows: 4096 uneven windows in one persistent launch ---
    windows = None
    if not args.no_windows:
        from paper_2603_02621_amd.workloads import config3_windows
        wins = config3_windows(0, 4096)
        wn = sum(n for _, n in wins)
        v.verify_windows(wins, sums=False)           # graph capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            v.verify_windows(wins, sums=False)
        torch.cuda.synchronize()
        wt = (time.perf_counter() - t0) / 2
        windows = {"windows": len(wins), "even_n": wn, "ms_per_step": 1e3 * wt, "value": wn / wt}
        print(f"# windows: {1e3*wt:.1f} ms for {wn} n in 4096 windows", file=sys.stderr, flush=True)

    # ---- Goldbach partition counts c(n) of 2^16 even n ending at 1e9 -------
    pcount = None
    if not args.no_pcount:
        pc_lo, pc_hi = PC_HI - 2 * (PC_N - 1), PC_HI
        v.partition_counts(pc_lo, pc_hi)             # buffers
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pk = []
        for _ in range(2):
            rp = v.partition_counts(pc_lo, pc_hi)
            pk.append(rp["kernel_ms"])
        torch.cuda.synchronize()
        pc_wall = (time.perf_counter() - t0) / 2
        # AND + popcount per 32 candidate pairs (p, n - p), p <= n/2: for even
        # n >= 6 the odd p = 2i + 1 with i <= floor((n/2 - 1)/2), in words of 32 i
        words = sum((((n // 2) - 1) // 2) // 32 + 1 for n in range(pc_lo, pc_hi + 1, 2))
        pc_t = sum(pk) / len(pk) / 1e3
        pc_ach = 2 * words / pc_t
        print(f"# partition counts: {1e3*pc_wall:.1f} ms/step, kernel {1e3*pc_t:.1f} ms",
              file=sys.stderr, flush=True)
        pcount = {"workload": f"Goldbach partition counts c(n) of the {PC_N} even n ending at {PC_HI}",
                  "value": PC_N / pc_wall, "unit": "even n/s", "ms_per_step": 1e3 * pc_wall,
                  "kernel_ms": 1e3 * pc_t,
                  "summary": {k: rp[k] for k in ("count", "sum", "min_c", "argmin_n", "max_c", "argmax_n")},
                  "roofline": {"bound": "alu", "achieved": pc_ach / 1e12, "peak": ALU_PEAK_OPS / 1e12,
                               "unit": "Tops/s (int32 lane ops)", "frac": pc_ach / ALU_PEAK_OPS,
                               "kernel": "k_pcount_res", "alg_ops": "2 per 32 candidate pairs",
                               "alg_ops_per_launch": 2 * words}}

    # ---- even n beyond 64 bits: 4096 n from 10^100 upward ----------------
    bign = None
    if not args.no_big:
        ns = [10**100 + 2 * i for i in range(BIG_N)]
        nl = (max(ns).bit_length() + 31) // 32
        words = np.frombuffer(b"".join(x.to_bytes(4 * nl, "little") for x in ns), dtype="<u4").reshape(BIG_N, nl)
        v.verify_big_words(words)                     # code, tables and buffers warm
        torch.cuda.synchronize()
        # the C call on limbs in host memory (what a C caller passes) ...
        t0 = time.perf_counter()
        for _ in range(5):
            ps = v.verify_big_words(words).tolist()
        big_wall = (time.perf_counter() - t0) / 5
        # ... and through the Python integers (their marshalling included)
        t0 = time.perf_counter()
        for _ in range(3):
            ps_int = v.verify_big(ns)
        big_wall_int = (time.perf_counter() - t0) / 3
        assert ps_int == ps
        # algorithmic work: for each n, a base-2 strong test of q = n - p for
        # every odd prime p up to p_min that no odd base 3 .. 97 rules out
        # (r | q), and 24 more tests of p_min's q.  A strong test of a b-bit q
        # to a small base is b - 1 Montgomery squarings (its multiplications
        # by the base cost O(k), not O(k^2), and are not counted); a product
        # is 2 k^2 32-bit multiply-adds with k = ceil(b / 32)
        odd_bases = (3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61, 67, 71, 73, 79,
                     83, 89, 97)
        primes_small = [q for q in range(3, max(ps) + 1, 2) if all(q % d for d in range(3, int(q**0.5) + 1, 2))]
        pres = [[q % r for r in odd_bases] for q in primes_small]
        mads = 0
        for n, pm in zip(ns, ps):
            b = n.bit_length()
            k = (b + 31) // 32
            nres = [n % r for r in odd_bases]
            tests2 = sum(1 for q, qr in zip(primes_small, pres)
                         if q <= pm and all(a != c for a, c in zip(qr, nres)))
            mads += (tests2 + 24) * (b - 1) * 2 * k * k
        print(f"# big n: {1e3*big_wall:.2f} ms for {BIG_N} n near 1e100 "
              f"({1e3*big_wall_int:.2f} ms from Python integers)", file=sys.stderr, flush=True)
        bign = {"workload": f"minimal p of the {BIG_N} even n from 10^100 upward (333 bits)",
                "value": BIG_N / big_wall, "unit": "even n/s", "ms_per_step": 1e3 * big_wall,
                "timed": "gb_verify_big on the n as 32-bit limbs in host memory (the C call)",
                "ms_per_step_python_ints": 1e3 * big_wall_int,
                "max_p": max(ps), "alg_mads": mads, "alg_mads_per_s": mads / big_wall}

    # ---- measured ceilings of the units (beside the nominal peaks) --------
    peaks = v.measure_peaks()

    if args.copy_calibrate:
        nb = args.copy_calibrate << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy calibration: {nb} bytes read, {nb} bytes written", file=sys.stderr, flush=True)

    # ---- roofline of the dominant kernel ------------------------------------
    t_launch = sum(tile_ms) / len(tile_ms) / 1e3
    achieved = ALG_OPS_PER_N * count / t_launch
    import hashlib
    # the kernel's sources and the compiler flags they were built with (paths left out)
    from paper_2603_02621_amd.build import HIPCC_FLAGS
    flags = " ".join(f for f in HIPCC_FLAGS if "/" not in f).encode()
    text = b"".join(open(os.path.join(ROOT, "paper_2603_02621_amd", "csrc", f), "rb").read()
                    for f in KERNEL_SOURCES)
    sha = hashlib.sha256(text + flags).hexdigest()[:16]
    same = (sha == TRAFFIC["kernel_sha256_prefix"] and p["tile_log2"] == TRAFFIC["tile_log2"]
            and p["wg_threads"] == TRAFFIC["wg_threads"])
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK_OPS / 1e12,
            "unit": "Tops/s (int32 lane ops)", "frac": achieved / ALU_PEAK_OPS,
            "traffic": TRAFFIC["bytes_per_launch"] if same else None,
            "traffic_unit": "bytes per launch (HBM, rocprofv3)",
            "kernel": "k_cls (persistent)", "kernel_sha256_prefix": sha, "launch_ms": t_launch * 1e3,
            "alg_ops_per_n": round(ALG_OPS_PER_N, 3),
            "frac_of_measured": {"valu_vop2": achieved / peaks["valu_vop2_ops"],
                                 "valu_vop3": achieved / peaks["valu_vop3_ops"]}}
    if bign is not None:
        bign["frac_of_measured_valu_vop3"] = bign["alg_mads_per_s"] / peaks["valu_vop3_ops"]
    if pcount is not None:
        pcount["roofline"]["frac_of_measured"] = {
            "valu_vop2": pc_ach / peaks["valu_vop2_ops"], "valu_vop3": pc_ach / peaks["valu_vop3_ops"]}

    out = {
        "metric": METRIC, "value": value, "unit": "even n/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32/u64 integer", "data": "synthetic (deterministic integer range)",
        "config": {"workload": "all even n in [1e12-2^36, 1e12], summaries only",
                   "n_per_step": count, "pmax": p["pmax"], "seg_log2": p["seg_log2"],
                   "tile_log2": p["tile_log2"], "wg_threads": p["wg_threads"],
                   "wheel_max": p["wheel_max"], "tile_n": geo["cls_tile_n"],
                   "tile_lds_bytes": geo["cls_lds_bytes"], "parallelism": "1 GPU"},
        "plain": plain,
        "batched_windows": windows,
        "bulk_verify": bulk,
        "partition_counts": pcount,
        "big_n": bign,
        "summary": {k: ref[k] for k in ("count", "max_p", "argmax_n", "checksum",
                                        "n_exhaustive", "n_failed")},
        "roofline": roof,
        "measured_peaks": peaks,
    }

    v.close()
    points = None
    if not args.no_serve:
        from paper_2603_02621_amd import serving
        qps = [float(x) for x in args.serve_qps.split(",") if x]
        log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
        points = serving.sweep(qps, count=args.serve_count, streams=args.serve_streams, log=log)
        out["serving_sweep"] = [pt["stats"] for pt in points]
    if not args.no_cpu:
        threads = len(os.sched_getaffinity(0))
        out["cpu_baseline"] = cpu_baseline(threads, serving_points=points)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
