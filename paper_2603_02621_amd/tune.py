"""Run the autotuner and write its choice as JSON.

    python -m paper_2603_02621_amd.tune [--out PATH] [--sample range|windows]

`range` (default) tunes on 16 windows of 2^27 even n cut from the range
[10^12 - 2^36, 10^12]; `windows` tunes on 256 of the seeded batched windows.
Every swept configuration must reproduce the same results; the library
reports a mismatch as an error.
"""
from __future__ import annotations

import argparse
import json
import os

from . import Verifier
from .workloads import CONFIG4, config3_windows

HERE = os.path.dirname(os.path.abspath(__file__))


def sample_windows(kind: str):
    if kind == "windows":
        return config3_windows(0, 4096)[:256]
    lo, _ = CONFIG4
    n = 1 << 27
    return [(lo + 2 * n * i, n) for i in range(16)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuned.json"))
    ap.add_argument("--sample", choices=("range", "windows"), default="range")
    args = ap.parse_args()
    with Verifier(0) as v:
        best = v.autotune(sample_windows(args.sample), args.out)
    with open(args.out) as f:
        d = json.load(f)
    d["sample_kind"] = args.sample
    with open(args.out, "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps({k: best[k] for k in ("tile_log2", "wg_threads", "search_mode", "pmax",
                                           "wheel_max", "seg_log2")}))


if __name__ == "__main__":
    main()
