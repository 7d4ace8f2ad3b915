"""The workload configurations at full size (GPU).

cfg 1 and cfg 2 are compared with the oracle n by n.  cfg 3 (4096 windows in
one persistent launch) is compared window by window.  cfg 4 is the
benchmark's range: the batched form in the benchmark's launch configuration is
checked against the plain form, against the oracle on its 2^26-n sub-slice,
on 4096 sampled n, and through properties that hold at any size (count,
histogram sums, a checksum recomputed from the per-n output).
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bench_params():
    path = os.path.join(ROOT, "paper_2603_02621_amd", "tuned.json")
    if os.path.exists(path):
        d = json.load(open(path))
        return {k: int(d[k]) for k in ("pmax", "seg_log2", "tile_log2", "wg_threads", "wheel_max", "search_mode") if k in d}
    return {}


def _same(got, ref, keys=("count", "max_p", "argmax_n", "checksum", "n_exhaustive", "n_failed")):
    for k in keys:
        assert got[k] == ref[k], (k, got[k], ref[k])


def test_config2_full(gpu, orc):
    from paper_2603_02621_amd import Verifier
    from paper_2603_02621_amd.workloads import CONFIG2, CONFIG2_PARAMS
    lo, hi = CONFIG2
    ref, rh, rs = orc.verify_range(lo, hi, pmax=CONFIG2_PARAMS["pmax"], per_n_bits=16,
                                   threads=len(os.sched_getaffinity(0)))
    with Verifier(0, **CONFIG2_PARAMS) as v:
        out = torch.zeros(len(ref), dtype=torch.int16, device="cuda")
        got = v.verify_range(lo, hi, pmin=out, seg_hist_rows=30)
        assert got["n_segments"] == 30
        assert np.array_equal(out.cpu().numpy().view(np.uint16), ref)
        assert np.array_equal(got["hist"], rh)
        assert np.array_equal(got["seg_hist"].sum(axis=0), rh)
        _same(got, rs)
        assert got["n_failed"] == 0 and got["count"] == 499_999_999


def test_config3_windows(gpu, orc):
    from paper_2603_02621_amd import Verifier
    from paper_2603_02621_amd.workloads import config3_windows
    wins = config3_windows(0, 4096)
    total = sum(n for _, n in wins)
    with Verifier(0, **_bench_params()) as v:
        out = torch.zeros(total, dtype=torch.int16, device="cuda")
        got = v.verify_windows(wins, pmin=out)
        off = 0
        hsum = np.zeros(6543, dtype=np.uint64)
        threads = len(os.sched_getaffinity(0))
        for (s, n), summ in zip(wins, got["sums"]):
            ref, rh, rs = orc.verify_range(s, s + 2 * (n - 1), per_n_bits=16, pmax=v.params["pmax"],
                                           threads=threads if n > 1 << 18 else 1)
            seg = out[off:off + n].cpu().numpy().view(np.uint16)
            assert np.array_equal(seg, ref), (s, n)
            _same(summ, rs)
            hsum += rh
            off += n
        assert np.array_equal(got["hist"], hsum)


def test_config4_bench_configuration(gpu, orc):
    from paper_2603_02621_amd import Verifier
    from paper_2603_02621_amd.workloads import CONFIG4, CONFIG4_SLICE
    lo, hi = CONFIG4
    count = (hi - lo) // 2 + 1
    with Verifier(0, **_bench_params()) as v:
        batched = v.verify_range(lo, hi, batched=True)       # the benchmark's call
        plain = v.verify_range(lo, hi)
        _same(batched, plain)
        assert np.array_equal(batched["hist"], plain["hist"])
        assert batched["count"] == count == int(batched["hist"].sum())
        assert batched["n_failed"] == 0 and batched["n_exhaustive"] == 0
        # per-n output over the whole range, in the same launch configuration
        out = torch.zeros(count, dtype=torch.int16, device="cuda")
        full = v.verify_range(lo, hi, pmin=out, batched=True)
        _same(full, batched)
        # the sub-slice of 2^26 even n ending at 10^12, n by n
        slo, shi = CONFIG4_SLICE
        ref, rh, rs = orc.verify_range(slo, shi, per_n_bits=16, threads=len(os.sched_getaffinity(0)))
        i0 = (slo - lo) // 2
        assert np.array_equal(out[i0:].cpu().numpy().view(np.uint16), ref)
        # 4096 sampled n over the whole range, one by one
        rng = np.random.default_rng(4)
        idx = np.sort(rng.integers(0, count, size=4096))
        ns = (lo + 2 * idx).astype(np.uint64)
        got_p = out[torch.from_numpy(idx).cuda()].cpu().numpy().view(np.uint16).astype(np.uint64)
        assert np.array_equal(got_p, orc.verify_many(ns, threads=8))
        # properties over all 2^35 + 1 n, recomputed from the per-n output
        primes = np.array([2] + [p for p in range(3, 65536, 2)
                                 if all(p % d for d in range(3, int(p ** 0.5) + 1, 2))], dtype=np.int64)
        h = batched["hist"].astype(np.int64)
        sum_p_hist = int((h[:6542] * primes).sum())
        sum_p, pmax = 0, 0
        cs = torch.zeros((), dtype=torch.int64, device="cuda")
        chunk = 1 << 28
        for a in range(0, count, chunk):
            p = out[a:a + chunk].to(torch.int32) & 0xFFFF
            sum_p += int(p.sum(dtype=torch.int64))
            pmax = max(pmax, int(p.max()))
            n = 2 * (torch.arange(a, a + p.numel(), device="cuda", dtype=torch.int64) + lo // 2)
            k = torch.div(n, 6, rounding_mode="floor")
            j = k & 63
            b = 3 * (k >> 6) + ((n - 6 * k) >> 1)
            w = (b << 33) + ((2 * (j >> 5) + 1) << (j & 31))
            cs += (w * p.to(torch.int64)).sum()   # int64 arithmetic wraps mod 2^64
            del p, n, k, j, b, w
        assert sum_p == sum_p_hist
        assert int(cs) % 2**64 == batched["checksum"]
        assert pmax == batched["max_p"]
