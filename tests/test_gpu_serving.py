"""Serving: continuous batching gives every request the result it gets alone
(and the oracle's), admission respects the memory budget, and launches on
different streams overlap (GPU)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _small_mix(count, seed=1):
    from paper_2603_02621_amd.workloads import config5_requests
    reqs = config5_requests(seed=seed, count=count, qps=1e6)   # all arrive at once
    for q in reqs:
        if q["kind"] == "range":
            q["len"] = min(q["len"], 1 << 16)
    return reqs


def test_alone_equals_mix_equals_oracle(gpu, orc):
    from paper_2603_02621_amd import Verifier
    from paper_2603_02621_amd.serving import Server, run_stream
    reqs = _small_mix(400)
    with Server(0, streams=3, max_batch=64) as srv:
        done, _ = run_stream(srv, reqs, want_pmin=True)
        stats = srv.stats()
    assert stats["completed"] == len(reqs) and stats["launches"] > 1
    ones = [(i, q) for i, q in enumerate(reqs) if q["kind"] == "one"]
    ref_one = orc.verify_many([q["n"] for _, q in ones], threads=8)
    with Verifier(0) as v:
        alone_one = v.verify_many(np.array([q["n"] for _, q in ones], dtype=np.uint64))
        for (i, q), r, a in zip(ones, ref_one, alone_one):
            assert done[i]["status"] == 0
            assert done[i]["p"] == int(r) == int(a), q
        for i, q in enumerate(reqs):
            if q["kind"] != "range":
                continue
            c = done[i]
            assert c["status"] == 0
            hi = q["n"] + 2 * (q["len"] - 1)
            ref, _, rs = orc.verify_range(q["n"], hi, per_n_bits=16)
            out = torch.zeros(q["len"], dtype=torch.int16, device="cuda")
            alone = v.verify_windows([(q["n"], q["len"])], pmin=out)["sums"][0]
            assert np.array_equal(c["pmin"], ref)
            assert np.array_equal(out.cpu().numpy().view(np.uint16), ref)
            for k in ("count", "max_p", "argmax_n", "checksum", "n_failed"):
                assert c["summary"][k] == rs[k] == alone[k], (k, q)


def test_admission_by_memory(gpu, orc):
    from paper_2603_02621_amd import GoldbachError
    from paper_2603_02621_amd.serving import Server
    budget = 300_000            # room for two 2^16-n ranges with per-n output
    with Server(0, streams=4, max_batch=16, mem_budget=budget) as srv:
        with pytest.raises(GoldbachError):
            srv.submit_range(10**12, 1 << 20, np.zeros(1 << 20, dtype=np.uint16))
        bufs = {}
        for j in range(12):
            start = 10**13 + j * (1 << 18)
            b = np.zeros(1 << 16, dtype=np.uint16)
            bufs[srv.submit_range(start, 1 << 16, b, tag=j)] = (start, b)
        got = []
        while len(got) < 12:
            got += srv.poll(wait_ms=50)
        st = srv.stats()
    assert st["rejected"] == 1
    assert st["peak_bytes_inflight"] <= budget
    for c in got:
        start, b = bufs[c["id"]]
        ref, _, _ = orc.verify_range(start, start + 2 * ((1 << 16) - 1), per_n_bits=16)
        assert c["status"] == 0 and np.array_equal(b, ref)


def test_launches_overlap(gpu):
    from paper_2603_02621_amd.serving import Server
    with Server(0, streams=4, max_batch=4) as srv:
        ids = [srv.submit_range(10**14 + j * (1 << 23), 1 << 21) for j in range(32)]
        ids += [srv.submit_one(2 * (10**17 + j)) for j in range(64)]
        got = []
        while len(got) < len(ids):
            got += srv.poll(wait_ms=50)
        st = srv.stats()
    assert all(c["status"] == 0 for c in got)
    assert st["peak_concurrent_launches"] >= 2
    assert len({c["stream"] for c in got}) >= 2


def test_quick_latency_reports_percentiles(gpu):
    from paper_2603_02621_amd.serving import quick_latency
    r = quick_latency(qps=500, count=300)
    assert r["failures"] == 0
    assert 0 < r["p50_ms_all"] <= r["p99_ms_all"]
    assert r["requests"] == 300
