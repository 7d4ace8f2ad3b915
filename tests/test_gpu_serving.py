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


def _mix(count, seed=1):
    from paper_2603_02621_amd.workloads import config5_requests
    return config5_requests(seed=seed, count=count, qps=1e6)   # all arrive at once


def test_alone_equals_mix_equals_oracle(gpu, orc):
    # the serving workload's requests at their full lengths (ranges up to
    # 2^22 n near 10^12 .. 10^15), all submitted at once so that the
    # scheduler batches them; every range asks for per-n output, half of
    # them into host memory and half into device memory
    from paper_2603_02621_amd import Verifier
    from paper_2603_02621_amd.serving import REQ_PMIN_DEVICE, Server
    reqs = _mix(240)
    rngs = [(i, q) for i, q in enumerate(reqs) if q["kind"] == "range"]
    ones = [(i, q) for i, q in enumerate(reqs) if q["kind"] == "one"]
    assert max(q["len"] for _, q in rngs) > 2**21 and len(rngs) >= 40
    host_out, dev_out = {}, {}
    with Server(0, streams=3, max_batch=64) as srv:
        ids = {}
        for j, (i, q) in enumerate(rngs):
            if j % 2:
                b = np.zeros(q["len"], dtype=np.uint16)
                host_out[i] = b
                ids[srv.submit_range(q["n"], q["len"], b, tag=i)] = i
            else:
                t = torch.zeros(q["len"], dtype=torch.int16, device="cuda")
                dev_out[i] = t
                ids[srv.submit_range_device(q["n"], q["len"], t, tag=i)] = i
        for i, q in ones:
            ids[srv.submit_one(q["n"], tag=i)] = i
        done = {}
        while len(done) < len(reqs):
            for c in srv.poll(wait_ms=50):
                done[ids[c["id"]]] = c
        stats = srv.stats()
    assert stats["completed"] == len(reqs) and stats["launches"] > 1
    ref_one = orc.verify_many([q["n"] for _, q in ones], threads=8)
    ref_out, ref_sums = orc.verify_windows([(q["n"], q["len"]) for _, q in rngs], threads=8)
    with Verifier(0) as v:
        alone_one = v.verify_many(np.array([q["n"] for _, q in ones], dtype=np.uint64))
        for (i, q), r, a in zip(ones, ref_one, alone_one):
            assert done[i]["status"] == 0
            assert done[i]["p"] == int(r) == int(a), q
        off = 0
        for (i, q), rs in zip(rngs, ref_sums):
            c = done[i]
            assert c["status"] == 0
            ref = ref_out[off:off + q["len"]]
            off += q["len"]
            got = host_out[i] if i in host_out else dev_out[i].cpu().numpy().view(np.uint16)
            assert np.array_equal(got, ref), q
            out = torch.zeros(q["len"], dtype=torch.int16, device="cuda")
            alone = v.verify_windows([(q["n"], q["len"])], pmin=out)["sums"][0]
            assert np.array_equal(out.cpu().numpy().view(np.uint16), ref)
            for k in ("count", "max_p", "argmax_n", "checksum", "n_failed"):
                assert c["summary"][k] == rs[k] == alone[k], (k, q)


def test_replay_equals_oracle_and_orders_times(gpu, orc):
    # the library's trace replay at 3000 requests/s: every result equals the
    # oracle's, the device per-n output of every range too, and each
    # completion's times are ordered (scheduled arrival <= launch <= done)
    from paper_2603_02621_amd.serving import Server, latency_stats, replay
    from paper_2603_02621_amd.workloads import config5_requests
    reqs = config5_requests(seed=3, count=600, qps=3000.0)
    nr = sum(q["len"] for q in reqs if q["kind"] == "range")
    arena = torch.zeros(nr, dtype=torch.int16, device="cuda")
    with Server(0, streams=4) as srv:
        done = replay(srv, reqs, arena)
    st = latency_stats(reqs, done)
    assert st["failures"] == 0 and st["requests"] == 600
    assert 0 < st["p50_ms_one"] <= st["p99_ms_one"] and 0 < st["p50_ms_range"] <= st["p99_ms_range"]
    for c in done:
        assert c["submit_ns"] <= c["launch_ns"] <= c["done_ns"]
    ones = [(i, q["n"]) for i, q in enumerate(reqs) if q["kind"] == "one"]
    ref_p = orc.verify_many([n for _, n in ones], threads=8)
    assert [done[i]["p"] for i, _ in ones] == [int(p) for p in ref_p]
    rngs = [(i, (q["n"], q["len"])) for i, q in enumerate(reqs) if q["kind"] == "range"]
    ref_out, ref_sums = orc.verify_windows([w for _, w in rngs], threads=8)
    assert np.array_equal(arena.cpu().numpy().view(np.uint16), ref_out)
    for (i, _), rs in zip(rngs, ref_sums):
        for k in ("count", "max_p", "argmax_n", "checksum", "n_failed"):
            assert done[i]["summary"][k] == rs[k]


def test_replay_rejects_malformed_trace(gpu):
    from paper_2603_02621_amd import GoldbachError
    from paper_2603_02621_amd.serving import Server, replay
    with Server(0, streams=1) as srv:
        with pytest.raises(GoldbachError):
            replay(srv, [{"t": 0.0, "kind": "one", "n": 7, "len": 1}])
        with pytest.raises(GoldbachError):     # arrival times out of order
            replay(srv, [{"t": 0.002, "kind": "one", "n": 10**12, "len": 1},
                         {"t": 0.001, "kind": "one", "n": 10**12 + 2, "len": 1}])
        assert replay(srv, []) == []


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
