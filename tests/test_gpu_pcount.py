"""Goldbach partition counts c(n) on the GPU against the CPU oracle (GPU).

Bit-exact: c(n) is an integer with one correct value.  Ranges span several
512-n workgroup blocks, ragged tails, odd ends, the n = 4 special case, and
blocks whose steps are split over many workgroups; at the benchmark's size
(2^16 even n ending at 10^9) a sample of n is compared one by one and the
summaries are recomputed from the per-n counts.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BENCH_LO, BENCH_HI = 10**9 - 2 * (2**16 - 1), 10**9


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def V():
    _gpu()
    from paper_2603_02621_amd import Verifier
    v = Verifier(0)
    yield v
    v.close()


def _n_list(lo, hi):
    first = max(lo, 4)
    first += first & 1
    last = hi - (hi & 1)
    return np.arange(first, last + 1, 2, dtype=np.uint64) if first <= last else np.zeros(0, np.uint64)


def _summary_of(ns, cs):
    cs = np.asarray(cs, dtype=np.uint64)
    if cs.size == 0:
        return {"count": 0, "sum": 0, "min_c": 0, "argmin_n": 0, "max_c": 0, "argmax_n": 0}
    imin, imax = int(np.argmin(cs)), int(np.argmax(cs))   # first occurrence = smallest n
    return {"count": int(cs.size), "sum": int(cs.sum(dtype=np.uint64)), "min_c": int(cs[imin]),
            "argmin_n": int(ns[imin]), "max_c": int(cs[imax]), "argmax_n": int(ns[imax])}


@pytest.mark.parametrize("lo,hi", [
    (4, 20_000),                        # n = 4, then 20 blocks of 512 n
    (4, 4), (6, 6), (8, 8), (4, 10),
    (5, 131),                           # odd ends, one partial block
    (10**6 - 2 * 4095, 10**6),          # 8 blocks exactly
    (10**7 - 2 * 1500, 10**7 + 1),      # ragged tail; steps split over many workgroups
    (123_456_788, 123_456_788 + 2 * 700),
])
def test_counts_vs_oracle(V, orc, lo, hi):
    ns = _n_list(lo, hi)
    ref, rs = orc.partition_counts(ns, threads=8)
    out = torch.full((max(ns.size, 1),), -1, dtype=torch.int64, device="cuda")
    got = V.partition_counts(lo, hi, counts=out)
    torch.cuda.synchronize()
    dev = out.cpu().numpy().view(np.uint64)[:ns.size]
    bad = np.nonzero(dev != ref)[0]
    assert bad.size == 0, [(int(ns[i]), int(dev[i]), int(ref[i])) for i in bad[:10]]
    for k in rs:
        assert got[k] == rs[k], (k, got[k], rs[k])


def test_summaries_only_equal_counts_form(V):
    lo, hi = 10**7 - 2 * 3000, 10**7
    out = torch.zeros(3001, dtype=torch.int64, device="cuda")
    a = V.partition_counts(lo, hi, counts=out)
    b = V.partition_counts(lo, hi)
    for k in ("count", "sum", "min_c", "argmin_n", "max_c", "argmax_n"):
        assert a[k] == b[k], k


def test_empty_and_limits(V):
    from paper_2603_02621_amd import GoldbachError
    e = V.partition_counts(100, 50)
    assert e["count"] == 0 and e["sum"] == 0
    assert V.partition_counts(3, 3)["count"] == 0
    with pytest.raises(GoldbachError):
        V.partition_counts(4, 4 + 2 * (1 << 25))          # more than 2^25 n
    with pytest.raises(GoldbachError):
        V.partition_counts(1 << 51, (1 << 51) + 100)      # above max_hi


def test_bench_size_sampled(V, orc):
    ns = _n_list(BENCH_LO, BENCH_HI)
    assert ns.size == 2**16
    out = torch.zeros(ns.size, dtype=torch.int64, device="cuda")
    got = V.partition_counts(BENCH_LO, BENCH_HI, counts=out)
    torch.cuda.synchronize()
    dev = out.cpu().numpy().view(np.uint64)
    # 256 n: for every residue of m = n/2 - 1 mod 32 (each residue is its
    # own wavefront), its first and last n, its n on both sides of two edges
    # of the 2048-m blocks a group of workgroups covers, and four more from a
    # seeded draw
    m = ns // 2 - 1
    rng = np.random.default_rng(7)
    idx = []
    for r in range(32):
        where = np.nonzero(m % 32 == r)[0]
        edges = [np.searchsorted(m[where], e) for e in (m[0] - m[0] % 2048 + 2048 * 3,
                                                        m[0] - m[0] % 2048 + 2048 * 17)]
        pick = [0, where.size - 1] + [e for e in edges] + [e - 1 for e in edges]
        pick += list(rng.integers(0, where.size, size=4))
        idx += [int(where[min(max(i, 0), where.size - 1)]) for i in pick]
    idx = np.unique(np.array(idx))
    assert idx.size >= 240 and len(set((m[idx] % 32).tolist())) == 32
    ref, _ = orc.partition_counts(ns[idx], threads=16)
    assert np.array_equal(dev[idx], ref), list(zip(ns[idx], dev[idx], ref))
    # summaries agree with the per-n counts
    assert got == {**_summary_of(ns, dev), "device_ms": got["device_ms"],
                   "kernel_ms": got["kernel_ms"]}
    # every n in this range has a partition
    assert got["min_c"] > 0

