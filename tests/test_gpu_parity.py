"""Parity of the HIP path with the CPU oracle, element by element (GPU).

Every comparison is bit-exact: the method is integer arithmetic, and p_min(n)
has exactly one correct value.  Inputs are deterministic ranges or seeded
windows; sizes span several tiles and a ragged tail.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def _make(**kw):
    from paper_2603_02621_amd import Verifier
    return Verifier(0, **kw)


def _unpack(words_t, nbits):
    w = words_t.cpu().numpy().view(np.uint32)
    bits = np.unpackbits(w.view(np.uint8), bitorder="little")
    return bits[:nbits]


def _dev_pmin(count, bits=16):
    dt = torch.int16 if bits == 16 else torch.int32
    return torch.zeros(count, dtype=dt, device="cuda")


def _host(t):
    a = t.cpu().numpy()
    return a.view(np.uint16) if a.dtype.itemsize == 2 else a.view(np.uint32)


def _same_summary(got, ref):
    for k in ("count", "max_p", "argmax_n", "checksum", "n_exhaustive", "n_failed",
              "first_failed_n"):
        assert got[k] == ref[k], (k, got[k], ref[k])


# --------------------------------------------------------------------------
# the LDS tile sieve alone
# --------------------------------------------------------------------------

@pytest.mark.parametrize("w0,nbits", [
    (1, 1 << 20),                                  # 1, the wheel primes, small squares
    (10**12 - (1 << 21) + 1, 1 << 21),             # near 10^12
    (1_000_003**2 - (1 << 19), 1 << 20),           # across 1000003^2
    ((1 << 50) - (1 << 22) - 1, 1 << 20),          # top of the default table
    (999_999_999_999_999_001, 64 * 4099),          # ragged tile count
    ((1 << 53) - (1 << 21) - 1, 1 << 20),          # last windows whose start is below 2^53
    ((1 << 53) - (1 << 20) + 1, 1 << 20),          # tiles on both sides of 2^53
])
def test_sieve_window_vs_oracle(orc, w0, nbits):
    _gpu()
    from paper_2603_02621_amd import Verifier
    v = Verifier(0, max_hi=max(1 << 50, w0 + 2 * nbits + 2))
    out = torch.zeros(nbits // 32, dtype=torch.int32, device="cuda")
    v.sieve_window(w0, nbits, out)
    torch.cuda.synchronize()
    got = _unpack(out, nbits)
    ref = orc.odd_primality(w0, nbits)
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, [(int(w0 + 2 * i), int(got[i]), int(ref[i])) for i in bad[:10]]
    v.close()


@pytest.mark.parametrize("k0,nk,kw", [
    (0, 64 * 300, {}),                                      # 1, the wheel primes, small squares
    (10**12 // 6 // 64 * 64 - 64 * 9000, 64 * 11000, {}),  # near 10^12, several tiles, ragged
    ((1_000_003**2 // 6) // 64 * 64 - 64 * 3000, 64 * 7000, dict(tile_log2=16, wheel_max=19)),
    ((1 << 50) // 6 // 64 * 64 - 64 * 6000, 64 * 5500, dict(tile_log2=20, wheel_max=7, wg_threads=256)),
    (((1 << 53) // 6) // 64 * 64 - 64 * 3000, 64 * 6000, dict(max_hi=1 << 54)),   # both sides of 2^53
])
def test_sieve_planes_vs_oracle(orc, k0, nk, kw):
    # the planes of the minimal-p search: bit k of plane i is 6 (k0 + k) + c_i
    # prime, c = (1, 5); the oracle's odd-number sieve picked apart
    _gpu()
    from paper_2603_02621_amd import Verifier
    kw = dict(kw)
    kw.setdefault("max_hi", 1 << 50)
    v = Verifier(0, **kw)
    out = torch.zeros(2 * nk // 32, dtype=torch.int32, device="cuda")
    v.sieve_planes(k0, nk, out)
    torch.cuda.synchronize()
    got = _unpack(out, 2 * nk).reshape(2, nk)
    w0 = 6 * k0 + 1
    ref_odd = orc.odd_primality(w0, 3 * nk)
    for i, c in enumerate((1, 5)):
        ref = ref_odd[3 * np.arange(nk) + (c - 1) // 2]
        bad = np.nonzero(got[i] != ref)[0]
        assert bad.size == 0, [(int(6 * (k0 + k) + c), int(got[i][k]), int(ref[k])) for k in bad[:10]]
    v.close()


# --------------------------------------------------------------------------
# ranges
# --------------------------------------------------------------------------

def test_config1_range_uint32(V, orc):
    # all even n in [4, 10^6], uint32 per-n output
    ref, rh, rs = orc.verify_range(4, 10**6, per_n_bits=32)
    out = _dev_pmin(len(ref), 32)
    got = V.verify_range(4, 10**6, pmin=out)
    assert np.array_equal(_host(out), ref)
    assert np.array_equal(got["hist"], rh)
    _same_summary(got, rs)


@pytest.mark.parametrize("lo,hi", [
    (10**12 - (1 << 22), 10**12),
    (5, 100_001),                       # odd ends
    (4, 4), (6, 6), (8, 8), (4, 130),
    ((1 << 50) - (1 << 20), 1 << 50),   # top of the default table
    (10**15, 10**15 + 2 * 70_001),      # ragged tail
])
def test_range_uint16_vs_oracle(V, orc, lo, hi):
    ref, rh, rs = orc.verify_range(lo, hi, per_n_bits=16, threads=4)
    out = _dev_pmin(len(ref), 16)
    got = V.verify_range(lo, hi, pmin=out)
    assert np.array_equal(_host(out), ref)
    assert np.array_equal(got["hist"], rh)
    _same_summary(got, rs)


@pytest.mark.parametrize("lo,hi", [
    ((1 << 53) - (1 << 21), (1 << 53) + (1 << 20)),   # first strikes on both sides of 2^53
    (1_000_003**2 - 200_000, 1_000_003**2 + 200_000),   # window starts on both sides of the top prime's square
    (94_906_249**2 - 200_000, 94_906_249**2 + 200_000),  # the same below 2^53 with the largest such prime
])
def test_range_near_2p53_vs_oracle(orc, lo, hi):
    _gpu()
    from paper_2603_02621_amd import Verifier
    v = Verifier(0, max_hi=1 << 54)
    ref, rh, rs = orc.verify_range(lo, hi, per_n_bits=16, threads=4)
    out = _dev_pmin(len(ref), 16)
    got = v.verify_range(lo, hi, pmin=out)
    assert np.array_equal(_host(out), ref)
    assert np.array_equal(got["hist"], rh)
    _same_summary(got, rs)
    v.close()


@pytest.mark.parametrize("tile_log2,pmax", [(20, 4096), (16, 4096), (20, 16384), (12, 1024)])
def test_tile_geometry(tile_log2, pmax):
    # the class tile: a multiple of 192 n between the n of an odd-number
    # tile of 2^tile_log2 bits and twice that, within the LDS; its lists hold
    # the odd primes up to P_max unless the LDS is short at the smallest tile
    v = _make(tile_log2=tile_log2, pmax=pmax)
    try:
        g = v.geometry
        t = 1 << tile_log2
        assert g["cls_tile_n"] % 192 == 0
        assert 192 * max(1, t // 192) <= g["cls_tile_n"] <= 192 * (t // 96)
        assert g["cls_lds_bytes"] <= 160 * 1024
        assert g["bulk_tile_n"] == g["cls_tile_n"]
        n_odd = sum(1 for q in range(3, pmax + 1, 2) if all(q % d for d in range(3, int(q**0.5) + 1, 2)))
        if g["cls_tile_n"] > 192 * max(1, t // 192):
            assert g["cls_list_primes"] == n_odd
        else:
            assert 0 < g["cls_list_primes"] <= n_odd
    finally:
        v.close()


def test_empty_range(V):
    got = V.verify_range(10, 8)
    assert got["count"] == 0 and got["status"] == 0
    got = V.verify_range(0, 3)
    assert got["count"] == 0


def test_host_output_buffer(V, orc):
    ref, _, _ = orc.verify_range(10**9, 10**9 + 50_000, per_n_bits=32)
    host = np.zeros(len(ref), dtype=np.uint32)
    V.verify_range(10**9, 10**9 + 50_000, pmin=host)
    assert np.array_equal(host, ref)


# --------------------------------------------------------------------------
# exhaustive phase
# --------------------------------------------------------------------------

@pytest.mark.parametrize("tile_log2", [19, 12])
@pytest.mark.parametrize("pmax,lo,hi", [
    (7, 4, 1 << 17),                    # almost every n goes to Miller-Rabin
    (2, 4, 1 << 14),                    # no odd prime in the fast path: every n except 4
    (1024, 10**12 - (1 << 22), 10**12), # a realistic trickle near 10^12
    (3, 10**15, 10**15 + 20_000),
])
def test_exhaustive_phase_vs_oracle(orc, pmax, lo, hi, tile_log2):
    _gpu()
    v = _make(pmax=pmax, tile_log2=tile_log2)
    ref, rh, rs = orc.verify_range(lo, hi, pmax=pmax, per_n_bits=16, threads=4)
    out = _dev_pmin(len(ref), 16)
    got = v.verify_range(lo, hi, pmin=out)
    assert np.array_equal(_host(out), ref)
    assert np.array_equal(got["hist"], rh)
    _same_summary(got, rs)
    n, p = v.exhaustive_list()
    assert len(n) == rs["n_exhaustive"]
    order = np.argsort(n)
    idx = ((n[order] - max(lo, 4)) // 2).astype(np.int64)
    assert np.array_equal(p[order].astype(np.uint64), ref[idx].astype(np.uint64))
    v.close()


def test_budget_reports_unresolved(orc):
    _gpu()
    v = _make(pmax=7, exhaustive_budget_p=11)
    lo, hi = 4, 20_000
    ref, _, rs = orc.verify_range(lo, hi, pmax=11, per_n_bits=32)
    want_failed = int(np.count_nonzero(ref > 11))
    first = 4 + 2 * int(np.nonzero(ref > 11)[0][0])
    got = v.verify_range(lo, hi, allow_unresolved=True)
    assert got["status"] == 5
    assert got["n_failed"] == want_failed
    assert got["first_failed_n"] == first
    v.close()


# --------------------------------------------------------------------------
# single n
# --------------------------------------------------------------------------

def test_verify_one_pins(V, orc):
    for n in (4, 6, 8, 98, 10**6, 10**12, 10**15, 2**62, 2**63, 2**63 - 2, 10**12 - 2**36):
        assert V.verify_one(n) == orc.verify_one(n), n


def test_verify_many_random(V, orc):
    rng = np.random.default_rng(11)
    ns = (2 * rng.integers(2, 2**62, size=4000, endpoint=True)).astype(np.uint64)
    ref = orc.verify_many(ns, threads=8)
    got = V.verify_many(ns)
    assert np.array_equal(got, ref)
    t = torch.from_numpy(ns.view(np.int64)).cuda()
    got_d = V.verify_many(t).cpu().numpy().view(np.uint64)
    assert np.array_equal(got_d, ref)


def test_verify_one_rejects_bad_n(V):
    from paper_2603_02621_amd import GoldbachError
    for n in (3, 2, 7, 2**63 + 2):
        with pytest.raises(GoldbachError):
            V.verify_one(n)


# --------------------------------------------------------------------------
# forms and parameters give identical results
# --------------------------------------------------------------------------

def test_plain_equals_batched_and_seg_hist(orc):
    _gpu()
    v = _make(seg_log2=20, tile_log2=16)
    lo, hi = 10**12 - (1 << 23), 10**12
    cnt = orc.n_even(lo, hi)
    rows = (cnt + (1 << 20) - 1) >> 20
    a = _dev_pmin(cnt)
    b = _dev_pmin(cnt)
    g1 = v.verify_range(lo, hi, pmin=a, seg_hist_rows=rows)
    g2 = v.verify_range(lo, hi, pmin=b, batched=True)
    g3 = v.verify_range(lo, hi, pmin=b, batched=True)   # graph replay
    assert torch.equal(a, b)
    for g in (g1, g2, g3):
        assert 0 < g["tile_ms"] <= g["device_ms"]
    assert g1["tile_launches"] == rows and g2["tile_launches"] == 1
    for g in (g2, g3):
        _same_summary(g, g1)
        assert np.array_equal(g["hist"], g1["hist"])
    assert np.array_equal(g1["seg_hist"].sum(axis=0), g1["hist"])
    # each segment's histogram is the oracle's over that segment
    for s in (0, rows - 1):
        slo = lo + 2 * (1 << 20) * s
        shi = min(hi, slo + 2 * ((1 << 20) - 1))
        _, rh, _ = orc.verify_range(slo, shi, per_n_bits=None)
        assert np.array_equal(g1["seg_hist"][s], rh)
    ref, _, rs = orc.verify_range(lo, hi, per_n_bits=16, threads=8)
    assert np.array_equal(_host(a), ref)
    _same_summary(g1, rs)
    v.close()


@pytest.mark.parametrize("kw", [
    dict(tile_log2=12, wg_threads=256, wheel_max=7),
    dict(tile_log2=16, wg_threads=1024, wheel_max=13, pmax=1024),
    dict(tile_log2=20, wg_threads=512, wheel_max=19),
    dict(tile_log2=19, wg_threads=512, wheel_max=19, pmax=65535),
    dict(tile_log2=17, wg_threads=512, wheel_max=11, pmax=3000),
    dict(tile_log2=14, wg_threads=512, wheel_max=17, seg_log2=16),
    dict(tile_log2=18, wg_threads=512),
    dict(tile_log2=16, wg_threads=256, pmax=1024, wheel_max=7),
])
def test_parameter_invariance(orc, kw):
    _gpu()
    lo, hi = 10**12 - (1 << 21) - 14, 10**12 + 6
    ref, rh, rs = orc.verify_range(lo, hi, per_n_bits=16, threads=8, pmax=kw.get("pmax", 8192))
    v = _make(**kw)
    out = _dev_pmin(len(ref))
    got = v.verify_range(lo, hi, pmin=out)
    assert np.array_equal(_host(out), ref)
    assert np.array_equal(got["hist"], rh)
    _same_summary(got, rs)
    out2 = _dev_pmin(len(ref))
    got2 = v.verify_range(lo, hi, pmin=out2, batched=True)
    assert torch.equal(out, out2)
    _same_summary(got2, rs)
    v.close()


def test_repeat_runs_bit_identical(V):
    lo, hi = 10**13, 10**13 + (1 << 23)
    a = _dev_pmin((hi - lo) // 2 + 1)
    b = _dev_pmin((hi - lo) // 2 + 1)
    g1 = V.verify_range(lo, hi, pmin=a, batched=True)
    g2 = V.verify_range(lo, hi, pmin=b, batched=True)
    assert torch.equal(a, b)
    _same_summary(g1, g2)


# --------------------------------------------------------------------------
# batched windows
# --------------------------------------------------------------------------

def test_windows_vs_oracle(V, orc):
    rng = np.random.default_rng(5)
    k = 96
    starts = 2 * rng.integers(2, 5 * 10**11, size=k, endpoint=True)
    lens = np.floor(2.0 ** (rng.random(k) * 16)).astype(np.int64) + 1
    starts[0], lens[0] = 4, 3000          # the start of the number line
    wins = list(zip(starts.tolist(), lens.tolist()))
    total = int(lens.sum())
    out = _dev_pmin(total)
    got = V.verify_windows(wins, pmin=out)
    host = _host(out)
    off = 0
    hsum = np.zeros(6543, dtype=np.uint64)
    for (s, ln), summ in zip(wins, got["sums"]):
        ref, rh, rs = orc.verify_range(s, s + 2 * (ln - 1), per_n_bits=16)
        assert np.array_equal(host[off:off + ln], ref), (s, ln)
        _same_summary(summ, rs)
        hsum += rh
        off += ln
    assert np.array_equal(got["hist"], hsum)


@pytest.mark.parametrize("tile_log2", [19, 12])
def test_window_alignment_vs_oracle(orc, tile_log2):
    # Windows start at every residue of n/2 mod 64 (the planner moves each
    # start down to a multiple of 128 and masks the n in front), with
    # lengths around one and two 64-n blocks and across tile edges, and at
    # the start of the number line, where n = 4 sits in the masked block.
    _gpu()
    v = _make(tile_log2=tile_log2)
    wins = []
    base = 10**12 - (1 << 20)
    lens = [1, 2, 31, 32, 33, 63, 64, 65, 127, 128, 129, 4096 + 7, 9000]
    for r in range(64):
        wins.append((base + 128 * r * 3 + 2 * r, lens[r % len(lens)]))
    for s in range(4, 260, 2):
        wins.append((s, 1 + (s % 70)))
    total = sum(ln for _, ln in wins)
    out = _dev_pmin(total)
    got = v.verify_windows(wins, pmin=out)
    host = _host(out)
    off = 0
    for (s, ln), summ in zip(wins, got["sums"]):
        ref, rh, rs = orc.verify_range(s, s + 2 * (ln - 1), per_n_bits=16)
        assert np.array_equal(host[off:off + ln], ref), (s, ln)
        _same_summary(summ, rs)
        off += ln
    v.close()


def test_search_mode_other_than_1_rejected():
    _gpu()
    from paper_2603_02621_amd._binding import GoldbachError
    with pytest.raises(GoldbachError):
        _make(search_mode=2)
