"""Bulk verification (gb_verify_range_bulk) against the oracle (GPU).

The bulk form records no minimal p per n, but its count, largest p_min with
its smallest n, n_exhaustive and failures must equal the oracle's, and the n
it leaves to the exhaustive phase must be exactly those whose p_min exceeds
P_max, with their p_min.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("pmax,lo,hi,tile_log2", [
    (8192, 10**12 - (1 << 22), 10**12, 19),
    (4096, 10**12 - (1 << 22), 10**12, 20),
    (7, 4, 1 << 17, 19),                     # almost every n goes to the exhaustive phase
    (2, 4, 1 << 14, 19),                     # no odd prime in the fast path
    (1024, 10**12 - (1 << 22) - 14, 10**12 + 6, 12),
    (8192, 4, 300_000, 19),                  # the start of the number line, n = 4
    (65535, 10**15, 10**15 + 2_000_000, 19),  # per-probe window reads (no group window)
    (8192, 4, 4, 19), (8192, 6, 6, 19), (8192, 4, 130, 12), (8192, 1_000_002, 1_000_002, 16),
])
def test_bulk_vs_oracle(orc, pmax, lo, hi, tile_log2):
    _gpu()
    from paper_2603_02621_amd import Verifier
    v = Verifier(0, pmax=pmax, tile_log2=tile_log2)
    ref, _, rs = orc.verify_range(lo, hi, pmax=pmax, per_n_bits=32, threads=8)
    got = v.verify_range_bulk(lo, hi)
    for k in ("count", "max_p", "argmax_n", "n_exhaustive", "n_failed", "first_failed_n"):
        assert got[k] == rs[k], (k, got[k], rs[k])
    assert got["checksum"] == 0
    n, p = v.exhaustive_list()
    a = max(lo, 4) + (max(lo, 4) & 1)
    ns = a + 2 * np.arange(len(ref), dtype=np.uint64)
    sel = ref.astype(np.uint64) > pmax
    order = np.argsort(n)
    assert np.array_equal(n[order], ns[sel])
    assert np.array_equal(p[order], ref[sel].astype(np.uint64))
    v.close()


def test_bulk_equals_minimal_form_near_1e12():
    _gpu()
    from paper_2603_02621_amd import Verifier
    v = Verifier(0)
    lo, hi = 10**12 - (1 << 30), 10**12
    full = v.verify_range(lo, hi, batched=True)
    bulk = v.verify_range_bulk(lo, hi)
    for k in ("count", "max_p", "argmax_n", "n_exhaustive", "n_failed", "first_failed_n"):
        assert bulk[k] == full[k], k
    v.close()


def test_bulk_rejects_per_n_output():
    _gpu()
    from paper_2603_02621_amd import Verifier
    from paper_2603_02621_amd._binding import Result, GoldbachError
    import ctypes
    v = Verifier(0)
    r = Result()
    buf = torch.zeros(100, dtype=torch.int16, device="cuda")
    r.pmin, r.pmin_bits, r.pmin_on_device = buf.data_ptr(), 16, 1
    st = v._lib.gb_verify_range_bulk(v._h, 10**9, 10**9 + 198, ctypes.byref(r), None)
    assert st == 1   # GB_EINVAL
    v.close()
