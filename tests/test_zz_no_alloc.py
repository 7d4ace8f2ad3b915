"""gb_verify_many_noalloc (no device allocation in the call; scratch in a
fixed device array of the library) against gb_verify_many, through the C
ABI: two calls in a row, the second with fewer n, then the size limit and an
invalid n (GPU)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_02621_amd import Verifier
    v = Verifier(0)
    yield v
    v.close()


def _call(V, dn, dp):
    torch.cuda.synchronize()
    st = V._lib.gb_verify_many_noalloc(V._h, dn.data_ptr(), dp.data_ptr(), dn.numel(), ctypes.c_void_p(0))
    torch.cuda.synchronize()
    return st


def test_noalloc_equals_verify_many_twice(V):
    rng = np.random.default_rng(17)
    for k in (40000, 3000):                   # the second call is smaller
        ns = 2 * rng.integers(2, 2**62, size=k, dtype=np.uint64)
        ns[:4] = [4, 6, 98, 2**62]
        want = V.verify_many(ns)              # the existing entry point, host arrays
        dn = torch.from_numpy(ns.view(np.int64)).cuda()
        dp = torch.full_like(dn, -1)
        assert _call(V, dn, dp) == 0, V.last_error
        got = dp.cpu().numpy().view(np.uint64)
        assert np.array_equal(got, want)


def test_noalloc_limits(V):
    from paper_2603_02621_amd import GoldbachError
    big = torch.full((65537,), 10**12, dtype=torch.int64, device="cuda")
    assert _call(V, big, torch.empty_like(big)) == 1          # GB_EINVAL: above the limit
    bad = torch.tensor([10**12, 10**12 + 1, 8], dtype=torch.int64, device="cuda")
    assert _call(V, bad, torch.empty_like(bad)) == 1          # GB_EINVAL: an odd n
    ok = torch.tensor([10**12, 8], dtype=torch.int64, device="cuda")
    assert V.verify_many_noalloc(ok).cpu().tolist() == [11, 3]
    with pytest.raises(GoldbachError):
        V.verify_many_noalloc(bad)
