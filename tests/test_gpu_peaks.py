"""Measured device ceilings (gb_measure_peaks): finite, positive, and in
the right units (GPU)."""
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

def test_measured_peaks_plausible(V):
    pk = V.measure_peaks()
    for k, val in pk.items():
        assert np.isfinite(val) and val > 0, k
    # orders of magnitude only (units): lane-ops/s and bytes/s of one device
    assert 1e12 < pk["valu_vop2_ops"] < 1e15
    assert 1e12 < pk["valu_vop3_ops"] < 1e15
    assert 1e12 < pk["lds_read_bytes"] < 1e15
    assert 1e11 < pk["lds_atomic_ops"] < 1e15
    assert 1e11 < pk["hbm_copy_bytes"] < 2e13
