"""The autotuner sweeps tile shape, P_max, wheel and segment size, checks that
every point gives the same results, and leaves the fastest in the context."""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_autotune_sweep(orc, tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_02621_amd import Verifier
    from paper_2603_02621_amd.workloads import config3_windows
    sample = config3_windows(0, 4096)[:96]
    path = tmp_path / "tuned.json"
    with Verifier(0) as v:
        best = v.autotune(sample, str(path))
        d = json.loads(path.read_text())
        assert d["tile_log2"] == best["tile_log2"] == v.params["tile_log2"]
        assert d["seg_log2"] == best["seg_log2"]
        assert len(d["trials"]) >= 20
        assert any(t["ms"] > 0 for t in d["trials"])
        # the tuned context still matches the oracle
        s, n = sample[3]
        out = torch.zeros(n, dtype=torch.int16, device="cuda")
        got = v.verify_windows([(s, n)], pmin=out)["sums"][0]
        ref, _, rs = orc.verify_range(s, s + 2 * (n - 1), per_n_bits=16, pmax=best["pmax"])
        assert np.array_equal(out.cpu().numpy().view(np.uint16), ref)
        assert got["checksum"] == rs["checksum"]
