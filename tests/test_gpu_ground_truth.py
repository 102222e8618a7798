"""The device brute force behind recall figures and k-NN graphs, checked on
the largest workload (5M x 96) against a plain fp64 scan of every base row."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def test_device_ground_truth_equals_fp64_scan_at_5m():
    X, Q = synth.gen_data(synth.DEEP_LIKE, nq=6)
    print(f"5M x 96 base, {len(Q)} queries", flush=True)
    gt, gd = synth.ground_truth(X, Q, 100, device=torch.device("cuda:0"))
    ids = np.arange(len(X))
    X64 = X.astype(np.float64)
    for i in range(len(Q)):
        d = ((X64 - Q[i].astype(np.float64)) ** 2).sum(1)
        want = np.lexsort((ids, d))[:100]
        assert np.array_equal(gt[i], want), f"query {i}"
        assert np.allclose(gd[i], d[want], rtol=0, atol=1e-12)
