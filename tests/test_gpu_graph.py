"""The direct solve on a system with its own stream is captured once into a HIP graph and
replayed.  Every replay, with other device work and host synchronizations in between, must
give exactly the eager solve (same kernels, same order): bit-identical solutions, also after
the column count changes (recapture) and after a new factorization."""
import os

import numpy as np
import pytest

import aifmm_inputs as I

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2301_12704_amd")
torch = pytest.importorskip("torch")


def _eager(s, b):
    os.environ["AIFMM_NO_GRAPH"] = "1"
    try:
        return s.solve(b)
    finally:
        del os.environ["AIFMM_NO_GRAPH"]


def test_graph_replays_equal_eager():
    c = I.small_case(8192, d=2, depth=4, tol=1e-8, kernel=("invmq", 1e-2, 1.0), nrhs=3, seed=61)
    stream = torch.cuda.Stream()
    s = A.System(c["pts"], c["kernel"], c["tol"], 64, 4, stream=stream.cuda_stream)
    s.factor()
    b = c["b"]
    ref = _eager(s, b)
    for rep in range(4):
        x = s.solve(b)
        np.testing.assert_array_equal(x, ref, err_msg=f"replay {rep}")
        # other device work and synchronizations between replays
        s.matvec(x)
        torch.ones(1 << 20, device="cuda").sum().item()
        torch.cuda.synchronize()
    b1 = np.asfortranarray(b[:, :1])
    ref1 = _eager(s, b1)
    for rep in range(3):
        np.testing.assert_array_equal(s.solve(b1), ref1, err_msg=f"one column, replay {rep}")
    np.testing.assert_array_equal(s.solve(b), ref)
    s.close()
