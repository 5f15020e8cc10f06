"""The allocation-free solve (aifmm_solve_noalloc, device pointers, work buffers in the
library's fixed scratch array) against aifmm_solve on the same factorization: identical
solutions on two calls in a row, the second with a smaller input (fewer columns, and a
smaller system), and the capacity error beyond the scratch maximum."""
import ctypes

import numpy as np
import pytest

import aifmm_inputs as I

pytestmark = pytest.mark.gpu
A = pytest.importorskip("paper_2301_12704_amd")
torch = pytest.importorskip("torch")


def _noalloc(g, b_host):
    """b (N x nr, numpy) -> solution through aifmm_solve_noalloc on device buffers."""
    n, nr = b_host.shape
    b_d = torch.from_numpy(np.ascontiguousarray(b_host.T)).cuda()  # (nr, N): column-major N x nr
    x_d = torch.empty_like(b_d)
    torch.cuda.synchronize()
    st = A.lib().aifmm_solve_noalloc(g._h, ctypes.c_void_p(b_d.data_ptr()), nr, n, ctypes.c_void_p(x_d.data_ptr()), n)
    if st != 0:
        raise A.AifmmError(st, A.lib().aifmm_last_error(g._h).decode())
    return x_d.cpu().numpy().T


def test_noalloc_matches_solve_two_calls():
    c = I.small_case(8192, d=2, depth=4, tol=1e-8, kernel=("invmq", 1e-2, 1.0), nrhs=4, seed=81)
    print("case no-alloc n=8192 depth 4 nrhs 4 then 1", flush=True)
    g = A.System(c["pts"], c["kernel"], c["tol"], 64, 4)
    g.factor()
    x1 = _noalloc(g, c["b"])
    np.testing.assert_array_equal(x1, g.solve(c["b"]))
    b2 = np.asfortranarray(c["b"][:, 1:2])
    x2 = _noalloc(g, b2)
    np.testing.assert_array_equal(x2, g.solve(b2))
    # a smaller system on the same scratch, after the larger one
    c3 = I.small_case(2048, d=3, depth=2, tol=1e-6, kernel=("invmq", 0.1, 1.0), nrhs=2, seed=82)
    print("case no-alloc n=2048 3D depth 2 nrhs 2", flush=True)
    h = A.System(c3["pts"], c3["kernel"], c3["tol"], 64, 2)
    h.factor()
    np.testing.assert_array_equal(_noalloc(h, c3["b"]), h.solve(c3["b"]))
    g.close()
    h.close()


def test_noalloc_rejects_beyond_scratch_and_host_pointers():
    c = I.small_case(8192, d=2, depth=4, tol=1e-8, kernel=("invmq", 1e-2, 1.0), nrhs=1, seed=83)
    print("case no-alloc limits n=8192", flush=True)
    g = A.System(c["pts"], c["kernel"], c["tol"], 64, 4)
    g.factor()
    big = np.asfortranarray(np.random.default_rng(84).standard_normal((8192, 1200)))
    with pytest.raises(A.AifmmError) as e:
        _noalloc(g, big)
    assert e.value.status == 7 and "maximum" in str(e.value)
    x = np.zeros((8192, 1), order="F")
    st = A.lib().aifmm_solve_noalloc(g._h, c["b"].ctypes.data_as(ctypes.c_void_p), 1, 8192,
                                     x.ctypes.data_as(ctypes.c_void_p), 8192)
    assert st == 1
    g.close()
