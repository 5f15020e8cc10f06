"""Host arrays with a leading dimension above N through the C ABI: solve, matvec and GMRES
read only the N rows of each column of b / x and write only the N rows of each column of the
result, so the caller's padding rows and the memory after the last column keep their values."""
import ctypes

import numpy as np
import pytest

import aifmm_inputs as I

pytestmark = pytest.mark.gpu
A = pytest.importorskip("paper_2301_12704_amd")

SENT = -7.25e300  # sentinel in the padding rows and after the last column


def _padded(mat, ld, extra):
    """Column-major N x nr array with leading dimension ld inside a flat buffer with `extra`
    doubles after the last column; padding rows and the tail hold the sentinel."""
    n, nr = mat.shape
    buf = np.full(ld * nr + extra, SENT)
    for c in range(nr):
        buf[c * ld: c * ld + n] = mat[:, c]
    return buf


def _cols(buf, n, ld, nr):
    return np.stack([buf[c * ld: c * ld + n] for c in range(nr)], axis=1)


def _pad_ok(buf, n, ld, nr):
    for c in range(nr):
        assert np.all(buf[c * ld + n: (c + 1) * ld] == SENT), f"padding of column {c} changed"
    assert np.all(buf[ld * nr:] == SENT), "memory after the last column changed"


def test_leading_dimension_above_n():
    c = I.small_case(2048, d=2, depth=3, tol=1e-8, kernel=("exp", 1.0, 0.1), nrhs=3, seed=71)
    print("case ld test n=2048 d=2 depth 3 nrhs 3", flush=True)
    g = A.System(c["pts"], c["kernel"], c["tol"], 64, 3)
    g.factor()
    L = A.lib()
    n, nr, ld, extra = 2048, 3, 2048 + 7, 11
    vp = ctypes.c_void_p
    b = _padded(c["b"], ld, extra)
    x = _padded(np.zeros((n, nr)), ld, extra)
    ref = g.solve(c["b"])
    assert L.aifmm_solve(g._h, b.ctypes.data_as(vp), nr, ld, x.ctypes.data_as(vp), ld) == 0
    np.testing.assert_array_equal(_cols(x, n, ld, nr), ref)
    _pad_ok(x, n, ld, nr)
    _pad_ok(b, n, ld, nr)
    y = _padded(np.zeros((n, nr)), ld, extra)
    assert L.aifmm_matvec(g._h, x.ctypes.data_as(vp), nr, ld, y.ctypes.data_as(vp), ld) == 0
    np.testing.assert_array_equal(_cols(y, n, ld, nr), g.matvec(ref))
    _pad_ok(y, n, ld, nr)
    xg = _padded(np.zeros((n, nr)), ld, extra)
    it = np.zeros(nr, np.int32)
    rr = np.zeros(nr)
    st = L.aifmm_gmres(None, g._h, b.ctypes.data_as(vp), nr, ld, 1e-10, 30, 100, xg.ctypes.data_as(vp), ld,
                       it.ctypes.data_as(vp), rr.ctypes.data_as(vp))
    assert st == 0
    xr, _, _ = g.gmres(c["b"], rtol=1e-10)
    np.testing.assert_array_equal(_cols(xg, n, ld, nr), xr)
    _pad_ok(xg, n, ld, nr)
    g.close()
