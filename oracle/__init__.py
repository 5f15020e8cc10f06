"""AIFMM CPU oracle (TEST INFRASTRUCTURE ONLY).

Plain FP64 C++ reference of the Algebraic Inverse FMM (arXiv 2301.12704), loaded with
ctypes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the HIP product path never does.

Pins: ``tests/test_oracle_units.py`` (ACA, RRQR, LU against closed forms and brute force),
``tests/test_oracle_tree.py`` (tree/list closed-form counts, eta = sqrt(d) admissibility),
``tests/test_oracle_system.py`` (extended-system Schur identity, tol -> 0 reduction to
dense LU, NNCA rank/tolerance invariant, end-to-end forward error and residual).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "aifmm_oracle.cpp")

KERNELS = {"exp": 0, "invmq": 1}


def build(force=True):
    """Compile the oracle with g++ (plain -O2, no fused multiply-add contraction)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    tmp = _SO + ".tmp"
    cmd = ["g++", "-O2", "-mfma", "-ffp-contract=off", "-fPIC", "-shared", "-std=c++17", "-o", tmp, _SRC]
    subprocess.check_call(cmd, cwd=_HERE)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        d, i64, i32, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.oracle_kernel_block.argtypes = [vp, i32, i32, d, d, vp, i64, vp, i64, vp]
        L.oracle_matvec.argtypes = [vp, i64, i32, i32, d, d, vp, i64, vp]
        L.oracle_matvec_rows.argtypes = [vp, i64, i32, i32, d, d, vp, i64, vp, i64, vp]
        L.oracle_dense_solve.argtypes = [i64, vp, i64, vp, vp]
        L.oracle_dense_solve.restype = i32
        L.oracle_aca.argtypes = [vp, i32, i32, d, vp, vp, vp, vp]
        L.oracle_aca.restype = i32
        L.oracle_cpqr.argtypes = [vp, i32, i32, d, i32, vp, vp, vp]
        L.oracle_cpqr.restype = i32
        L.oracle_create.argtypes = [vp, i64, i32, i32, d, d, d, i32, i32]
        L.oracle_create.restype = vp
        L.oracle_create_mode.argtypes = [vp, i64, i32, i32, d, d, d, i32, i32, i32]
        L.oracle_create_mode.restype = vp
        L.oracle_rhs_violations.argtypes = [vp]
        L.oracle_rhs_violations.restype = i64
        L.oracle_row_set.argtypes = [vp, i32, i32, vp]
        L.oracle_row_set.restype = i32
        L.oracle_kexp.argtypes = [vp, i64, vp]
        L.oracle_h2_matvec.argtypes = [vp, vp, i64, vp]
        L.oracle_h2_matvec.restype = i32
        L.oracle_error.argtypes = [vp]
        L.oracle_error.restype = ctypes.c_char_p
        for name in ["oracle_depth"]:
            getattr(L, name).argtypes = [vp]
            getattr(L, name).restype = i32
        for name in ["oracle_box_count", "oracle_nnca_ranks", "oracle_final_ranks",
                     "oracle_xsize", "oracle_elim_order"]:
            getattr(L, name).argtypes = [vp, i32, vp]
            getattr(L, name).restype = i32
        L.oracle_pivots.argtypes = [vp, i32, i32, vp, vp]
        L.oracle_pivots.restype = i32
        L.oracle_perm.argtypes = [vp, vp]
        L.oracle_nnca_U.argtypes = [vp, i32, i32, vp]
        L.oracle_nnca_U.restype = i32
        L.oracle_dense_extended.argtypes = [vp, P(i64), vp, vp]
        L.oracle_dense_extended.restype = i32
        L.oracle_factor.argtypes = [vp]
        L.oracle_factor.restype = i32
        L.oracle_solve.argtypes = [vp, vp, i64, vp]
        L.oracle_solve.restype = i32
        L.oracle_trace.argtypes = [vp, vp, i64]
        L.oracle_trace.restype = i64
        L.oracle_trace_ranks.argtypes = [vp, vp, vp, i64]
        L.oracle_trace_ranks.restype = i64
        L.oracle_lists.argtypes = [vp, i32, i32, vp, vp]
        L.oracle_lists.restype = i32
        L.oracle_far_fill_count.argtypes = [vp]
        L.oracle_far_fill_count.restype = i64
        L.oracle_margins.argtypes = [vp, P(d), P(d), P(d)]
        L.oracle_flops.argtypes = [vp, vp]
        L.oracle_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def kernel_block(pts, kernel, rows, cols):
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros((len(rows), len(cols)))
    lib().oracle_kernel_block(_p(pts), pts.shape[1], KERNELS[kernel[0]], kernel[1], kernel[2],
                              _p(rows), len(rows), _p(cols), len(cols), _p(out))
    return out


def dense_matrix(pts, kernel):
    n = pts.shape[0]
    idx = np.arange(n, dtype=np.int64)
    return kernel_block(pts, kernel, idx, idx)


def matvec(pts, kernel, x):
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    x2 = np.asfortranarray(x.reshape(pts.shape[0], -1), dtype=np.float64)
    y = np.zeros_like(x2, order="F")
    lib().oracle_matvec(_p(pts), pts.shape[0], pts.shape[1], KERNELS[kernel[0]], kernel[1], kernel[2],
                        _p(x2), x2.shape[1], _p(y))
    return y.reshape(x.shape)


def matvec_rows(pts, kernel, rows, x):
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    x2 = np.asfortranarray(x.reshape(pts.shape[0], -1), dtype=np.float64)
    y = np.zeros((len(rows), x2.shape[1]), order="F")
    lib().oracle_matvec_rows(_p(pts), pts.shape[0], pts.shape[1], KERNELS[kernel[0]], kernel[1],
                             kernel[2], _p(rows), len(rows), _p(x2), x2.shape[1], _p(y))
    return y


def dense_solve(A, B):
    A = np.ascontiguousarray(A, dtype=np.float64)
    B2 = np.asfortranarray(B.reshape(A.shape[0], -1), dtype=np.float64)
    X = np.zeros_like(B2, order="F")
    st = lib().oracle_dense_solve(A.shape[0], _p(A), B2.shape[1], _p(B2), _p(X))
    if st:
        raise np.linalg.LinAlgError(f"zero pivot at step {st - 1}")
    return X.reshape(B.shape)


def aca(M, tol):
    M = np.ascontiguousarray(M, dtype=np.float64)
    m, n = M.shape
    k = min(m, n)
    I = np.zeros(k, np.int32)
    J = np.zeros(k, np.int32)
    U = np.zeros((k, m))
    V = np.zeros((k, n))
    r = lib().oracle_aca(_p(M), m, n, tol, _p(I), _p(J), _p(U), _p(V))
    return I[:r], J[:r], U[:r].T.copy(), V[:r].copy()


def kexp(x):
    """The exponential kernel's e^x routine, elementwise."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    lib().oracle_kexp(_p(x), x.size, _p(out))
    return out


# readings where the paper fixes no order or routine (oracle.h, ORACLE_MODE_*)
MODE_STD_EXP, MODE_ASC_SUMS, MODE_ASC_BACK, MODE_SEQUENTIAL = 1, 2, 4, 8
MODE_TEXTBOOK = 15


def cpqr(M, tol, qcols=None):
    M = np.ascontiguousarray(M, dtype=np.float64)
    m, n = M.shape
    qcols = m if qcols is None else qcols
    Q = np.zeros((m, qcols))
    perm = np.zeros(n, np.int32)
    R = np.zeros((min(m, n), n))
    k = lib().oracle_cpqr(_p(M), m, n, tol, qcols, _p(Q), _p(perm), _p(R))
    return k, Q, perm, R[:k]


class System:
    """Oracle AIFMM system: build (tree, lists, NNCA, extended system) in the constructor."""

    def __init__(self, pts, kernel, tol, leaf_size=64, depth=0, mode=0):
        self.pts = np.ascontiguousarray(pts, dtype=np.float64)
        self.N, self.d = self.pts.shape
        self.kernel = kernel
        L = lib()
        self.h = L.oracle_create_mode(_p(self.pts), self.N, self.d, KERNELS[kernel[0]], kernel[1],
                                      kernel[2], tol, leaf_size, depth, int(mode))
        err = L.oracle_error(self.h).decode()
        if err:
            raise RuntimeError(err)
        self.L = L.oracle_depth(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().oracle_destroy(self.h)
            self.h = None

    def _levelarr(self, fn, level):
        nb = 1 << (self.d * level)
        out = np.zeros(nb, np.int32)
        r = fn(self.h, level, _p(out))
        if r < 0:
            raise RuntimeError("level query failed")
        return out

    def counts(self, level):
        return self._levelarr(lib().oracle_box_count, level)

    def nnca_ranks(self, level):
        return self._levelarr(lib().oracle_nnca_ranks, level)

    def final_ranks(self, level):
        return self._levelarr(lib().oracle_final_ranks, level)

    def xsizes(self, level):
        return self._levelarr(lib().oracle_xsize, level)

    def elim_order(self, level):
        return self._levelarr(lib().oracle_elim_order, level)

    def pivots(self, level, box):
        t = np.zeros(4096, np.int64)
        s = np.zeros(4096, np.int64)
        k = lib().oracle_pivots(self.h, level, box, _p(t), _p(s))
        return t[:k].copy(), s[:k].copy()

    def nnca_U(self, level, box):
        k = int(self.nnca_ranks(level)[box])
        out = np.zeros(4096 * max(k, 1))
        m = lib().oracle_nnca_U(self.h, level, box, _p(out))
        return out[: m * k].reshape(m, k)

    def perm(self):
        p = np.zeros(self.N, np.int64)
        lib().oracle_perm(self.h, _p(p))
        return p

    def dense_extended(self):
        dim = ctypes.c_int64(0)
        lib().oracle_dense_extended(self.h, ctypes.byref(dim), None, None)
        M = np.zeros((dim.value, dim.value))
        xc = np.zeros(self.N, np.int64)
        st = lib().oracle_dense_extended(self.h, ctypes.byref(dim), _p(M), _p(xc))
        if st:
            raise RuntimeError("dense_extended failed")
        return M, xc

    def h2_matvec(self, x):
        """NNCA-based H^2 product with the system's operators (oracle_h2_matvec)."""
        x2 = np.asfortranarray(x.reshape(self.N, -1), dtype=np.float64)
        y = np.zeros_like(x2, order="F")
        st = lib().oracle_h2_matvec(self.h, _p(x2), x2.shape[1], _p(y))
        if st:
            raise RuntimeError(f"h2 matvec status {st}")
        return y.reshape(x.shape)

    def factor(self):
        st = lib().oracle_factor(self.h)
        if st:
            raise RuntimeError(lib().oracle_error(self.h).decode() or f"factor status {st}")

    def solve(self, b):
        b2 = np.asfortranarray(b.reshape(self.N, -1), dtype=np.float64)
        x = np.zeros_like(b2, order="F")
        st = lib().oracle_solve(self.h, _p(b2), b2.shape[1], _p(x))
        if st:
            raise RuntimeError(f"solve status {st}")
        return x.reshape(b.shape)

    def trace(self):
        n = lib().oracle_trace(self.h, None, 0)
        out = np.zeros((max(n, 1), 4), np.int32)
        lib().oracle_trace(self.h, _p(out), n)
        return out[:n]

    def trace_ranks(self):
        n = lib().oracle_trace(self.h, None, 0)
        rk = np.zeros((max(n, 1), 6), np.int32)
        ra = np.zeros((max(n, 1), 8))
        lib().oracle_trace_ranks(self.h, _p(rk), _p(ra), n)
        return rk[:n], ra[:n]

    def lists(self, level, box):
        nb = np.zeros(64, np.int32)
        il = np.zeros(256, np.int32)
        r = lib().oracle_lists(self.h, level, box, _p(nb), _p(il))
        return nb[:r // 1000].copy(), il[:r % 1000].copy()

    def far_fill(self):
        return lib().oracle_far_fill_count(self.h)

    def rhs_violations(self):
        return lib().oracle_rhs_violations(self.h)

    def row_set(self, level, box):
        n = lib().oracle_row_set(self.h, level, box, None)
        out = np.zeros(max(n, 1), np.int64)
        lib().oracle_row_set(self.h, level, box, _p(out))
        return out[:n]

    def margins(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        lib().oracle_margins(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return a.value, b.value, c.value

    def flops(self):
        f = np.zeros(5)
        lib().oracle_flops(self.h, _p(f))
        return f
