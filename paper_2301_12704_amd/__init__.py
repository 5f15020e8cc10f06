"""Python binding of the MI355X AIFMM library (libaifmm.so, C ABI in include/aifmm.h).

Argument marshalling only: every numerical step runs in the library's HIP kernels.  The
binding fails loudly when the compiled library is missing; there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libaifmm.so")
KERNELS = {"exp": 0, "invmq": 1}

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_NOMEM", 3: "ERR_SINGULAR", 4: "ERR_STATE", 5: "ERR_DEVICE",
          6: "ERR_NOCONV", 7: "ERR_CAPACITY", 8: "ERR_BUSY"}
STAT_NAMES = ["build_s", "factor_s", "solve_s", "schur_flops", "schur_bytes", "trsm_flops", "lu_flops",
              "device_bytes", "schur_kernel_s", "schur_launches", "compress_kernel_s", "compress_launches", "gmres_s",
              "trsm_kernel_s", "trsm_launches", "solve_bytes"]
LSTAT_NAMES = ["factor_s", "schur_flops", "schur_bytes", "trsm_flops", "trsm_flops_impl", "lu_flops", "schur_kernel_s",
               "trsm_kernel_s", "compress_kernel_s", "compress_flops", "compressions", "rounds", "crit_steps",
               "pivot_steps", "boxes"]


class AifmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("scale", ctypes.c_double), ("shift", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("leaf_size", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("device", ctypes.c_int32), ("stream", ctypes.c_void_p), ("prec", ctypes.c_int32),
                ("matvec_tol", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
        # One HIP runtime per process: when PyTorch is present its runtime is loaded first, and
        # the library's libamdhip64.so.7 dependency then resolves to that same object.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIBPATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.aifmm_options_default.argtypes = [ctypes.POINTER(_Options)]
        L.aifmm_build.argtypes = [vp, i64, _Kernel, d, ctypes.POINTER(_Options), ctypes.POINTER(vp)]
        L.aifmm_factor.argtypes = [vp]
        L.aifmm_solve.argtypes = [vp, vp, i64, i64, vp, i64]
        L.aifmm_get_depth.argtypes = [vp, ctypes.POINTER(i32)]
        L.aifmm_get_ranks.argtypes = [vp, i32, vp]
        L.aifmm_get_stats.argtypes = [vp, vp]
        L.aifmm_get_level_stats.argtypes = [vp, i32, vp]
        L.aifmm_get_level_stats.restype = ctypes.c_int
        L.aifmm_get_trace.argtypes = [vp, vp, vp, i64, ctypes.POINTER(i64)]
        L.aifmm_get_trace.restype = ctypes.c_int
        L.aifmm_solve_noalloc.argtypes = [vp, vp, i64, i64, vp, i64]
        L.aifmm_solve_noalloc.restype = ctypes.c_int
        L.aifmm_matvec.argtypes = [vp, vp, i64, i64, vp, i64]
        L.aifmm_matvec.restype = ctypes.c_int
        L.aifmm_matvec_h2.argtypes = [vp, vp, i64, i64, vp, i64]
        L.aifmm_matvec_h2.restype = ctypes.c_int
        L.aifmm_gmres.argtypes = [vp, vp, vp, i64, i64, d, i32, i32, vp, i64, vp, vp]
        L.aifmm_gmres.restype = ctypes.c_int
        L.aifmm_get_nnca.argtypes = [vp, i32, i32, vp, vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.aifmm_get_nnca.restype = ctypes.c_int
        L.aifmm_last_error.argtypes = [vp]
        L.aifmm_last_error.restype = ctypes.c_char_p
        L.aifmm_destroy.argtypes = [vp]
        L.aifmm_server_create.argtypes = [vp, i32, ctypes.c_size_t, d, i32, ctypes.POINTER(vp)]
        L.aifmm_server_create.restype = ctypes.c_int
        L.aifmm_server_submit.argtypes = [vp, i32, vp, i64, i64, ctypes.POINTER(i64)]
        L.aifmm_server_submit.restype = ctypes.c_int
        L.aifmm_server_wait.argtypes = [vp, i64, vp, i64, ctypes.POINTER(d), ctypes.POINTER(i32), vp, vp]
        L.aifmm_server_wait.restype = ctypes.c_int
        L.aifmm_server_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_size_t)]
        L.aifmm_server_stats.restype = ctypes.c_int
        L.aifmm_server_destroy.argtypes = [vp]
        L.aifmm_factor_batch.argtypes = [vp, i32, i32]
        L.aifmm_factor_batch.restype = ctypes.c_int
        for f in ["aifmm_options_default", "aifmm_build", "aifmm_factor", "aifmm_solve", "aifmm_get_depth",
                  "aifmm_get_ranks", "aifmm_get_stats"]:
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st, h=None):
    if st != 0:
        msg = lib().aifmm_last_error(h).decode() if h is not None else lib().aifmm_last_error(None).decode()
        raise AifmmError(st, msg)


def _ptr(a):
    """Data pointer of a numpy array or a torch tensor (host or device)."""
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


class System:
    """One N-body system A x = b, A_ij = kappa(|p_i - p_j|) + shift delta_ij (aifmm_build)."""

    def __init__(self, points, kernel, tol, leaf_size=64, depth=0, device=0, stream=None, precision="fp64",
                 matvec_tol=0.0):
        self._h = None
        if hasattr(points, "data_ptr"):
            pts = points.contiguous()
            n, d = pts.shape
        else:
            pts = np.ascontiguousarray(points, dtype=np.float64)
            n, d = pts.shape
        self._pts = pts
        self.N, self.d = int(n), int(d)
        opt = _Options()
        _check(lib().aifmm_options_default(ctypes.byref(opt)))
        opt.dim, opt.leaf_size, opt.depth, opt.device = d, leaf_size, depth, device
        opt.stream = stream
        opt.prec = {"fp64": 0, "fp32": 1}[precision]
        opt.matvec_tol = float(matvec_tol)
        self.matvec_tol = float(matvec_tol)
        k = _Kernel(KERNELS[kernel[0]], float(kernel[1]), float(kernel[2]))
        h = ctypes.c_void_p()
        _check(lib().aifmm_build(_ptr(pts), n, k, float(tol), ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        L = ctypes.c_int32()
        _check(lib().aifmm_get_depth(self._h, ctypes.byref(L)), self._h)
        self.L = L.value

    def close(self):
        if self._h is not None:
            lib().aifmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def factor(self):
        _check(lib().aifmm_factor(self._h), self._h)

    def solve(self, b, out=None):
        """b: N x nrhs (numpy, Fortran order, or a device torch tensor of shape (nrhs, N))."""
        if hasattr(b, "data_ptr"):
            bt = b.contiguous()
            nrhs = bt.shape[0] if bt.dim() == 2 else 1
            x = out if out is not None else bt.new_empty(bt.shape)
            _check(lib().aifmm_solve(self._h, _ptr(bt), nrhs, self.N, _ptr(x), self.N), self._h)
            return x
        b2 = np.asfortranarray(np.asarray(b, dtype=np.float64).reshape(self.N, -1))
        x = np.zeros_like(b2, order="F")
        _check(lib().aifmm_solve(self._h, _ptr(b2), b2.shape[1], self.N, _ptr(x), self.N), self._h)
        return x.reshape(np.shape(b))

    def matvec(self, x):
        """y = A x (exact FP64, every kernel entry evaluated on the device)."""
        x2 = np.asfortranarray(np.asarray(x, dtype=np.float64).reshape(self.N, -1))
        y = np.zeros_like(x2, order="F")
        _check(lib().aifmm_matvec(self._h, _ptr(x2), x2.shape[1], self.N, _ptr(y), self.N), self._h)
        return y.reshape(np.shape(x))

    def matvec_h2(self, x):
        """y = A~ x, the NNCA-based H^2 product at the system's matvec tolerance."""
        x2 = np.asfortranarray(np.asarray(x, dtype=np.float64).reshape(self.N, -1))
        y = np.zeros_like(x2, order="F")
        _check(lib().aifmm_matvec_h2(self._h, _ptr(x2), x2.shape[1], self.N, _ptr(y), self.N), self._h)
        return y.reshape(np.shape(x))

    def gmres(self, b, rtol=1e-10, restart=30, maxit=200, raise_on_noconv=True, op="auto"):
        """FGMRES to ||Ax-b||/||b|| <= rtol, preconditioned by the factorization.  op: the
        System whose H^2 product is the operator; "auto" = this system's own when it was built
        with a matvec tolerance, else the exact product; None = the exact product.
        Returns (x, iters, relres)."""
        if isinstance(op, str):
            op = self if self.matvec_tol > 0 else None
        oph = op._h if op is not None else None
        b2 = np.asfortranarray(np.asarray(b, dtype=np.float64).reshape(self.N, -1))
        x = np.zeros_like(b2, order="F")
        it = np.zeros(b2.shape[1], np.int32)
        rr = np.zeros(b2.shape[1])
        st = lib().aifmm_gmres(oph, self._h, _ptr(b2), b2.shape[1], self.N, float(rtol), restart, maxit, _ptr(x),
                               self.N, _ptr(it), _ptr(rr))
        if st != 0 and (raise_on_noconv or st != 6):
            _check(st, self._h)
        return x.reshape(np.shape(b)), it, rr

    def ranks(self, level):
        out = np.zeros(1 << (self.d * level), np.int32)
        _check(lib().aifmm_get_ranks(self._h, level, _ptr(out)), self._h)
        return out

    def nnca(self, level, box):
        """(t_i, s_i, U) of one box: pivots as original point indices, the NNCA operator."""
        k, m = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().aifmm_get_nnca(self._h, level, box, None, None, None, ctypes.byref(k), ctypes.byref(m)), self._h)
        ti = np.zeros(max(k.value, 1), np.int64)
        si = np.zeros(max(k.value, 1), np.int64)
        U = np.zeros((max(m.value, 1), max(k.value, 1)))
        U = np.zeros((m.value, k.value))
        _check(lib().aifmm_get_nnca(self._h, level, box, _ptr(ti), _ptr(si), _ptr(U) if U.size else None,
                                    ctypes.byref(k), ctypes.byref(m)), self._h)
        return ti[: k.value], si[: k.value], U

    def trace(self):
        """Compression decision log: (records n x 10 int32, ratios n x 8)."""
        cnt = ctypes.c_int64()
        _check(lib().aifmm_get_trace(self._h, None, None, 0, ctypes.byref(cnt)), self._h)
        n = cnt.value
        rec = np.zeros((max(n, 1), 10), np.int32)
        rat = np.zeros((max(n, 1), 8))
        _check(lib().aifmm_get_trace(self._h, _ptr(rec), _ptr(rat), n, ctypes.byref(cnt)), self._h)
        return rec[:n], rat[:n]

    def level_stats(self, level):
        """Per-level figures of the last factorization (aifmm_get_level_stats)."""
        out = np.zeros(16)
        _check(lib().aifmm_get_level_stats(self._h, level, _ptr(out)), self._h)
        return dict(zip(LSTAT_NAMES, out[: len(LSTAT_NAMES)]))

    def stats(self):
        out = np.zeros(16)
        _check(lib().aifmm_get_stats(self._h, _ptr(out)), self._h)
        return dict(zip(STAT_NAMES, out[: len(STAT_NAMES)]))


def factor_batch(systems, group=256):
    """Factor independent systems in lockstep groups of up to `group` systems
    (aifmm_factor_batch): each launch carries the work of every system of a group."""
    arr = (ctypes.c_void_p * len(systems))(*[s._h for s in systems])
    st = lib().aifmm_factor_batch(arr, len(systems), int(group))
    if st != 0:
        bad = [i for i, s in enumerate(systems) if lib().aifmm_last_error(s._h)]
        raise AifmmError(st, f"batched factorization failed (systems with errors: {bad[:8]})")


class Server:
    """Resident factorizations answering solve requests with continuous per-system batching
    (aifmm_server_*).  submit() copies the right-hand sides and returns a ticket; wait(ticket)
    returns (x, latency_s, batch_cols, iters, relres)."""

    def __init__(self, systems, hbm_budget=0, rtol=1e-10, max_cols=64):
        self._systems = list(systems)
        arr = (ctypes.c_void_p * len(self._systems))(*[s._h for s in self._systems])
        h = ctypes.c_void_p()
        _check(lib().aifmm_server_create(arr, len(self._systems), int(hbm_budget), float(rtol), int(max_cols),
                                         ctypes.byref(h)))
        self._h = h
        self._nrhs = {}

    def submit(self, sys, b):
        if not 0 <= int(sys) < len(self._systems):
            raise AifmmError(1, f"no system {sys} on this server")
        s = self._systems[sys]
        b2 = np.asfortranarray(np.asarray(b, dtype=np.float64).reshape(s.N, -1))
        t = ctypes.c_int64()
        _check(lib().aifmm_server_submit(self._h, int(sys), _ptr(b2), b2.shape[1], s.N, ctypes.byref(t)))
        self._nrhs[t.value] = (sys, b2.shape[1], np.shape(b))
        return t.value

    def wait(self, ticket):
        sys, nr, shape = self._nrhs.pop(ticket)
        n = self._systems[sys].N
        x = np.zeros((n, nr), order="F")
        lat = ctypes.c_double()
        bc = ctypes.c_int32()
        it = np.zeros(nr, np.int32)
        rr = np.zeros(nr)
        _check(lib().aifmm_server_wait(self._h, int(ticket), _ptr(x), n, ctypes.byref(lat), ctypes.byref(bc), _ptr(it),
                                       _ptr(rr)))
        return x.reshape(shape), lat.value, bc.value, it, rr

    def stats(self):
        b, r, p = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        _check(lib().aifmm_server_stats(self._h, ctypes.byref(b), ctypes.byref(r), ctypes.byref(p)))
        return {"batches": b.value, "requests": r.value, "peak_bytes": p.value}

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().aifmm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
