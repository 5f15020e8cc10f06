"""The C-ABI library loads on a machine without a GPU and exports every function that
include/aifmm.h declares; argument checks that precede any device call return the
documented status codes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aifmm.h")
LIB = os.path.join(ROOT, "paper_2301_12704_amd", "libaifmm.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aifmm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libaifmm.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert {"aifmm_build", "aifmm_factor", "aifmm_solve", "aifmm_destroy"} <= set(names)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/aifmm.h but not exported"


def test_argument_errors_without_device(lib):
    import paper_2301_12704_amd as A
    L = A.lib()
    opt = A._Options()
    assert L.aifmm_options_default(ctypes.byref(opt)) == 0
    assert (opt.dim, opt.leaf_size, opt.depth, opt.device) == (2, 64, 0, 0)
    h = ctypes.c_void_p()
    k = A._Kernel(0, 1.0, 0.1)
    assert L.aifmm_build(None, 100, k, 1e-8, ctypes.byref(opt), ctypes.byref(h)) == 1
    import numpy as np
    pts = np.zeros((10, 2))
    bad = A._Kernel(7, 1.0, 0.1)
    assert L.aifmm_build(pts.ctypes.data_as(ctypes.c_void_p), 10, bad, 1e-8, ctypes.byref(opt), ctypes.byref(h)) == 1
    assert L.aifmm_build(pts.ctypes.data_as(ctypes.c_void_p), 10, k, 0.0, ctypes.byref(opt), ctypes.byref(h)) == 1
    opt.dim = 4
    assert L.aifmm_build(pts.ctypes.data_as(ctypes.c_void_p), 10, k, 1e-8, ctypes.byref(opt), ctypes.byref(h)) == 1
    assert L.aifmm_get_depth(None, None) == 1
    assert L.aifmm_factor(None) == 1
    assert L.aifmm_solve(None, None, 1, 1, None, 1) == 1
    assert "NULL" in L.aifmm_last_error(None).decode() or L.aifmm_last_error(None)
    L.aifmm_destroy(None)


def test_server_argument_errors_without_device(lib):
    import paper_2301_12704_amd as A
    L = A.lib()
    h = ctypes.c_void_p()
    assert L.aifmm_server_create(None, 1, 0, 0.0, 8, ctypes.byref(h)) == 1
    arr = (ctypes.c_void_p * 1)(None)
    assert L.aifmm_server_create(arr, 1, 0, 0.0, 8, ctypes.byref(h)) == 1
    assert L.aifmm_server_create(arr, 0, 0, 0.0, 8, ctypes.byref(h)) == 1
    t = ctypes.c_int64()
    assert L.aifmm_server_submit(None, 0, None, 1, 1, ctypes.byref(t)) == 1
    assert L.aifmm_server_wait(None, 1, None, 1, None, None, None, None) == 1
    assert L.aifmm_server_stats(None, None, None, None) == 1
    L.aifmm_server_destroy(None)


def test_binding_argument_counts_match_header():
    """Every function the binding declares takes as many arguments as include/aifmm.h says."""
    import paper_2301_12704_amd as A
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    decl = {}
    for m in re.finditer(r"\b(aifmm_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", text):
        args = m.group(2).strip()
        decl[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    L = A.lib()
    checked = 0
    for name, n in decl.items():
        at = getattr(L, name).argtypes
        if at is not None:
            assert len(at) == n, f"{name}: binding has {len(at)} argument types, header {n}"
            checked += 1
    assert checked >= 20
