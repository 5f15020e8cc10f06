"""Precision form: Schur updates and compressions in FP32 (FP32 MFMA, FP32 accumulation), the
pivot-block LU, solves, matvec and GMRES in FP64.  The FP32 factorization is an approximate
inverse used as the preconditioner of FP64 flexible GMRES, which must reach a true relative
residual of 1e-10 (checked with the oracle's FP64 O(N^2) product).  The error of each result
against the FP64 oracle is printed: the FP32 direct solve against the oracle's FP64 AIFMM
solution at the same tolerance (bounded by a loose 1e-2, FP32 rounding and rank changes), and
the GMRES solution against the oracle's (bounded by the residual times the conditioning).
"""
import numpy as np
import pytest

import aifmm_inputs as I
import oracle

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2301_12704_amd")

CASES = [
    # (name, n, d, depth, kernel, tol, nrhs, seed)
    ("3d_reduced_shape", 4096, 3, 2, ("invmq", 4096 ** (-1.0 / 3.0), 1.0), 1e-5, 3, 3002),
    ("2d_invmq", 8192, 2, 4, ("invmq", 1e-2, 1.0), 1e-5, 2, 41),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fp32_factor_preconditions_fp64_gmres(case):
    name, n, d, depth, kernel, tol, nrhs, seed = case
    c = I.small_case(n, d=d, depth=depth, tol=tol, kernel=kernel, nrhs=nrhs, seed=seed)
    pts, b = c["pts"], c["b"]
    print(f"case {name} n={n} d={d} depth={depth} tol={tol}", flush=True)
    g32 = A.System(pts, kernel, tol, 64, depth, precision="fp32")
    g32.factor()
    o = oracle.System(pts, kernel, tol, 64, depth)
    o.factor()
    xo = o.solve(b)
    x32 = g32.solve(b)
    e_direct = np.linalg.norm(x32 - xo) / np.linalg.norm(xo)
    r_direct = np.linalg.norm(oracle.matvec(pts, kernel, x32) - b) / np.linalg.norm(b)
    r_oracle = np.linalg.norm(oracle.matvec(pts, kernel, xo) - b) / np.linalg.norm(b)
    print(f"FP32 direct solve: error vs FP64 oracle AIFMM {e_direct:.2e}, residual {r_direct:.2e} "
          f"(oracle's own residual {r_oracle:.2e})")
    assert e_direct <= 1e-2
    ranks32 = [g32.ranks(l) for l in range(2, g32.L + 1)]
    ranks64 = [o.final_ranks(l) for l in range(2, g32.L + 1)]
    diff = sum(int(np.sum(a != bb)) for a, bb in zip(ranks32, ranks64))
    print(f"final ranks differing from the FP64 oracle: {diff} boxes")
    x, it, rr = g32.gmres(b, rtol=1e-10, restart=30, maxit=200)
    res = np.linalg.norm(oracle.matvec(pts, kernel, x) - b, axis=0) / np.linalg.norm(b, axis=0)
    print(f"FGMRES: iterations {list(it)}, true residuals {res}")
    assert np.all(rr <= 1e-10)
    assert np.all(res <= 2e-10)
    e_gm = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print(f"FGMRES solution vs FP64 oracle AIFMM solution: {e_gm:.2e} (the oracle's is limited by its residual)")
    assert e_gm <= 10 * max(r_oracle, 1e-10) * 1e3
