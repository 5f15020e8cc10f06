"""Full-size checks at the benchmark's workload (c2: N=262144, 2D, depth 6, 16 RHS), in the
launch configuration bench.py times.  The oracle cannot factor this size in reasonable time,
so the checks are on outputs it computes one by one and on properties that hold at any size:
- the FGMRES solution's residual on 256 sampled rows, each row product done by the oracle
  in FP64 (relative to the sampled right-hand side, <= 1e-9);
- every pivoted QR of every compression obeys the truncation rule: the last kept pivot is
  above the tolerance and the first rejected one at or below it (decision ratios of the log);
- the direct solve agrees with the FGMRES solution to the direct factorization's accuracy:
  at this tolerance its relative residual is about 1e-3 (truncation errors of the compressed
  fill-ins, amplified through the elimination), measured agreement 8e-5, checked <= 1e-3.
A second workload (N=65536) is factored twice: the factorizations are bit-identical."""
import numpy as np
import pytest

import aifmm_inputs as I
import oracle

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2301_12704_amd")


def test_c2_fullsize_properties():
    cfg = I.config("c2")
    pts, b = cfg["pts"], cfg["b"]
    print(f"c2 N={cfg['n']} depth {cfg['depth']} tol {cfg['tol']} nrhs {cfg['nrhs']}", flush=True)
    s = A.System(pts, cfg["kernel"], cfg["tol"], cfg["leaf"], cfg["depth"])
    s.factor()
    print("factored", flush=True)
    rec, rat = s.trace()
    assert len(rec) > 0
    kinds = rec[:, 2]
    for q in range(4):
        kept, nxt = rat[:, 2 * q], rat[:, 2 * q + 1]
        used = (kinds == 0) | (q < 2)
        assert np.all(kept[used & (kept > 0)] > 1.0 - 1e-12), f"RRQR {q + 1}: a kept pivot below tolerance"
        assert np.all(nxt[used] <= 1.0), f"RRQR {q + 1}: a rejected pivot above tolerance"
    for l in range(2, s.L + 1):
        assert np.all(s.ranks(l) >= 0)
    res_d = oracle.matvec_rows(pts, cfg["kernel"], np.arange(0, cfg["n"], 1024), s.solve(b)) - b[::1024]
    print(f"direct solve, sampled-row residual {np.linalg.norm(res_d) / np.linalg.norm(b[::1024]):.2e}")
    xd = s.solve(b)
    x, its, rr = s.gmres(b, rtol=1e-10, restart=30, maxit=100)
    assert np.all(rr <= 1e-10)
    rows = np.random.default_rng(7).choice(cfg["n"], 256, replace=False)
    res = oracle.matvec_rows(pts, cfg["kernel"], rows, x) - b[rows]
    rel = np.linalg.norm(res, axis=0) / np.linalg.norm(b[rows], axis=0)
    print(f"sampled-row residuals: max {rel.max():.2e}; FGMRES iterations {list(its)}", flush=True)
    assert np.all(rel <= 1e-9)
    dd = np.linalg.norm(xd - x) / np.linalg.norm(x)
    print(f"direct vs FGMRES solution: {dd:.2e}")
    assert dd <= 1e-3
    s.close()


def test_factorization_is_deterministic():
    c = I.small_case(65536, d=2, depth=5, tol=1e-8, kernel=("invmq", 1e-2, 1.0), nrhs=2, seed=2001)
    out = []
    for _ in range(2):
        s = A.System(c["pts"], c["kernel"], c["tol"], 64, 5)
        s.factor()
        rec, rat = s.trace()
        out.append((rec, rat, [s.ranks(l) for l in range(2, 6)], s.solve(c["b"])))
        s.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    for a, b in zip(out[0][2], out[1][2]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(out[0][3], out[1][3])
