"""The NNCA-based H^2 product (Sec. 2.3 operator table; the paper's GMRES operator, Sec. 4) on the
device, and flexible GMRES with it as the operator.

- against the brute-force FP64 product of the oracle: the device's H^2 error is the same
  approximation error as the oracle's own H^2 product with the same NNCA (within a factor 3,
  and <= 5e-11 relative at eps_G = 1e-12 on these workloads): the truncation of the far field
  is the only difference from the exact product;
- FGMRES with the H^2 operator at eps_G = 1e-14 and the factorization at eps_A as
  preconditioner reaches 1e-10 on the operator, and the oracle's brute-force residual of the
  result is <= 1e-10 plus the operator's own error (at eps_G = 1e-12 the operator error alone
  leaves brute-force residuals of 2-5e-10 on this workload, hence the tighter eps_G);
- an operator system given separately gives the same iterates as the built-in one, and one
  from other points is rejected.
"""
import ctypes

import numpy as np
import pytest

import aifmm_inputs as I
import oracle

pytestmark = pytest.mark.gpu
A = pytest.importorskip("paper_2301_12704_amd")

H2_CASES = [
    # (name, n, d, depth, kernel, eps_G)
    ("exp_2d", 4096, 2, 3, ("exp", 1.0, 0.1), 1e-12),
    ("invmq_2d", 4096, 2, 3, ("invmq", 1e-2, 1.0), 1e-12),
    ("invmq_2d_L4", 8192, 2, 4, ("invmq", 1e-2, 1.0), 1e-10),
    ("invmq_3d", 4096, 3, 2, ("invmq", 4096 ** (-1.0 / 3.0), 1.0), 1e-12),
]


@pytest.mark.parametrize("case", H2_CASES, ids=[c[0] for c in H2_CASES])
def test_h2_matvec_against_brute_force(case):
    name, n, d, depth, kern, epsg = case
    c = I.small_case(n, d=d, depth=depth, tol=epsg, kernel=kern, nrhs=5, seed=51)
    print(f"case h2 {name} n={n} d={d} depth {depth} eps_G {epsg}", flush=True)
    g = A.System(c["pts"], kern, epsg, 64, depth)
    y = g.matvec_h2(c["b"])
    yex = oracle.matvec(c["pts"], kern, c["b"])
    o = oracle.System(c["pts"], kern, epsg, 64, depth)
    yo = o.h2_matvec(c["b"])
    e_dev = np.linalg.norm(y - yex) / np.linalg.norm(yex)
    e_or = np.linalg.norm(yo - yex) / np.linalg.norm(yex)
    print(f"H2 error vs brute force: device {e_dev:.2e}, oracle {e_or:.2e}")
    assert e_dev <= 3.0 * e_or + 1e-14
    if epsg <= 1e-12:
        assert e_dev <= 5e-11
    g.close()


def test_gmres_with_h2_operator():
    c = I.small_case(8192, d=2, depth=4, tol=1e-8, kernel=("invmq", 1e-2, 1.0), nrhs=3, seed=52)
    print("case gmres h2 n=8192 depth 4", flush=True)
    g = A.System(c["pts"], c["kernel"], 1e-8, 64, 4, matvec_tol=1e-14)
    g.factor()
    x, its, rr = g.gmres(c["b"], rtol=1e-10, restart=30, maxit=100)
    assert np.all(rr <= 1e-10)
    true = np.linalg.norm(oracle.matvec(c["pts"], c["kernel"], x) - c["b"], axis=0) / np.linalg.norm(c["b"], axis=0)
    print("iterations", its, "operator residual", rr, "brute-force residual", true)
    assert np.all(true <= 1.2e-10), true
    # a separate operator system built from the same points gives the same iterates
    op = A.System(c["pts"], c["kernel"], 1e-14, 64, 4)
    x2, its2, rr2 = g.gmres(c["b"], rtol=1e-10, restart=30, maxit=100, op=op)
    np.testing.assert_array_equal(x2, x)
    np.testing.assert_array_equal(its2, its)
    # an operator from other points is rejected
    c2 = I.small_case(8192, d=2, depth=4, tol=1e-8, kernel=("invmq", 1e-2, 1.0), nrhs=1, seed=53)
    bad = A.System(c2["pts"], c["kernel"], 1e-14, 64, 4)
    with pytest.raises(A.AifmmError) as e:
        g.gmres(c["b"], op=bad)
    assert e.value.status == 1
    for s in (g, op, bad):
        s.close()
