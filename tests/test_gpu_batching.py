"""Batching form: independent systems of different sizes and depths factored in lockstep
(aifmm_factor_batch: every launch carries the work of all systems) give exactly the factors of
one-at-a-time factorization: compression traces (ranks and decision ratios), rank tables and
solutions are bit-identical, and the FP64 ones match the oracle (ranks bit-exact, solution
within 1e-8) on a sampled system."""
import numpy as np
import pytest

import aifmm_inputs as I
import oracle

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2301_12704_amd")


def _batch(count=6, prec="fp64", tol=1e-8):
    sizes = I.batch_sizes(count=count, seed=4999, lo=2048, hi=8192)
    out = []
    for q, n in enumerate(sizes):
        pts, b = I.points_and_rhs(int(n), 2, 1, 4000 + q)
        out.append((pts, b))
    return out


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-5)])
def test_batch_equals_sequential(prec, tol):
    kern = ("exp", 0.5, 0.05)
    data = _batch()
    seq = [A.System(p, kern, tol, 64, 0, precision=prec) for p, _ in data]
    for s in seq:
        s.factor()
    bat = [A.System(p, kern, tol, 64, 0, precision=prec) for p, _ in data]
    A.factor_batch(bat)
    assert len({s.L for s in bat}) > 1, "the batch should mix depths"
    for (p, b), s1, s2 in zip(data, seq, bat):
        r1, q1 = s1.trace()
        r2, q2 = s2.trace()
        np.testing.assert_array_equal(r1, r2)
        np.testing.assert_array_equal(q1, q2)
        for l in range(2, s1.L + 1):
            np.testing.assert_array_equal(s1.ranks(l), s2.ranks(l))
        np.testing.assert_array_equal(s1.solve(b), s2.solve(b))
    if prec == "fp64":
        p, b = data[0]
        o = oracle.System(p, kern, tol, 64, 0)
        o.factor()
        for l in range(2, bat[0].L + 1):
            np.testing.assert_array_equal(bat[0].ranks(l), o.final_ranks(l))
        xo = o.solve(b)
        err = np.linalg.norm(bat[0].solve(b) - xo) / np.linalg.norm(xo)
        assert err <= 1e-8
    for s in seq + bat:
        s.close()


def test_batch_argument_errors():
    p, _ = _batch(count=1)[0]
    s = A.System(p, ("exp", 0.5, 0.05), 1e-8, 64, 0)
    with pytest.raises(A.AifmmError):
        A.factor_batch([s, s])
    s.factor()
    with pytest.raises(A.AifmmError):
        A.factor_batch([s])
    s.close()
