"""Pins of the readings where the paper fixes no operation order or arithmetic routine.

The oracle's default mode takes the orders the device also takes: the e^x routine of the
exponential kernel (Cody-Waite reduction and a Taylor polynomial), row sums of the pivoted QRs
in sixteen interleaved chains and a tree, the column-oriented back substitution of the pivot
blocks, and colour rounds (all compressions of a colour round, left factors then right factors,
then the colour's eliminations).  The textbook mode replaces each by its plainest reading:
the C library's exp, one ascending chain per row sum, ascending back substitution, and the
Algorithm's box-by-box order (Sec. 3.3).

A rank decision of a pivoted QR compares a pivot of size about eps_A |R_11| with eps_A |R_11|;
rounding changes that pivot by about u |R_11|, i.e. by u / eps_A relative, and a different
pivot order (near-equal trailing norms) changes the whole sequence of pivots.  So no rank
table is independent of the operation order: ranks agree bit for bit only between two codes
that execute the same operations (the device and the default mode).  What the readings must
not change is the method's accuracy.  The pins:
- the NNCA (Sec. 2.3) is independent of the three elimination readings, and of the exp
  routine at the tolerances used here: identical ranks and pivots;
- the textbook mode's solution differs from the default mode's by at most a quarter of the
  method's own error against the dense solution (numpy.linalg.solve), and the two brute-force
  residuals agree within 10%; the rank tables differ only by a few units in a few boxes;
- in both modes no compression transforms a row whose right-hand side can be nonzero (the
  right-hand side is untouched by compressions, so the solve needs no compression data);
- the exp routine is within one unit in the last place of numpy.exp over [-745, 0].
"""
import numpy as np
import pytest

import aifmm_inputs as I
import oracle

CASES = [
    # (name, n, d, depth, kernel, tol, nrhs, seed): the GPU parity cases the oracle finishes in seconds
    ("exp_L2", 1024, 2, 2, ("exp", 1.0, 0.1), 1e-10, 1, 7),
    ("c1_config", 4096, 2, 3, ("exp", 1.0, 0.1), 1e-10, 1, 1001),
    ("invmq_L3", 4096, 2, 3, ("invmq", 1e-2, 1.0), 1e-8, 3, 21),
    ("ragged_2000", 2000, 2, 3, ("exp", 1.0, 0.1), 1e-8, 2, 22),
    ("3d_L2_small", 1500, 3, 2, ("invmq", 1500 ** (-1.0 / 3.0), 1.0), 1e-6, 2, 24),
]


def _ulps(a, b):
    """Distance in units in the last place between non-negative doubles."""
    ia = a.view(np.int64)
    ib = b.view(np.int64)
    return np.abs(ia - ib)


def test_kexp_within_one_ulp_of_numpy():
    rng = np.random.default_rng(11)
    x = np.concatenate([
        rng.uniform(-745.0, 0.0, 200000),
        rng.uniform(-1.0, 0.0, 50000),                     # the kernel's usual range
        -np.arange(0, 1075) * np.log(2.0),                 # reduction boundaries k ln 2
        -np.arange(0, 1075) * np.log(2.0) - 0.5 * np.log(2.0),  # half-way points of the reduction
        np.linspace(-745.0, -708.0, 20001),               # subnormal results
        [0.0, -0.0, -1e-300, -5e-324, -745.0, -708.3964185322641, -1.0],
    ])
    x = x[x >= -745.0]
    got = oracle.kexp(x)
    ref = np.exp(x)
    assert np.all(np.isfinite(got)) and np.all(got >= 0.0)
    d = _ulps(got, ref)
    assert d.max() <= 1, f"max {d.max()} ulp at x = {x[np.argmax(d)]!r}"
    assert np.mean(d == 0) > 0.9  # mostly correctly rounded
    assert oracle.kexp(np.array([-746.0, -1e4]))[0] == 0.0


def _dense_error(c, x):
    A = oracle.dense_matrix(c["pts"], c["kernel"])
    xd = np.linalg.solve(A, c["b"])
    return np.linalg.norm(x - xd) / np.linalg.norm(xd)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_textbook_readings_are_accuracy_neutral(case):
    name, n, d, depth, kern, tol, nrhs, seed = case
    c = I.small_case(n, d=d, depth=depth, tol=tol, kernel=kern, nrhs=nrhs, seed=seed)
    sys = {}
    for mode in (0, oracle.MODE_TEXTBOOK):
        o = oracle.System(c["pts"], kern, tol, 64, depth, mode=mode)
        o.factor()
        sys[mode] = (o, o.solve(c["b"]))
    (o0, x0), (o1, x1) = sys[0], sys[oracle.MODE_TEXTBOOK]
    for l in range(2, o0.L + 1):
        np.testing.assert_array_equal(o0.nnca_ranks(l), o1.nnca_ranks(l), err_msg=f"NNCA ranks level {l}")
        for box in range(0, 1 << (d * l), max(1, (1 << (d * l)) // 8)):
            for a, b in zip(o0.pivots(l, box), o1.pivots(l, box)):
                np.testing.assert_array_equal(a, b)
    assert o0.rhs_violations() == 0 and o1.rhs_violations() == 0
    assert o0.far_fill() == 0 and o1.far_fill() == 0
    err0 = _dense_error(c, x0)
    diff = np.linalg.norm(x1 - x0) / np.linalg.norm(x0)
    assert diff <= 0.25 * err0 + 1e-13, (diff, err0)  # plus a rounding floor where nothing is truncated
    r0 = np.linalg.norm(oracle.matvec(c["pts"], kern, x0) - c["b"]) / np.linalg.norm(c["b"])
    r1 = np.linalg.norm(oracle.matvec(c["pts"], kern, x1) - c["b"]) / np.linalg.norm(c["b"])
    assert abs(r1 - r0) <= 0.1 * r0, (r0, r1)
    dk = np.concatenate([o1.final_ranks(l) - o0.final_ranks(l) for l in range(2, o0.L + 1)])
    assert np.abs(dk).max() <= 5 and np.count_nonzero(dk) <= 0.2 * dk.size, dk[dk != 0]
    print(f"{name}: error vs dense {err0:.2e}, textbook - default {diff:.2e}, "
          f"ranks differing {np.count_nonzero(dk)}/{dk.size}")


def test_sequential_order_matches_colour_rounds():
    """Colour rounds against the Algorithm's box-by-box order alone (the other readings kept):
    same-colour boxes touch disjoint rows and columns except for a left and a right factor
    on some interaction blocks, which commute in exact arithmetic, so the two orders differ by
    rounding only: the same compressions, rank tables within a unit in a few boxes, and
    solutions within a small fraction of the method's error against the dense solve."""
    c = I.small_case(4096, d=2, depth=3, tol=1e-8, kernel=("invmq", 1e-2, 1.0), nrhs=3, seed=21)
    o0 = oracle.System(c["pts"], c["kernel"], c["tol"], 64, 3)
    o1 = oracle.System(c["pts"], c["kernel"], c["tol"], 64, 3, mode=oracle.MODE_SEQUENTIAL)
    o0.factor()
    o1.factor()
    dk = np.concatenate([o1.final_ranks(l) - o0.final_ranks(l) for l in (2, 3)])
    assert np.abs(dk).max() <= 2 and np.count_nonzero(dk) <= 0.05 * dk.size, dk[dk != 0]
    # the same compressions (as a set); the sequential log lists them box by box
    assert sorted(map(tuple, o0.trace())) == sorted(map(tuple, o1.trace()))
    x0, x1 = o0.solve(c["b"]), o1.solve(c["b"])
    err0 = _dense_error(c, x0)
    assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) <= 0.25 * err0


def test_interpolation_identity():
    """U_B = A[T_B, s^{B,i}] (A[t^{B,i}, s^{B,i}])^{-1} reproduces the identity on its own
    pivot rows t^{B,i} (Sec. 2.3, the NNCA interpolation operators), at every level.  A
    transposed cross matrix, a wrong pivot list or a missing inverse is off by O(1)."""
    c = I.small_case(2048, d=2, depth=3, tol=1e-8, kernel=("exp", 1.0, 0.1), nrhs=1, seed=91)
    o = oracle.System(c["pts"], c["kernel"], c["tol"], 64, 3)
    checked = 0
    for l in (2, 3):
        for box in range(1 << (2 * l)):
            k = int(o.nnca_ranks(l)[box])
            if k == 0:
                continue
            T = o.row_set(l, box)
            U = o.nnca_U(l, box)
            ti, si = o.pivots(l, box)
            assert U.shape == (len(T), k)
            pos = {int(t): r for r, t in enumerate(T)}
            rows = np.array([pos[int(t)] for t in ti])
            # exact in exact arithmetic; in FP64 to about u cond(C) (the cross matrix C of an
            # ACA at tolerance eps_A is as ill-conditioned as about 1 / eps_A)
            C = oracle.kernel_block(c["pts"], c["kernel"], ti, si)
            bound = 100 * np.finfo(float).eps * np.linalg.cond(C)
            np.testing.assert_allclose(U[rows], np.eye(k), rtol=0, atol=max(bound, 1e-14))
            checked += 1
    assert checked > 60
