"""Pins of the oracle's dense building blocks against closed forms, library routines used as
independent references, and brute force on tiny inputs.

- ACA with partial pivoting (the NNCA pivot search): an exact rank-r matrix is recovered with rank r; the
  skeleton (cross) identity M[:,J] M[I,J]^{-1} M[I,:]; the pivot rule (argmax of the residual
  row/column) checked step by step from the returned factors.
- RRQR (Sec. 3.2.1, Householder QR with column pivoting): orthonormal Q, upper-triangular R in pivoted order,
  truncation rank against prescribed singular values, truncation residual bound.
- Dense partial-pivot LU against numpy.linalg.solve and a singular case.
- Kernel entries against closed forms; brute-force matvec against a numpy product.
"""
import numpy as np
import pytest

import oracle


def test_kernel_closed_form():
    pts = np.array([[0.0, 0.0], [3.0, 4.0], [0.0, 1.0]])
    K = oracle.dense_matrix(pts, ("exp", 2.0, 0.5))
    assert K[0, 1] == pytest.approx(np.exp(-5.0 / 2.0), rel=1e-15)
    assert K[0, 0] == pytest.approx(1.5, rel=1e-15)
    K2 = oracle.dense_matrix(pts, ("invmq", 0.01, 1.0))
    assert K2[0, 2] == pytest.approx(1.0 / np.sqrt(1.0 + 1e-4), rel=1e-15)
    assert K2[2, 2] == pytest.approx(1.0 / 0.01 + 1.0, rel=1e-15)
    assert np.array_equal(K2, K2.T)


def test_matvec_matches_dense_product():
    rng = np.random.default_rng(1)
    pts = rng.uniform(-1, 1, (300, 2))
    x = rng.standard_normal((300, 3))
    A = oracle.dense_matrix(pts, ("exp", 1.0, 0.1))
    y = oracle.matvec(pts, ("exp", 1.0, 0.1), np.asfortranarray(x))
    np.testing.assert_allclose(y, A @ x, rtol=1e-12, atol=1e-12)
    rows = np.array([5, 17, 299])
    yr = oracle.matvec_rows(pts, ("exp", 1.0, 0.1), rows, np.asfortranarray(x))
    np.testing.assert_allclose(yr, (A @ x)[rows], rtol=1e-12)


def test_dense_solve():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((60, 60)) + 10 * np.eye(60)
    B = rng.standard_normal((60, 4))
    X = oracle.dense_solve(A, np.asfortranarray(B))
    np.testing.assert_allclose(X, np.linalg.solve(A, B), rtol=1e-12, atol=1e-13)
    S = A.copy()
    S[:, 7] = 0.0
    with pytest.raises(np.linalg.LinAlgError):
        oracle.dense_solve(S, np.asfortranarray(B))


@pytest.mark.parametrize("r", [1, 3, 8])
def test_aca_exact_rank(r):
    rng = np.random.default_rng(10 + r)
    M = rng.standard_normal((40, r)) @ rng.standard_normal((r, 70))
    I, J, U, V = oracle.aca(M, 1e-12)
    # the stopping test is taken after a term is added and that term is kept, so on an
    # exact rank-r matrix the last of at most r+1 terms is rounding noise below the tolerance
    assert len(I) in (r, r + 1)
    if len(I) == r + 1:
        assert np.linalg.norm(U[:, r]) * np.linalg.norm(V[r]) <= 1e-12 * np.linalg.norm(U @ V)
        I, J, U, V = I[:r], J[:r], U[:, :r], V[:r]
    err = np.linalg.norm(M - U @ V) / np.linalg.norm(M)
    assert err < 1e-12
    cross = M[:, J] @ np.linalg.solve(M[np.ix_(I, J)], M[I, :])
    assert np.linalg.norm(U @ V - cross) / np.linalg.norm(M) < 1e-12


def test_aca_pivot_rule_stepwise():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (30, 2))
    y = rng.uniform(3, 4, (50, 2))
    M = 1.0 / np.sqrt(((x[:, None, :] - y[None, :, :]) ** 2).sum(-1))
    I, J, U, V = oracle.aca(M, 1e-9)
    assert I[0] == 0
    for k in range(len(I)):
        R = M - U[:, :k] @ V[:k]
        row = np.abs(R[I[k]])
        row[J[:k]] = -1
        assert J[k] == int(np.argmax(row))
        if k + 1 < len(I):
            col = np.abs(R[:, J[k]])
            col[I[: k + 1]] = -1
            assert I[k + 1] == int(np.argmax(col))
    # the approximation meets the tolerance on this smooth block
    assert np.linalg.norm(M - U @ V) / np.linalg.norm(M) < 1e-7


def test_aca_zero_matrix_and_empty():
    I, J, U, V = oracle.aca(np.zeros((5, 6)), 1e-8)
    assert len(I) == 0


def test_cpqr_full_rank_factorization():
    rng = np.random.default_rng(4)
    M = rng.standard_normal((20, 12))
    k, Q, perm, R = oracle.cpqr(M, 1e-15)
    assert k == 12
    assert np.linalg.norm(Q.T @ Q - np.eye(20)) < 1e-13
    assert np.allclose(np.tril(R[:, :12], -1), 0.0)
    np.testing.assert_allclose(Q[:, :12] @ R, M[:, perm], atol=1e-13)
    d = np.abs(np.diag(R))
    assert np.all(d[:-1] >= d[1:] * (1 - 1e-12))  # pivoting gives non-increasing |R_kk|
    assert sorted(perm) == list(range(12))


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
def test_cpqr_truncation_rank(tol):
    rng = np.random.default_rng(5)
    Ua, _ = np.linalg.qr(rng.standard_normal((40, 15)))
    Va, _ = np.linalg.qr(rng.standard_normal((30, 15)))
    sig = 10.0 ** (-np.arange(15) * 0.75)
    M = Ua @ np.diag(sig) @ Va.T
    k, Q, perm, R = oracle.cpqr(M, tol, qcols=40)
    sv = np.linalg.svd(M, compute_uv=False)
    # |R_kk| brackets the singular values within the classical factor sqrt(n) (k+1 ...)
    assert sv[k] <= np.sqrt(30) * np.sqrt(k + 1) * tol * sv[0] * 10 or k == 15
    res = np.linalg.norm(M[:, perm] - Q[:, :k] @ R, 2)
    nxt = np.linalg.norm((Q[:, k:].T @ M[:, perm])[:, k:], axis=0).max() if k < 15 else 0.0
    assert res <= np.sqrt(30 - k) * max(nxt, 1e-300) * (1 + 1e-9) + 1e-15
    assert nxt <= tol * abs(R[0, 0]) * (1 + 1e-12)
    assert abs(R[k - 1, k - 1]) > tol * abs(R[0, 0])
    assert np.linalg.norm(Q.T @ Q - np.eye(40)) < 1e-13


def test_cpqr_zero_and_tiny():
    k, Q, perm, R = oracle.cpqr(np.zeros((6, 4)), 1e-8)
    assert k == 0
    assert np.allclose(Q, np.eye(6))
    k, Q, perm, R = oracle.cpqr(np.ones((3, 1)), 1e-8)
    assert k == 1 and abs(abs(R[0, 0]) - np.sqrt(3)) < 1e-14
