"""Serving form: resident factorizations answer queued solve requests in per-system batches.

Each request's result must be the same alone and in a mix with other requests: with the
direct solve every right-hand side column goes through the same operations whatever the
batch, so the results are equal bit for bit (and equal to aifmm_solve); with GMRES to 1e-10 a
column may take extra iterations while its batch mates converge, so alone and mixed results
agree to the stated tolerance (both residuals <= 1e-10, solutions within 1e-8 relative), and
the true residual of every result is checked with the oracle's O(N^2) product.
"""
import numpy as np
import pytest

import aifmm_inputs as I
import oracle

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2301_12704_amd")


def _systems():
    cases = [
        I.small_case(4096, d=2, depth=3, tol=1e-8, kernel=("exp", 1.0, 0.1), nrhs=1, seed=51),
        I.small_case(3000, d=3, depth=2, tol=1e-6, kernel=("invmq", 3000 ** (-1.0 / 3.0), 1.0), nrhs=1, seed=52),
    ]
    out = []
    for c in cases:
        s = A.System(c["pts"], c["kernel"], c["tol"], 64, 0)
        s.factor()
        out.append((s, c))
    return out


def _rhs(n, k, seed):
    return np.asfortranarray(np.random.default_rng(seed).standard_normal((n, k)))


def test_direct_alone_equals_mixed_and_solve():
    sy = _systems()
    b0 = _rhs(sy[0][0].N, 3, 1)
    x_ref = sy[0][0].solve(b0)
    srv = A.Server([s for s, _ in sy], rtol=0.0, max_cols=64)
    try:
        t = srv.submit(0, b0)
        x_alone, _, bc_alone, _, _ = srv.wait(t)
        np.testing.assert_array_equal(x_alone, x_ref)
        # a burst of requests on both systems, the probe request in the middle
        tickets = []
        for q in range(12):
            sys = q % 2
            tickets.append((sys, srv.submit(sys, _rhs(sy[sys][0].N, 1 + q % 5, 100 + q)), None))
            if q == 5:
                tickets.append((0, srv.submit(0, b0), "probe"))
        merged = 0
        for sys, t, tag in tickets:
            x, lat, bc, _, _ = srv.wait(t)
            assert lat >= 0.0
            if tag == "probe":
                np.testing.assert_array_equal(x, x_alone)
                print(f"probe served in a batch of {bc} columns")
            merged = max(merged, bc)
        st = srv.stats()
        assert st["requests"] == 14
        print("server stats", st, "largest batch", merged)
    finally:
        srv.close()


def test_gmres_alone_and_mixed_within_tolerance():
    sy = _systems()
    srv = A.Server([s for s, _ in sy], rtol=1e-10, max_cols=64)
    try:
        b1 = _rhs(sy[1][0].N, 2, 7)
        x_alone, _, _, it, rr = srv.wait(srv.submit(1, b1))
        assert np.all(rr <= 1e-10)
        tickets = [srv.submit(q % 2, _rhs(sy[q % 2][0].N, 1 + q % 4, 200 + q)) for q in range(6)]
        tp = srv.submit(1, b1)
        tickets += [srv.submit(q % 2, _rhs(sy[q % 2][0].N, 2, 300 + q)) for q in range(4)]
        x_mix, _, bc, it2, rr2 = srv.wait(tp)
        for t in tickets:
            srv.wait(t)
        assert np.all(rr2 <= 1e-10)
        s, c = sy[1]
        for x in (x_alone, x_mix):
            res = np.linalg.norm(oracle.matvec(c["pts"], c["kernel"], x) - b1, axis=0) / np.linalg.norm(b1, axis=0)
            assert np.all(res <= 2e-10), res
        err = np.linalg.norm(x_mix - x_alone) / np.linalg.norm(x_alone)
        print(f"alone vs mixed (batch {bc} columns): rel. difference {err:.2e}, iters {it} / {it2}")
        assert err <= 1e-8
    finally:
        srv.close()


def test_server_argument_errors():
    sy = _systems()
    srv = A.Server([sy[0][0]], rtol=0.0, max_cols=4)
    try:
        with pytest.raises(A.AifmmError):
            srv.submit(0, _rhs(sy[0][0].N, 5, 1))   # more columns than max_cols
        with pytest.raises(A.AifmmError):
            srv.submit(3, _rhs(sy[0][0].N, 1, 1))   # no such system
    finally:
        srv.close()
    with pytest.raises(A.AifmmError):
        A.Server([sy[0][0], sy[0][0]])              # a system listed twice


def test_admission_by_memory_budget():
    """With a budget smaller than any batch, batches are admitted one at a time (a batch with no
    other running is admitted): results are unchanged, and the peak charge is what the systems
    hold in retained workspaces plus at most one batch's growth."""
    sy = _systems()
    srv = A.Server([s for s, _ in sy], hbm_budget=1, rtol=0.0, max_cols=8)
    try:
        reqs = [(q % 2, _rhs(sy[q % 2][0].N, 1 + q % 8, 400 + q)) for q in range(10)]
        tickets = [srv.submit(sys, b) for sys, b in reqs]
        for (sys, b), t in zip(reqs, tickets):
            x, _, bc, _, _ = srv.wait(t)
            np.testing.assert_array_equal(x, sy[sys][0].solve(b))
        st = srv.stats()
        # retained solve workspaces of both systems at 8 columns, plus one batch's estimate
        bound = sum(s.N for s, _ in sy) * 8 * 8 * 8 * 4 + max(s.N for s, _ in sy) * 8 * 8 * 8
        print("peak charged bytes", st["peak_bytes"], "bound", bound)
        assert 0 < st["peak_bytes"] <= bound
    finally:
        srv.close()


def test_busy_when_device_memory_is_short(monkeypatch):
    """A batch whose workspace growth does not fit in the device's free memory, with no other
    batch running, completes its requests with AIFMM_ERR_BUSY instead of failing (the free
    memory figure is forced to zero from the host); submitted again with memory available,
    the same request is served and equals the direct solve."""
    sy = _systems()
    s0 = sy[0][0]
    b = _rhs(s0.N, 4, 77)
    monkeypatch.setenv("AIFMM_DEBUG_FREE_BYTES", "0")
    srv = A.Server([s0], rtol=0.0, max_cols=8)
    try:
        t = srv.submit(0, b)
        with pytest.raises(A.AifmmError) as ei:
            srv.wait(t)
        assert ei.value.status == 8
    finally:
        srv.close()
    monkeypatch.delenv("AIFMM_DEBUG_FREE_BYTES")
    srv = A.Server([s0], rtol=0.0, max_cols=8)
    try:
        x, _, _, _, _ = srv.wait(srv.submit(0, b))
        np.testing.assert_array_equal(x, s0.solve(b))
    finally:
        srv.close()
