"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar (from the method's required outputs): per-level box -> rank tables bit-exact (NNCA ranks,
pivot lists and the ranks chosen by every compression), the decision ratios |R_kk| / (eps_A |R_11|)
of every pivoted QR bit-identical (so every operation on the rank-deciding path agrees, not only
the decisions), solution relative error <= 1e-8
against the oracle's solution, and the brute-force residual of the GPU solution no worse than the
oracle's (0.1%; the solve sums in a blocked order).  Both sides execute the same IEEE operation sequence on the
rank-deciding path (explicit fused multiply-adds, no contraction elsewhere), so the decisions
agree exactly unless a decision ratio lies within rounding of the threshold; the oracle's
decision-margin log is printed on failure for attribution.
"""
import numpy as np
import pytest

import aifmm_inputs as I
import oracle

pytestmark = pytest.mark.gpu

A = pytest.importorskip("paper_2301_12704_amd")

CASES = [
    # (name, n, d, depth, kernel, tol, nrhs, seed)
    ("exp_L2", 1024, 2, 2, ("exp", 1.0, 0.1), 1e-10, 1, 7),
    ("c1_config", 4096, 2, 3, ("exp", 1.0, 0.1), 1e-10, 1, 1001),
    ("invmq_L3", 4096, 2, 3, ("invmq", 1e-2, 1.0), 1e-8, 3, 21),
    ("ragged_2000", 2000, 2, 3, ("exp", 1.0, 0.1), 1e-8, 2, 22),
    ("exp_half_L4", 8192, 2, 4, ("exp", 0.5, 0.05), 1e-8, 1, 23),
    ("3d_L2", 3000, 3, 2, ("invmq", 3000 ** (-1.0 / 3.0), 1.0), 1e-6, 2, 24),
    # 3D with a non-leaf level: the level-2 boxes stack the children's ranks (8 children each)
    ("3d_L3", 2048, 3, 3, ("invmq", 2048 ** (-1.0 / 3.0), 1.0), 1e-5, 2, 26),
]

# Switches of the library that change which kernel path runs, never an operation's order:
# compression columns without the register tier (LDS, then workspace); in registers with the
# rest in the workspace on two-member teams; all in the workspace on teams of up to 128
# members (every member's share small, some members with no column) or of at most 4; lone
# workgroups only; pivot-block LU panels factored in device memory instead of LDS (the path of
# pivot blocks above ~1050 rows); and the pivot-block inverse by the left-looking kernel (the
# small cases otherwise take the right-looking one).
SWITCHES = [
    ("no_register_columns", {"AIFMM_NO_REG_COLUMNS": "1"}),
    ("register_then_workspace_columns", {"AIFMM_NO_LDS_COLUMNS": "1", "AIFMM_TEAM_MAX": "1"}),
    ("workspace_columns_large_teams", {"AIFMM_NO_REG_COLUMNS": "1", "AIFMM_NO_LDS_COLUMNS": "1"}),
    ("workspace_columns_small_teams", {"AIFMM_NO_REG_COLUMNS": "1", "AIFMM_NO_LDS_COLUMNS": "1",
                                       "AIFMM_TEAM_MAX": "2"}),
    ("no_teams", {"AIFMM_NO_TEAMS": "1"}),
    ("lu_panels_in_memory", {"AIFMM_NO_LDS_PANELS": "1"}),
    ("pivot_inverse_left_looking", {"AIFMM_PINV_LEFT": "1"}),
]
SWITCH_CASES = [c for c in CASES if c[0] in ("invmq_L3", "exp_half_L4", "3d_L3")]


def _run(n, d, depth, kernel, tol, nrhs, seed, pts=None):
    if pts is None:
        c = I.small_case(n, d=d, depth=depth, tol=tol, kernel=kernel, nrhs=nrhs, seed=seed)
        pts, b = c["pts"], c["b"]
    else:
        b = np.asfortranarray(np.random.default_rng(seed).standard_normal((pts.shape[0], nrhs)))
    print(f"case n={pts.shape[0]} d={d} depth={depth} kernel={kernel} tol={tol} nrhs={nrhs} seed={seed}", flush=True)
    g = A.System(pts, kernel, tol, 64, depth)
    o = oracle.System(pts, kernel, tol, 64, depth)
    return g, o, pts, b


def _compare(g, o, pts, b, kernel):
    L = g.L
    assert L == o.L
    for l in range(2, L + 1):
        np.testing.assert_array_equal(g.ranks(l), o.nnca_ranks(l), err_msg=f"NNCA ranks level {l}")
        for box in range(0, 1 << (g.d * l), max(1, (1 << (g.d * l)) // 16)):
            ti, si, _ = g.nnca(l, box)
            oti, osi = o.pivots(l, box)
            np.testing.assert_array_equal(ti, oti, err_msg=f"row pivots level {l} box {box}")
            np.testing.assert_array_equal(si, osi, err_msg=f"column pivots level {l} box {box}")
    g.factor()
    o.factor()
    grec, grat = g.trace()
    otr = o.trace()
    ork, ora = o.trace_ranks()
    assert len(grec) == len(otr)
    gmap = {tuple(r[:4]): r[4:] for r in grec}
    rmap = {tuple(r[:4]): q for q, r in enumerate(grec)}
    # the decision ratios |R_kk| / (eps_A |R_11|) of every pivoted QR, as a measure of how far the
    # two sides' arithmetic agrees beyond the ranks (identical when every operation agrees)
    rd = [np.max(np.abs(grat[rmap[tuple(otr[q])]] - ora[q]) / np.maximum(np.abs(ora[q]), 1e-300))
          for q in range(len(otr)) if tuple(otr[q]) in rmap]
    if rd:
        print(f"decision ratios: {np.mean(np.array(rd) == 0):.3f} identical, max rel diff {max(rd):.3e}", flush=True)
        assert max(rd) == 0.0, "decision ratios differ from the oracle's: the arithmetic is not the same"
    for q in range(len(otr)):
        key = tuple(otr[q])
        assert key in gmap, f"compression {key} missing on the device"
        if not np.array_equal(gmap[key], ork[q]):
            pytest.fail(f"compression {key}: device ranks {gmap[key]} oracle {ork[q]} "
                        f"(oracle decision ratios {ora[q]}, min margin {o.margins()[0]:.3e})")
    for l in range(2, L + 1):
        np.testing.assert_array_equal(g.ranks(l), o.final_ranks(l), err_msg=f"final ranks level {l}")
    x = g.solve(b)
    xo = o.solve(b)
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    assert err <= 1e-8, f"solution error vs oracle {err:.3e}"
    res_g = np.linalg.norm(oracle.matvec(pts, kernel, x) - b) / np.linalg.norm(b)
    res_o = np.linalg.norm(oracle.matvec(pts, kernel, xo) - b) / np.linalg.norm(b)
    # the solve phase sums in another order than the oracle (blocked sweeps), so the residuals
    # agree to rounding: the GPU residual may not be worse than the oracle's by more than 0.1%
    assert res_g <= 1.001 * res_o + 1e-14, (res_g, res_o)
    return err, res_g


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_parity(case):
    _, n, d, depth, kernel, tol, nrhs, seed = case
    g, o, pts, b = _run(n, d, depth, kernel, tol, nrhs, seed)
    err, res = _compare(g, o, pts, b, kernel)
    print(f"solution error vs oracle {err:.3e}, residual {res:.3e}")


@pytest.mark.parametrize("case", SWITCH_CASES, ids=[c[0] for c in SWITCH_CASES])
@pytest.mark.parametrize("switch", SWITCHES, ids=[w[0] for w in SWITCHES])
def test_parity_kernel_paths(case, switch, monkeypatch):
    """The same bar on the kernel paths the switches select (bit-exact ranks and pivots)."""
    for k, v in switch[1].items():
        monkeypatch.setenv(k, v)
    print(f"switch {switch[0]}", flush=True)
    _, n, d, depth, kernel, tol, nrhs, seed = case
    g, o, pts, b = _run(n, d, depth, kernel, tol, nrhs, seed)
    err, res = _compare(g, o, pts, b, kernel)
    print(f"solution error vs oracle {err:.3e}, residual {res:.3e}")


def test_team_abort_reports_device_error(monkeypatch):
    """A team barrier that gives up raises the abort flag; the kernels then stop using data
    exchanged through the team and run to their end, and the factorization returns
    AIFMM_ERR_DEVICE.  Forced from the host: the flag is raised before the level's first
    launch, so every team barrier falls through at once (no wait is timed out)."""
    monkeypatch.setenv("AIFMM_DEBUG_ABORT", "1")
    c = I.small_case(8192, d=2, depth=4, tol=1e-8, kernel=("exp", 0.5, 0.05), nrhs=1, seed=37)
    print("case abort n=8192 depth 4", flush=True)
    g = A.System(c["pts"], c["kernel"], c["tol"], 64, 4)
    with pytest.raises(A.AifmmError) as e:
        g.factor()
    assert e.value.status == 5 and "barrier" in str(e.value)
    g.close()
    monkeypatch.delenv("AIFMM_DEBUG_ABORT")
    g = A.System(c["pts"], c["kernel"], c["tol"], 64, 4)
    g.factor()  # the next factorization on the device is unaffected
    g.close()


def test_empty_and_sparse_boxes():
    """Points clustered in one corner and a thin strip: many empty leaves and boxes with a
    handful of points (ranks capped by box sizes)."""
    rng = np.random.default_rng(31)
    a = rng.uniform(-1, -0.2, (1500, 2))
    strip = np.c_[rng.uniform(-1, 1, 500), rng.uniform(0.9, 1.0, 500)]
    pts = np.ascontiguousarray(np.vstack([a, strip]))
    g, o, pts, b = _run(0, 2, 3, ("exp", 1.0, 0.1), 1e-8, 2, 32, pts=pts)
    assert (o.counts(3) == 0).sum() > 10
    _compare(g, o, pts, b, ("exp", 1.0, 0.1))


def test_tiny_boxes():
    """N=200 on a depth-3 tree: ~3 points per leaf, ranks limited by box sizes."""
    c = I.small_case(200, depth=3, tol=1e-10, kernel=("invmq", 1e-2, 1.0), nrhs=1, seed=33)
    g, o, pts, b = _run(200, 2, 3, ("invmq", 1e-2, 1.0), 1e-10, 1, 33, pts=c["pts"])
    _compare(g, o, pts, b, ("invmq", 1e-2, 1.0))


def test_solve_repeat_and_multi_rhs_consistency():
    c = I.small_case(4096, depth=3, tol=1e-8, kernel=("invmq", 1e-2, 1.0), nrhs=5, seed=34)
    g = A.System(c["pts"], c["kernel"], c["tol"], 64, 3)
    g.factor()
    x5 = g.solve(c["b"])
    x1 = g.solve(np.asfortranarray(c["b"][:, 2:3]))
    np.testing.assert_allclose(x1[:, 0], x5[:, 2], rtol=0, atol=1e-13 * np.abs(x5).max())
    x5b = g.solve(c["b"])
    np.testing.assert_array_equal(x5, x5b)


def test_device_pointers():
    torch = pytest.importorskip("torch")
    c = I.small_case(2048, depth=3, tol=1e-8, kernel=("exp", 1.0, 0.1), nrhs=2, seed=35)
    pts_d = torch.from_numpy(c["pts"]).cuda()
    g = A.System(pts_d, c["kernel"], c["tol"], 64, 3)
    g.factor()
    b_d = torch.from_numpy(np.ascontiguousarray(c["b"].T)).cuda()  # (nrhs, N): column-major N x nrhs
    x_d = g.solve(b_d)
    x_h = g.solve(c["b"])
    np.testing.assert_array_equal(x_d.cpu().numpy().T, x_h)


def test_state_errors():
    c = I.small_case(1024, depth=2)
    g = A.System(c["pts"], c["kernel"], c["tol"], 64, 2)
    with pytest.raises(A.AifmmError) as e:
        g.solve(c["b"])
    assert e.value.status == 4
    g.factor()
    with pytest.raises(A.AifmmError) as e:
        g.factor()
    assert e.value.status == 4


def test_singular_self_block_reports_box():
    """Duplicated points with zero diagonal shift make a leaf self-block exactly singular."""
    rng = np.random.default_rng(36)
    p = rng.uniform(-1, 1, (512, 2))
    pts = np.ascontiguousarray(np.vstack([p, p]))
    g = A.System(pts, ("exp", 1.0, 0.0), 1e-8, 64, 2)
    with pytest.raises(A.AifmmError) as e:
        g.factor()
    assert e.value.status == 3
    assert "box" in str(e.value)
