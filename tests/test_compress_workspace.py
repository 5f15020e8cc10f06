"""Host replay of the compression kernel's workspace use (k_compress, team routines).

The kernel carves one workspace per compression (22 cap^2 + 10 cap + 16 entries, cap = largest
box size of the level) into named regions, runs the two chains of pivoted QRs of a compression
either on two half-teams at once or one after the other on one workgroup, and keeps results in
regions across later phases.  This replay restates that layout and the order of the kernel's
phases (which region each phase writes, and which earlier phase produced each region it reads)
and checks, for every capacity the workloads reach (95 to 949 at N=262144, 2D) and beyond:
- every region lies inside the workspace and no two regions overlap;
- in the one-workgroup order, every region a phase reads still holds what its producer wrote
  (no later phase overwrote it in between): this is the check that fails when a chain's column
  storage is placed on a region that still holds a finished block;
- on split teams, the two halves never touch the same region between two joins;
- the exchange slots, barrier counters and publication slots of every team size up to 128
  members stay inside their allocations, and the host's team shapes keep LDS within the
  kernel's limit and teams co-resident, with the register tier covering every row;
- the 16-lane groups of the column passes cover the rows s..m-1 of a column exactly once, for
  the batch depths used (16) and others (4, 48).
"""
import itertools

import pytest

# ---- workspace regions (entries of the compression's precision), as the kernel lays them out
def regions(cap):
    c2 = cap * cap
    r = {}
    o = 0
    for name, size in [("Lb_i", c2), ("Rb_i", c2), ("Lb_j", c2), ("Rb_j", c2), ("M", 2 * c2),
                       ("V1", c2), ("V2", c2), ("V3", c2), ("V4", c2),
                       ("nU", c2), ("nV", c2), ("nUj", c2), ("nVj", c2),
                       ("t1", 2 * c2), ("t2", c2), ("tau", 4 * cap), ("nrm", 2 * cap),
                       ("Mb", 2 * c2), ("t1b", 2 * c2), ("nrmb", 2 * cap)]:
        r[name] = (o, o + size)
        o += size
    return r, 22 * c2 + 10 * cap + 16


@pytest.mark.parametrize("cap", list(range(1, 40)) + list(range(95, 950, 17)) + [949, 1024, 2048])
def test_regions_inside_and_disjoint(cap):
    r, wsz = regions(cap)
    spans = sorted(r.values())
    assert spans[-1][1] <= wsz
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert a1 <= b0
    # the largest uses: M holds ni x (ki + nj) <= cap x 2cap; a chain's column storage holds
    # n columns of m rows (n <= 2 cap, m <= cap); the new bases cap x cap with ld cap
    assert r["M"][1] - r["M"][0] >= cap * 2 * cap
    for g in ("t1", "t1b"):
        assert r[g][1] - r[g][0] >= 2 * cap * cap


# ---- phases of one compression: (half, name, writes, {region read: producing phase})
# half "A" / "B": the chain; "T": the whole team (after a join).  "S" is the slab (inputs).
def phases(kind, split):
    gcB = "t1b" if split else "t1"    # P2P: chain B's column storage
    McB = "Mb" if split else "M"
    ncB = "nrmb" if split else "nrm"
    u1, u2 = ("t1b", "Mb") if split else ("t1", "t2")
    if kind == "p2p":
        seg1 = [
            ("A", "copy_in1", {"M"}, {}),
            ("A", "rrqr1", {"t1", "nrm", "V1", "tau"}, {"M": "copy_in1"}),
            ("A", "formq1", {"t1", "nU"}, {"V1": "rrqr1", "tau": "rrqr1"}),
            ("A", "in3", {"M"}, {"nU": "formq1"}),
            ("A", "rrqr3", {"t1", "nrm", "V3", "tau"}, {"M": "in3"}),
            ("B", "copy_in2", {McB}, {}),
            ("B", "rrqr2", {gcB, ncB, "V2", "tau"}, {McB: "copy_in2"}),
            ("B", "formq2", {gcB, "nUj"}, {"V2": "rrqr2", "tau": "rrqr2"}),
            ("B", "in4", {McB}, {"nUj": "formq2"}),
            ("B", "rrqr4", {gcB, ncB, "V4", "tau"}, {McB: "in4"}),
        ]
        seg2 = [
            ("A", "bases_i", {"t1", "nU", "nV", "Lb_i", "Rb_i"},
             {"V1": "rrqr1", "V4": "rrqr4", "nU": "formq1"}),
            ("B", "bases_j", {gcB, "nUj", "nVj", "Lb_j", "Rb_j"},
             {"V2": "rrqr2", "V3": "rrqr3", "nUj": "formq2"}),
        ]
        seg3 = [
            ("A", "pair_ij", {"t1", "t2", "S"}, {"nU": "bases_i", "nVj": "bases_j", "Lb_i": "bases_i",
                                                 "Rb_j": "bases_j"}),
            ("B", "pair_ji", {u1, u2, "S"}, {"nUj": "bases_j", "nV": "bases_i", "Lb_j": "bases_j",
                                             "Rb_i": "bases_i"}),
        ]
        seg4 = [("T", "commit", {"S"}, {"nU": "bases_i", "nV": "bases_i", "nUj": "bases_j", "nVj": "bases_j"})]
        return [seg1, seg2, seg3, seg4]
    # P2L pair (r eliminated, i): chain A [V_i | P2L^*], chain B [U_i | M2P]
    seg1 = [
        ("A", "in5", {"M"}, {}),
        ("A", "rrqr5", {"t1", "nrm", "V1", "tau"}, {"M": "in5"}),
        ("B", "in6", {McB}, {}),
        ("B", "rrqr6", {"t1b", ncB, "V2", "tau"}, {McB: "in6"}),
    ]
    seg2 = [
        ("A", "side_v", {"t1", "nV", "Rb_i"}, {"V1": "rrqr5"}),          # t1 ends holding the new A_ri
        ("B", "side_u", {"t1b", "nU", "Lb_i", "t2"}, {"V2": "rrqr6"}),  # t2 ends holding the new A_ir
    ]
    seg3 = [("T", "commit", {"S"}, {"t1": "side_v", "t2": "side_u", "nU": "side_u", "nV": "side_v"})]
    return [seg1, seg2, seg3]


def _check(kind, split):
    segs = phases(kind, split)
    last = {}  # region -> phase that wrote it last
    for seg in segs:
        if split:
            halves = {h: [p for p in seg if p[0] == h] for h in "ABT"}
            touched = {h: set().union(*[p[2] | set(p[3]) for p in halves[h]]) if halves[h] else set()
                       for h in "AB"}
            shared = (touched["A"] & touched["B"]) - {"S", "tau"}
            assert not shared, f"{kind}: both halves touch {shared} between two joins"
            order = halves["A"] + halves["B"] + halves["T"]
            # reads see the state at the segment start plus the reader's own half's writes
            start = dict(last)
            own = {"A": {}, "B": {}, "T": {}}
            for h, name, wr, rd in order:
                for reg, prod in rd.items():
                    src = own[h].get(reg, start.get(reg))
                    assert src == prod, f"{kind} split: {name} reads {reg} from {src}, expected {prod}"
                for reg in wr:
                    own[h][reg] = name
            for h in "ABT":
                last.update(own[h])
        else:
            for h, name, wr, rd in seg:  # one workgroup: chain A, then chain B, in program order
                for reg, prod in rd.items():
                    assert last.get(reg) == prod, f"{kind}: {name} reads {reg} last written by {last.get(reg)}, " \
                                                  f"expected {prod}"
                for reg in wr:
                    last[reg] = name


@pytest.mark.parametrize("kind,split", list(itertools.product(["p2p", "p2l"], [False, True])))
def test_phase_dataflow(kind, split):
    _check(kind, split)


def test_dataflow_check_catches_clobbered_block():
    """Planting the defect this replay guards against: chain B's Q formation on t1 in the
    one-workgroup P2L order overwrites the new A_ri before it is committed."""
    orig = phases

    def planted(kind, split):
        segs = orig(kind, split)
        if kind == "p2l" and not split:
            h, n, w, r = segs[1][1]
            segs[1][1] = (h, n, (w - {"t1b"}) | {"t1"}, r)
        return segs

    globals()["phases"] = planted
    try:
        with pytest.raises(AssertionError):
            _check("p2l", False)
    finally:
        globals()["phases"] = orig


# ---- team exchange slots, counters and publication slots
CAND_STRIDE, CTR_STRIDE = 8, 64   # exchange slots 8 entries (192 bytes) apart, counters 64 words


def reg_rows(cap):
    """Rows a lane of the register column tier holds (16 lanes a column), 0 beyond 1024 rows."""
    for r in (16, 32, 40, 64):
        if 16 * r >= cap:
            return r
    return 0


def reg_slots(rmax, rs):
    """Register slots a 16-lane group holds: 64 FP64 values a lane, FP32 at most 4 slots."""
    if rmax == 0:
        return 0
    return max(1, 64 // rmax) if rs == 8 else min(4, 128 // rmax)


@pytest.mark.parametrize("G", list(range(1, 129)))
@pytest.mark.parametrize("cap", [95, 262, 610, 949, 958, 1024, 1500])
def test_team_slots_inside(G, cap):
    GMAX, maxcol = 128, 7
    GA = G // 2
    vlen = max(cap, 16 * reg_rows(cap))    # reflector and publication-slot length
    for e in range(maxcol):
        # whole team: 2 G exchange slots; halves: 2 GA and 2 (G - GA) after them; member q of
        # slot t at (t G + q) CAND_STRIDE
        lo, hi = e * 4 * G, e * 4 * G + 2 * G
        if G > 1:
            hiA = e * 4 * G + 2 * G + 2 * GA
            hiB = hiA + 2 * (G - GA)
            hi = max(hi, hiB)
        assert 0 <= lo and hi * CAND_STRIDE <= maxcol * 4 * GMAX * CAND_STRIDE
        # counters: the team's at e, the halves' at nent + 2 e (+1), CTR_STRIDE words apart
        assert (max(e, maxcol + 2 * e + 1) + 1) * CTR_STRIDE <= 3 * maxcol * CTR_STRIDE
        # publication: 2 G vlen per compression, half B's slots after half A's 2 GA vlen; a
        # slot of a half-team of g members written at ((s & 1) g + member) PS .. + PS - 1 with
        # PS = 16 RMAX (register tier) or m <= cap, both <= vlen
        for g, base in ((GA, e * 2 * G * vlen), (G - GA, e * 2 * G * vlen + 2 * GA * vlen)):
            if g == 0:
                continue
            PS = 16 * reg_rows(cap) if reg_rows(cap) else cap
            assert PS <= vlen
            top = base + (2 * g - 1) * PS + PS  # odd step, last member
            assert top <= e * 2 * G * vlen + 2 * G * vlen <= maxcol * 2 * GMAX * vlen


@pytest.mark.parametrize("rs", [8, 4])
@pytest.mark.parametrize("cap", list(range(1, 2049, 37)) + [95, 256, 257, 262, 512, 610, 640, 641, 958, 1024, 1025, 2048])
def test_register_tier_and_team_shape(cap, rs):
    """The host's team shape: LDS within the kernel's limit, teams co-resident, every column of
    a pivoted QR (n <= 2 cap) held in registers, LDS or the workspace region, and the register
    tier's rows (lane q: q, q + 16, ..) covering every row m <= cap."""
    CT, GMAX, lds_max, coop = 512, 128, 152 * 1024, 256
    rmax = reg_rows(cap)
    if rmax:
        assert 16 * rmax >= cap
        assert sorted(q + 16 * u for q in range(16) for u in range(rmax))[:cap] == list(range(cap))
    nreg = (CT // 16) * reg_slots(rmax, rs)
    vlen = max(cap, 16 * rmax)
    base = vlen * rs + 4 * cap * 4 + 2 * cap * rs
    if base > lds_max:
        return  # the library reports AIFMM_ERR_CAPACITY
    colb = (cap | 1) * rs
    ldsc = (lds_max - base) // colb
    for ne in (1, 2, 8, 37, 157, 300):
        need = 2 * cap
        h = max(1, min(-(-need // max(1, nreg + ldsc)), 64, GMAX // 2))
        G = 1
        if ne * 2 <= coop:
            G = 2 * min(h, coop // (2 * ne))
        share = -(-need // (G // 2)) if G > 1 else need
        lcols = min(ldsc, max(0, share - nreg))
        # the same LDS region stages the register Q formation's 8 reflectors of 16 RMAX entries
        shm = base + max(lcols * colb, 8 * 16 * rmax * rs)
        assert shm <= lds_max
        assert G == 1 or (G % 2 == 0 and 2 <= G <= GMAX and ne * G <= coop)
        # a member's columns: registers, then LDS, then the workspace (column c at c m of a
        # 2 cap^2 region, c < n <= 2 cap, m <= cap)
        assert share <= nreg + lcols + max(0, share - nreg - lcols)
        assert (2 * cap - 1) * cap + cap <= 2 * cap * cap


# ---- the 16-lane groups of the column passes
@pytest.mark.parametrize("batch", [4, 16, 48])
def test_column_pass_rows_once(batch):
    PL = 16
    for m in list(range(1, 70)) + [949]:
        for s in range(0, min(m, 40)):
            seen = []
            for lane in range(PL):
                r0 = s + ((lane - s) & (PL - 1))
                for i0 in range(r0, m, PL * batch):
                    for u in range(batch):
                        i = i0 + PL * u
                        if i < m:
                            assert i % PL == lane % PL  # chain = row mod 16, the fixed summation order
                            seen.append(i)
            assert sorted(seen) == list(range(s, m))
