"""Pins of the oracle's tree, lists and elimination order (Sec. 2.1-2.2).

- Closed-form pair counts on the uniform grid with s = 2^l boxes per side:
  (3s-2)^d ordered pairs at Chebyshev distance <= 1 (self included), and
  (5s-6)^d - (3s-2)^d at distance exactly 2.
- The interaction list equals the brute-force geometric definition with eta = sqrt(d)
  (max diam <= eta * dist on the actual box geometry) restricted to children of the
  parent's neighbours, for every box at levels 2..4.
- Depth rule and box point counts; the colour order puts equal colours >= 5 apart.
"""
import itertools

import numpy as np
import pytest

import aifmm_inputs as I
import oracle


def _box_dist(c1, c2, h):
    gap = np.maximum(np.abs(np.array(c1) - np.array(c2)) - 1, 0) * h
    return np.sqrt((gap ** 2).sum())


@pytest.mark.parametrize("d,L", [(2, 4), (3, 3)])
def test_lists_closed_forms_and_geometry(d, L):
    c = I.small_case(512 if d == 2 else 800, d=d, depth=L, kernel=("exp", 1.0, 0.1), tol=1e-4)
    s = oracle.System(c["pts"], c["kernel"], c["tol"], 64, L)
    for l in range(2, L + 1):
        side = 1 << l
        nb = side ** d
        coords = [tuple(((b >> (bit * d + t)) & 1) << bit for t in range(d)) for b in range(nb) for bit in range(l)]
        coords = []
        for b in range(nb):
            cc = [0] * d
            for bit in range(l):
                for t in range(d):
                    cc[t] |= ((b >> (bit * d + t)) & 1) << bit
            coords.append(tuple(cc))
        nn = 0
        h = 1.0 / side
        for b in range(nb):
            nbr, il = s.lists(l, b)
            nn += len(nbr)
            assert b in nbr
            assert len(nbr) <= 3 ** d and len(il) <= 6 ** d - 3 ** d
            parent = b >> d
            pn, _ = s.lists(l - 1, parent)
            cand = [(q << d) | ch for q in pn for ch in range(1 << d)]
            diam = np.sqrt(d) * h
            geo = sorted(q for q in cand
                         if diam <= np.sqrt(d) * _box_dist(coords[b], coords[q], h) * (1 + 1e-12))
            assert list(il) == geo
        assert nn == (3 * side - 2) ** d
        # distance-2 ordered pairs
        n2 = 0
        for a, b in itertools.product(range(nb), repeat=2):
            if max(abs(x - y) for x, y in zip(coords[a], coords[b])) == 2:
                n2 += 1
        assert n2 == (5 * side - 6) ** d - (3 * side - 2) ** d


def test_depth_rule_and_counts():
    c = I.small_case(4096, depth=0)
    s = oracle.System(c["pts"], c["kernel"], 1e-4, 64, 0)
    assert s.L == 3
    cnt = s.counts(3)
    assert cnt.sum() == 4096 and len(cnt) == 64
    for l in (2, 1, 0):
        up = s.counts(l)
        assert np.array_equal(up, cnt.reshape(-1, 4).sum(1))
        cnt = up
    assert s.counts(0)[0] == 4096
    # leaf membership by the hypercube rule (bounding-box midpoint, largest extent), recomputed
    # independently
    pts = c["pts"]
    lo, hi = pts.min(0), pts.max(0)
    side = (hi - lo).max()
    base = (lo + hi) * 0.5 - side * 0.5
    q = np.clip(np.floor((pts - base) / side * 8).astype(int), 0, 7)
    code = np.zeros(4096, int)
    for bit in range(3):
        for t in range(2):
            code |= ((q[:, t] >> bit) & 1) << (bit * 2 + t)
    perm = s.perm()
    assert np.array_equal(np.sort(perm), np.arange(4096))
    assert np.all(np.diff(code[perm]) >= 0)
    assert np.array_equal(np.bincount(code, minlength=64), s.counts(3))


def test_colour_order():
    c = I.small_case(4096, depth=4, tol=1e-3)
    s = oracle.System(c["pts"], c["kernel"], 1e-3, 64, 4)
    order = s.elim_order(4)
    assert sorted(order) == list(range(256))
    def coord(b):
        return ((b & 1) | ((b >> 2) & 1) << 1 | ((b >> 4) & 1) << 2 | ((b >> 6) & 1) << 3,
                ((b >> 1) & 1) | ((b >> 3) & 1) << 1 | ((b >> 5) & 1) << 2 | ((b >> 7) & 1) << 3)
    cols = [(coord(b)[0] % 5) * 5 + coord(b)[1] % 5 for b in order]
    assert cols == sorted(cols)
    for a in range(256):
        for b in range(a + 1, 256):
            if cols[a] == cols[b]:
                ca, cb = coord(order[a]), coord(order[b])
                assert max(abs(ca[0] - cb[0]), abs(ca[1] - cb[1])) >= 5
