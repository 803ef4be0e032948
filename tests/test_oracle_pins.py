"""Pins of the CPU oracle to things other than itself.

* predicates against geometry (Heron's area, exact circumcentres in
  rationals) and the tie rule against the sign of an epsilon-polynomial
  4x4 determinant expanded term by term;
* closed-form worked examples (tests/golden/);
* the Bowyer-Watson oracle against the O(n^4) empty-circle definition on
  small, highly degenerate lattice subsets with random id labelings;
* against scipy's Qhull on inputs in general position;
* invariants at larger sizes (certificate.py).
"""
import json
import math
import os
from fractions import Fraction
from itertools import combinations, permutations

import numpy as np
import pytest

import oracle
from oracle import definition as D
from tests import certificate

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ----------------------------------------------------------------- predicates

def _rand_pts(rng, k, lo=0, hi=1 << 24):
    return [(int(rng.integers(lo, hi)), int(rng.integers(lo, hi))) for _ in range(k)]


def test_orient_matches_heron_and_turn_direction():
    L = oracle.lib()
    rng = np.random.default_rng(1)
    for trial in range(3000):
        hi = 1 << (24 if trial % 3 else 6)
        a, b, c = _rand_pts(rng, 3, 0, hi)
        o = L.oracle_orient(*a, *b, *c)
        # Heron in squared side lengths: 16 A^2 = 4 p q - (p + q - r)^2, |orient| = 2A
        p = (b[0] - a[0]) ** 2 + (b[1] - a[1]) ** 2
        q = (c[0] - a[0]) ** 2 + (c[1] - a[1]) ** 2
        r = (c[0] - b[0]) ** 2 + (c[1] - b[1]) ** 2
        assert 4 * o * o == 4 * p * q - (p + q - r) ** 2
        if o != 0 and abs(o) > 1e-6 * max(p, q, r, 1):
            # turn direction from angles, independent of the determinant
            t1 = math.atan2(b[1] - a[1], b[0] - a[0])
            t2 = math.atan2(c[1] - a[1], c[0] - a[0])
            turn = (t2 - t1 + math.pi) % (2 * math.pi) - math.pi
            assert (turn > 0) == (o > 0)


def _circumcentre(a, b, c):
    ax, ay, bx, by, cx, cy = (Fraction(v) for v in (*a, *b, *c))
    d = 2 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
    ux = ((ax * ax + ay * ay) * (by - cy) + (bx * bx + by * by) * (cy - ay)
          + (cx * cx + cy * cy) * (ay - by)) / d
    uy = ((ax * ax + ay * ay) * (cx - bx) + (bx * bx + by * by) * (ax - cx)
          + (cx * cx + cy * cy) * (bx - ax)) / d
    return ux, uy


def _geom_incircle(a, b, c, d):
    """Sign of R^2 - |d - O|^2 (inside > 0) for counter-clockwise abc."""
    ux, uy = _circumcentre(a, b, c)
    r2 = (a[0] - ux) ** 2 + (a[1] - uy) ** 2
    d2 = (d[0] - ux) ** 2 + (d[1] - uy) ** 2
    return (r2 > d2) - (r2 < d2)


def test_incircle_matches_exact_circumcentre():
    L = oracle.lib()
    rng = np.random.default_rng(2)
    checked = 0
    while checked < 2000:
        hi = 1 << (24 if checked % 2 else 5)
        a, b, c, d = _rand_pts(rng, 4, 0, hi)
        o = D.orient(a, b, c)
        if o == 0:
            continue
        if o < 0:
            b, c = c, b
        g = _geom_incircle(a, b, c, d)
        assert L.oracle_incircle_sign(*a, *b, *c, *d) == g
        assert (D.incircle(a, b, c, d) > 0) - (D.incircle(a, b, c, d) < 0) == g
        checked += 1


def test_incircle_closed_forms():
    L = oracle.lib()
    # unit square: four cocircular corners
    assert L.oracle_incircle_sign(0, 0, 1, 0, 1, 1, 0, 1) == 0
    # (1,1) is the centre of the circle through (0,0), (2,0), (0,2)
    assert L.oracle_incircle_sign(0, 0, 2, 0, 0, 2, 1, 1) == 1
    assert L.oracle_incircle_sign(0, 0, 2, 0, 0, 2, 3, 3) == -1
    # Pythagorean points on the circle of radius 5 about (7, 9)
    on = [(7 + 3, 9 + 4), (7 - 4, 9 + 3), (7 - 5, 9), (7, 9 - 5), (7 + 4, 9 - 3)]
    for d in on[3:]:
        assert L.oracle_incircle_sign(*on[0], *on[1], *on[2], *d) == 0
    # coordinate extremes: the largest magnitudes the input range allows
    M = (1 << 24) - 1
    assert L.oracle_incircle_sign(0, 0, M, 0, 0, M, M, M) == 0
    assert L.oracle_incircle_sign(0, 0, M, 0, 0, M, M - 1, M - 1) == 1
    assert L.oracle_incircle_sign(0, 0, M, 0, 0, M, M, M - 1) == 1
    assert L.oracle_orient(0, 0, M, 0, 0, M) == M * M


def _det(m):
    """Determinant by Leibniz expansion; entries are polynomials in eps given
    as {exponent: coefficient} dicts."""
    n = len(m)
    total = {}
    for perm in permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        term = {0: -1 if inv % 2 else 1}
        for r in range(n):
            e = m[r][perm[r]]
            nt = {}
            for k1, v1 in term.items():
                for k2, v2 in e.items():
                    nt[k1 + k2] = nt.get(k1 + k2, 0) + v1 * v2
            term = nt
        for k, v in term.items():
            total[k] = total.get(k, 0) + v
    return total


def _eps_sign(a, b, c, d, ids):
    """Sign, as eps -> 0+, of det rows (x, y, x^2 + y^2 + eps^(K - id), 1):
    the larger the id the larger the lift."""
    K = max(ids) + 1
    rows = []
    for p, i in zip((a, b, c, d), ids):
        rows.append([{0: p[0]}, {0: p[1]}, {0: p[0] ** 2 + p[1] ** 2, K - i: 1}, {0: 1}])
    poly = _det(rows)
    for k in sorted(poly):
        if poly[k]:
            return (poly[k] > 0) - (poly[k] < 0)
    return 0


def test_tie_rule_matches_epsilon_determinant():
    L = oracle.lib()
    rng = np.random.default_rng(3)
    # cocircular quadruples on small lattices (squares, rectangles, kites),
    # plus general quadruples where the exact sign decides
    quads = []
    for _ in range(600):
        pts = _rand_pts(rng, 4, 0, 4)
        if len(set(pts)) == 4:
            quads.append(pts)
    cocirc = 0
    for a, b, c, d in quads:
        o = D.orient(a, b, c)
        if o == 0:
            continue
        if o < 0:
            b, c = c, b
        for ids in ([0, 1, 2, 3], [3, 2, 1, 0], list(rng.permutation(4))):
            ids = [int(i) for i in ids]
            want = _eps_sign(a, b, c, d, ids)
            assert want != 0
            got = L.oracle_incircle_star(*a, ids[0], *b, ids[1], *c, ids[2], *d, ids[3])
            assert got == want, (a, b, c, d, ids)
            assert D.incircle_star(a, b, c, d, *ids) == want
            cocirc += D.incircle(a, b, c, d) == 0
    assert cocirc > 50  # the degenerate branch was exercised


def test_ghost_rule_closed_forms():
    L = oracle.lib()
    # hull edge b->a = (2,0)->(0,0); ghost (a,b,inf) = ((0,0),(2,0)) is the
    # half-plane y > 0 plus the open segment
    assert L.oracle_ghost_conflict(0, 0, 2, 0, 1, 5) == 1
    assert L.oracle_ghost_conflict(0, 0, 2, 0, 1, -5) == 0
    assert L.oracle_ghost_conflict(0, 0, 2, 0, 1, 0) == 1   # strictly inside the segment
    assert L.oracle_ghost_conflict(0, 0, 2, 0, 3, 0) == 0   # on the line, beyond b
    assert L.oracle_ghost_conflict(0, 0, 2, 0, -1, 0) == 0  # on the line, before a


# ---------------------------------------------------------- worked examples

@pytest.mark.parametrize("name", ["unit_square.json", "grid3x3.json"])
def test_golden_examples(name):
    g = json.load(open(os.path.join(HERE, "golden", name)))
    want = [tuple(t) for t in g["dt"]]
    assert [tuple(t) for t in oracle.dt_star(g["xy"], g["ids"]).tolist()] == want
    assert D.dt_star_bf(g["xy"], g["ids"]) == want


# ------------------------------------------------ oracle vs the definition

def test_oracle_equals_definition_on_degenerate_lattice_subsets():
    rng = np.random.default_rng(4)
    done = 0
    for trial in range(1500):
        w = (4, 5, 8)[trial % 3]
        n = int(rng.integers(3, 13))
        cells = rng.choice(w * w, size=n, replace=False)
        xy = np.stack([cells % w, cells // w], 1).astype(np.int32)
        ids = rng.permutation(n).astype(np.int64) * 7 + 3
        bf = D.dt_star_bf(xy, ids)
        if not bf:
            with pytest.raises(oracle.OracleError):
                oracle.dt_star(xy, ids)
            continue
        got = [tuple(t) for t in oracle.dt_star(xy, ids).tolist()]
        assert got == bf, (xy.tolist(), ids.tolist())
        done += 1
    assert done > 1300


def test_every_subset_of_3x3_grid_all_labelings_of_4():
    """Exhaustive over the 3x3 lattice: all 2^9 subsets, 3 labelings each."""
    pts = [(x, y) for y in range(3) for x in range(3)]
    rng = np.random.default_rng(5)
    for mask in range(1, 1 << 9):
        sub = [pts[i] for i in range(9) if mask >> i & 1]
        if len(sub) < 3:
            continue
        for lab in range(3):
            ids = list(range(len(sub))) if lab == 0 else [int(v) for v in rng.permutation(len(sub))]
            bf = D.dt_star_bf(sub, ids)
            if not bf:
                continue
            got = [tuple(t) for t in oracle.dt_star(sub, ids).tolist()]
            assert got == bf


def test_oracle_equals_qhull_in_general_position():
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(6)
    for trial in range(20):
        n = int(rng.integers(10, 400))
        xy = np.unique(rng.integers(0, 1 << 24, size=(n, 2)), axis=0).astype(np.int32)
        rng.shuffle(xy)
        tri = Delaunay(xy.astype(np.float64)).simplices
        P = [(int(x), int(y)) for x, y in xy]
        ref = []
        for a, b, c in tri:
            if D.orient(P[a], P[b], P[c]) < 0:
                b, c = c, b
            ref.append((int(a), int(b), int(c)))
        got = [tuple(t) for t in oracle.dt_star(xy).tolist()]
        assert got == D.canonical(ref)


# ------------------------------------------------------------- invariants

@pytest.mark.parametrize("seed,n,side", [(7, 300, 32), (8, 1500, 64), (9, 1024, 2048)])
def test_oracle_certificate_dense_lattice(seed, n, side):
    rng = np.random.default_rng(seed)
    cells = rng.choice(side * side, size=n, replace=False)
    xy = np.stack([cells % side, cells // side], 1).astype(np.int32)
    ids = rng.permutation(n).astype(np.int64)
    certificate.check(xy, ids, oracle.dt_star(xy, ids))


def test_oracle_collinear_hull_and_full_lattice():
    # a full 12x12 lattice: every hull point collinear with its neighbours,
    # every cell cocircular
    xy = np.array([(x, y) for y in range(12) for x in range(12)], np.int32)
    t = oracle.dt_star(xy)
    assert len(t) == 2 * 144 - 2 - 44
    certificate.check(xy, np.arange(144), t)


def test_oracle_errors():
    with pytest.raises(oracle.OracleError) as e:
        oracle.dt_star([[0, 0], [1, 1], [0, 0], [3, 1]])
    assert e.value.code == -3
    with pytest.raises(oracle.OracleError) as e:
        oracle.dt_star([[0, 0], [1, 1], [2, 2], [3, 3]])
    assert e.value.code == -4
    with pytest.raises(oracle.OracleError) as e:
        oracle.dt_star([[0, 0], [1, 1]])
    assert e.value.code == -4
    with pytest.raises(oracle.OracleError) as e:
        oracle.dt_star([[0, 0], [1, 1], [1 << 24, 0]])
    assert e.value.code == -2


def test_certificate_rejects_planted_mistakes():
    """The certificate itself must catch a wrong triangulation: flip one
    interior edge of a correct answer, or drop a triangle."""
    xy = np.array([(x, y) for y in range(5) for x in range(5)], np.int32)
    good = oracle.dt_star(xy)
    certificate.check(xy, np.arange(25), good)
    # flip the diagonal of the unit cell at the origin: (0,1,5),(1,6,5) -> (0,1,6),(0,6,5)
    bad = [tuple(t) for t in good.tolist() if tuple(t) not in {(0, 1, 5), (1, 6, 5)}]
    bad += [(0, 1, 6), (0, 6, 5)]
    with pytest.raises(AssertionError):
        certificate.check(xy, np.arange(25), bad)
    with pytest.raises(AssertionError):
        certificate.check(xy, np.arange(25), good[1:])


def test_every_subset_of_4x4_lattice_three_labelings():
    """Exhaustive over the 4 x 4 lattice: all 2^16 subsets of at least 3
    points, 3 labelings of the 16 points each.  The definition is evaluated
    once per labeling as a table -- for every counter-clockwise triple of
    lattice points, the set of other lattice points its perturbed circle
    holds -- so DT*(M) of a subset M is every triple inside M whose table
    set misses M.  All-collinear subsets have no triangulation: the oracle
    refuses them."""
    pts = [(x, y) for y in range(4) for x in range(4)]
    tri_ids = list(combinations(range(16), 3))
    masks = np.arange(1 << 16, dtype=np.int64)
    popc = np.array([bin(m).count("1") for m in range(1 << 16)])
    rng = np.random.default_rng(44)
    checked = 0
    for lab in range(3):
        label = np.arange(16) if lab == 0 else rng.permutation(16) * 5 + 2
        ccw, bits, bad, canon = [], [], [], []
        for i, j, k in tri_ids:
            o = D.orient(pts[i], pts[j], pts[k])
            if o == 0:
                continue
            if o < 0:
                j, k = k, j
            m = 0
            for d in range(16):
                if d in (i, j, k):
                    continue
                if D.incircle_star(pts[i], pts[j], pts[k], pts[d], label[i], label[j], label[k], label[d]) > 0:
                    m |= 1 << d
            ccw.append((i, j, k))
            bits.append((1 << i) | (1 << j) | (1 << k))
            bad.append(m)
            canon.append(D.canonical([(int(label[i]), int(label[j]), int(label[k]))])[0])
        bits, bad = np.array(bits, np.int64), np.array(bad, np.int64)
        inside = ((bits[None, :] & ~masks[:, None]) == 0) & ((bad[None, :] & masks[:, None]) == 0)
        for mask in range(1 << 16):
            if popc[mask] < 3:
                continue
            idx = [i for i in range(16) if mask >> i & 1]
            sub = [pts[i] for i in idx]
            ids = [int(label[i]) for i in idx]
            want = sorted(canon[t] for t in np.nonzero(inside[mask])[0])
            if not want:  # every point on one line
                with pytest.raises(oracle.OracleError):
                    oracle.dt_star(sub, ids)
                continue
            got = [tuple(t) for t in oracle.dt_star(sub, ids).tolist()]
            assert got == want, (lab, mask)
            checked += 1
    assert checked > 3 * 65000
