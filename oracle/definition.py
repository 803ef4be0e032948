"""DT*(S) straight from its definition, in exact Python integers.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The Delaunay triangulation is the set of triangles whose circumcircle holds
no other point of the set (Sec. I).  On lattice input four or more points are
often cocircular, and the paper's uniqueness claim (Sec. I) then needs a rule
for points exactly on a circle: every point's paraboloid height is raised by
an infinitesimal that grows with its id.  This module writes that definition
out directly, O(n^4), for the small inputs that pin the Bowyer-Watson oracle.
"""
from __future__ import annotations

from itertools import combinations


def orient(a, b, c) -> int:
    """Twice the signed area of triangle abc (> 0: counter-clockwise)."""
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])


def incircle(a, b, c, d) -> int:
    """The 3x3 lifted determinant with rows (p - d, |p - d|^2) for p = a, b, c;
    for counter-clockwise abc it is > 0 iff d is strictly inside their circle."""
    rows = []
    for p in (a, b, c):
        dx, dy = p[0] - d[0], p[1] - d[1]
        rows.append((dx, dy, dx * dx + dy * dy))
    (a0, a1, a2), (b0, b1, b2), (c0, c1, c2) = rows
    return (a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0)
            + a2 * (b0 * c1 - b1 * c0))


def _sign(v: int) -> int:
    return (v > 0) - (v < 0)


def incircle_star(a, b, c, d, ia, ib, ic, id_) -> int:
    """Sign of the incircle test after lifting each point by an infinitesimal
    that increases with its id; ties go to the point with the largest id.

    Raising the lifted height of point m by delta changes the 4x4 determinant
    with rows (x, y, x^2 + y^2, 1) in the order a, b, c, d by delta times the
    cofactor of m's height entry; that cofactor is a 3x3 orientation of the
    other three points, with sign (-1)^(row + 3)."""
    s = _sign(incircle(a, b, c, d))
    if s:
        return s
    m = max((ia, 0), (ib, 1), (ic, 2), (id_, 3))[1]
    if m == 0:
        return _sign(orient(b, c, d))
    if m == 1:
        return -_sign(orient(a, c, d))
    if m == 2:
        return _sign(orient(a, b, d))
    return -_sign(orient(a, b, c))


def canonical(tris):
    """Rotate every triangle to start at its smallest id; sort the list."""
    out = []
    for t in tris:
        k = min(range(3), key=lambda i: t[i])
        out.append((t[k], t[(k + 1) % 3], t[(k + 2) % 3]))
    return sorted(out)


def dt_star_bf(pts, ids=None):
    """All counter-clockwise (a, b, c) with no other point d inside or on the
    perturbed circle, as a canonical list of id triples."""
    n = len(pts)
    ids = list(range(n)) if ids is None else [int(i) for i in ids]
    pts = [(int(p[0]), int(p[1])) for p in pts]
    tris = []
    for i, j, k in combinations(range(n), 3):
        o = orient(pts[i], pts[j], pts[k])
        if o == 0:
            continue
        if o < 0:
            j, k = k, j
        ok = True
        for m in range(n):
            if m in (i, j, k):
                continue
            if incircle_star(pts[i], pts[j], pts[k], pts[m], ids[i], ids[j], ids[k], ids[m]) >= 0:
                ok = False
                break
        if ok:
            tris.append((ids[i], ids[j], ids[k]))
    return canonical(tris)
