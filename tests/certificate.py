"""Independent checks of a triangulation, for tests only.

Given points and a list of counter-clockwise triangles (global ids) this
verifies, without any triangulation code, that the list is the Delaunay
triangulation DT* of the points:
  * every triangle is strictly counter-clockwise;
  * every directed edge is used at most once, so each undirected edge has at
    most two triangles, on opposite sides;
  * the edges used by one triangle only are exactly the edges of the convex
    hull, with collinear hull points kept as vertices (monotone chain below);
  * the triangle count is 2n - 2 - h (h = points on the hull boundary) and
    every point is a vertex, which with the two items above makes the list a
    triangulation of the hull;
  * every interior edge is locally Delaunay under the perturbed incircle
    test; for a (weighted) Delaunay lifting, locally convex everywhere means
    globally convex, so the triangulation is DT*.
"""
from __future__ import annotations

import numpy as np

from oracle.definition import incircle_star


def hull_edges(xy, ids):
    """Directed counter-clockwise hull edges (id pairs), every point on the
    hull boundary kept as a vertex (Andrew's monotone chain, collinear-
    inclusive)."""
    pts = sorted((int(x), int(y), int(i)) for (x, y), i in zip(xy, ids))

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) < 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) < 0:
            upper.pop()
        upper.append(p)
    ring = lower[:-1] + upper[:-1]
    # collinear-inclusive chains can repeat points when every point is on the hull
    seen, cyc = set(), []
    for p in ring:
        if p[2] not in seen:
            seen.add(p[2])
            cyc.append(p[2])
    return {(cyc[i], cyc[(i + 1) % len(cyc)]) for i in range(len(cyc))}


def check(xy, ids, tris):
    """Raise AssertionError unless `tris` is DT*(points)."""
    xy = np.asarray(xy, dtype=np.int64)
    ids = [int(i) for i in ids]
    pos = {i: (int(x), int(y)) for (x, y), i in zip(xy, ids)}
    tris = [tuple(int(v) for v in t) for t in np.asarray(tris).reshape(-1, 3)]
    n = len(ids)
    directed = {}
    used = set()
    for k, (a, b, c) in enumerate(tris):
        pa, pb, pc = pos[a], pos[b], pos[c]
        o = (pb[0] - pa[0]) * (pc[1] - pa[1]) - (pb[1] - pa[1]) * (pc[0] - pa[0])
        assert o > 0, f"triangle {(a, b, c)} not counter-clockwise"
        for u, v, w in ((a, b, c), (b, c, a), (c, a, b)):
            assert (u, v) not in directed, f"directed edge {(u, v)} used twice"
            directed[(u, v)] = w
        used.update((a, b, c))
    assert len(used) == n, f"{n - len(used)} points are not vertices"
    boundary = {e for e in directed if (e[1], e[0]) not in directed}
    hull = hull_edges(xy, ids)
    # a triangle edge with no twin is a hull edge traversed counter-clockwise
    assert boundary == hull, "boundary edges differ from the convex hull"
    h = len(hull)
    assert len(tris) == 2 * n - 2 - h, f"{len(tris)} triangles, expected {2 * n - 2 - h}"
    for (u, v), w in directed.items():
        if (v, u) in directed and u < v:
            x = directed[(v, u)]
            s = incircle_star(pos[u], pos[v], pos[w], pos[x], u, v, w, x)
            assert s < 0, f"edge {(u, v)} not locally Delaunay"
    return True
