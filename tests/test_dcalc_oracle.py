"""Pins of the d-calculation oracle (oracle/dcalc.py) -- Sec. III,
"Notation and definitions": closed forms on lattices, a pure-Python
recomputation by sorting, the running minimum / maximum over time, and the
reading the device relies on (the N nearest neighbours of a point are found
by a best-first search along the edges of DT*), checked against the brute
force on the CPU oracle's triangulations."""
import heapq
import math

import numpy as np
import pytest

from oracle import dt_star
from oracle.dcalc import NONE, DTracker, block_values, dcalc
from paper_2308_06484_amd import workloads as W


def test_lattice_closed_forms():
    g = np.array([(x, y) for y in range(5) for x in range(5)])
    # an interior point has 4 neighbours at 1, 4 at sqrt 2, 4 at 2
    assert [block_values(g, N)[0] for N in (1, 4, 5, 8, 9, 12)] == [1, 1, 2, 2, 4, 4]
    assert block_values(g, 1)[1] == 32  # diameter of the 5x5 lattice: 4 sqrt 2
    # a 2 x 3 lattice scaled by 7: the best point (the middle of a long side)
    # has 3 neighbours at 7, then two at 7 sqrt 2
    r = np.array([(7 * x, 7 * y) for y in range(2) for x in range(3)])
    assert [block_values(r, N)[0] for N in (1, 3, 4, 5)] == [49, 49, 98, 98]
    assert block_values(r, 5)[1] == 14 ** 2 + 7 ** 2
    assert block_values(r, 6)[0] == NONE  # only 5 other points


def test_against_sorting_in_python():
    rng = np.random.default_rng(1)
    for trial in range(40):
        n = int(rng.integers(2, 30))
        pts = np.unique(rng.integers(0, 20, size=(n, 2)), axis=0)
        for N in (1, 2, 3, 6):
            want = NONE
            for i, (x, y) in enumerate(pts.tolist()):
                d = sorted((x - u) ** 2 + (y - v) ** 2 for j, (u, v) in enumerate(pts.tolist()) if j != i)
                if len(d) >= N:
                    want = min(want, d[N - 1])
            diam = max((a - c) ** 2 + (b - e) ** 2 for a, b in pts.tolist() for c, e in pts.tolist())
            assert block_values(pts, N) == (want, diam), (trial, N)


def test_tracker_keeps_running_min_and_max():
    T = DTracker(2)
    d2, sp = T.update(np.array([9, 16]), np.array([100, 400]), 9)
    assert d2 == 9 and sp.tolist() == [math.sqrt(100 / 9), math.sqrt(400 / 9)]
    d2, sp = T.update(np.array([25, 16]), np.array([900, 100]), 16)
    assert d2 == 9 and sp.tolist() == [math.sqrt(900 / 16), math.sqrt(400 / 9)]
    xy = np.array([(0, 0), (3, 0), (0, 4), (10, 10), (11, 10), (10, 11)])
    m, d, g = dcalc(xy, np.array([0, 3, 6]), 1)
    assert m.tolist() == [9, 1] and d.tolist() == [25, 2] and g == 1


def _neighbours(tris):
    nb = {}
    for a, b, c in tris.tolist():
        for u, v in ((a, b), (b, c), (c, a)):
            nb.setdefault(u, set()).add(v)
            nb.setdefault(v, set()).add(u)
    return nb


def best_first_nth(p, N, xy, nb):
    """The device's search: take the closest candidate not taken yet, add
    its DT neighbours; the N-th taken is the N-th nearest neighbour."""
    d2 = lambda u: int((xy[u, 0] - xy[p, 0]) ** 2 + (xy[u, 1] - xy[p, 1]) ** 2)
    seen = {p}
    heap = []
    for u in nb[p]:
        seen.add(u)
        heapq.heappush(heap, (d2(u), u))
    last = None
    for _ in range(N):
        last, v = heapq.heappop(heap)
        for u in nb[v]:
            if u not in seen:
                seen.add(u)
                heapq.heappush(heap, (d2(u), u))
    return last


@pytest.mark.parametrize("kind", ["uniform", "lattice", "mixture"])
def test_delaunay_best_first_search_finds_the_nth_neighbour(kind):
    rng = np.random.default_rng({"uniform": 2, "lattice": 3, "mixture": 4}[kind])
    for trial in range(6):
        if kind == "uniform":
            xy = W._distinct_uniform(rng, 300, 0, 0, 2000, 2000)
        elif kind == "lattice":  # cocircular everywhere: ties decided by DT*
            full = np.array([(x, y) for y in range(16) for x in range(16)])
            xy = full[rng.permutation(len(full))[:180]]
        else:
            xy = W._distinct_gmm(rng, 300, 0, 4096)
        xy = np.asarray(xy, np.int64)
        nb = _neighbours(dt_star(xy))
        for N in (1, 2, 4, 8):
            got = min(best_first_nth(p, N, xy, nb) for p in range(len(xy)))
            assert got == block_values(xy, N)[0], (kind, trial, N)
