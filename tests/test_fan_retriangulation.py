"""The fan test of the star-only retriangulation, checked against the oracle
on the CPU (no GPU): when no triangle outside p's star is destroyed by the
new place q, DT*(S - p + q) is DT*(S) with p's star replaced by the fan
(q_s, q_s+1, q) exactly when q lies strictly left of every link edge and no
link vertex lies inside the perturbed circle of any fan triangle.  Dense
small lattices make exact cocircular ties common, so the id perturbation is
exercised.  Also the order in which the fan's triangles are listed: the
order of the candidate search (pairs (i < j) by j, then i)."""
import numpy as np
import pytest

import oracle
from oracle.definition import incircle_star, orient


def _tris(xy):
    t = oracle.dt_star(xy)
    return {tuple(int(v) for v in r) for r in t if min(r) >= 0}


def _canon(t):
    k = min(range(3), key=lambda i: t[i])
    return (t[k], t[(k + 1) % 3], t[(k + 2) % 3])


def _link(tris, p):
    """Counter-clockwise link of an interior vertex p, or None on the hull."""
    nxt = {}
    for t in tris:
        if p in t:
            i = t.index(p)
            nxt[t[(i + 1) % 3]] = t[(i + 2) % 3]
    if not nxt or set(nxt) != set(nxt.values()):
        return None
    a0 = next(iter(nxt))
    out, a = [a0], nxt[a0]
    while a != a0:
        out.append(a)
        a = nxt[a]
    return out if len(out) == len(nxt) else None


def _fan_holds(xy, link, p, q):
    k = len(link)
    for s in range(k):
        a, b = link[s], link[(s + 1) % k]
        if orient(xy[a], xy[b], q) <= 0:
            return False
        for m in link:
            if m in (a, b):
                continue
            if incircle_star(xy[a], xy[b], q, xy[m], a, b, p, m) >= 0:
                return False
    return True


@pytest.mark.parametrize("seed,n,side", [(1, 70, 24), (2, 90, 40), (3, 60, 1000)])
def test_fan_is_the_retriangulation_exactly_when_the_test_passes(seed, n, side):
    rng = np.random.default_rng(seed)
    cells = rng.choice(side * side, size=n, replace=False)
    xy = np.stack([cells % side, cells // side], axis=1).astype(np.int64)
    T = _tris(xy)
    P = [tuple(v) for v in xy.tolist()]  # Python ints for the exact predicates
    taken = set(P)
    checked = held = 0
    for p in range(n):
        link = _link(T, p)
        if link is None:
            continue
        star = {t for t in T if p in t}
        for _ in range(6):
            d = rng.integers(-4, 5, size=2)
            q = (int(xy[p, 0] + d[0]), int(xy[p, 1] + d[1]))
            if q in taken or not (0 <= q[0] < side and 0 <= q[1] < side):
                continue
            # only moves whose region is the star: no outside triangle destroyed
            if any(incircle_star(P[t[0]], P[t[1]], P[t[2]], q, t[0], t[1], t[2], p) > 0
                   for t in T - star):
                continue
            xy2 = xy.copy()
            xy2[p] = q
            got = _tris(xy2)
            fan = {_canon((link[s], link[(s + 1) % len(link)], p)) for s in range(len(link))}
            is_fan = got == (T - star) | fan
            assert is_fan == _fan_holds(P, link, p, q), (seed, p, q)
            checked += 1
            held += is_fan
    # both outcomes occur on every set
    assert checked >= 20 and 0 < held < checked, (checked, held)


def _search_order(k):
    """Fan triangles in the order the candidate search meets them: the pairs
    (i < j) in colex order, each kept when it is a link edge, the pair
    (0, k-1) turned counter-clockwise as (k-1, 0)."""
    out = []
    for j in range(1, k):
        for i in range(j):
            if j == i + 1:
                out.append((i, j))
            elif i == 0 and j == k - 1:
                out.append((k - 1, 0))
    return out


@pytest.mark.parametrize("k", range(3, 16))
def test_fan_listing_order(k):
    # the listing the library uses: t_s at s (s < k-2), t_k-1 at k-2, t_k-2 at k-1
    listed = [(s, (s + 1) % k) for s in
              [h if h < k - 2 else (k - 1 if h == k - 2 else k - 2) for h in range(k)]]
    assert listed == _search_order(k)
