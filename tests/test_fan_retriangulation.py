"""The fan test of the star-only retriangulation, checked against the oracle
on the CPU (no GPU): when no triangle outside p's star is destroyed by the
new place q, DT*(S - p + q) is DT*(S) with p's star replaced by the fan
(q_s, q_s+1, q) exactly when q lies strictly left of every link edge and no
link vertex lies inside the perturbed circle of any fan triangle.  Dense
small lattices make exact cocircular ties common, so the id perturbation is
exercised.  Also the order in which the fan's triangles are listed: the
order of the candidate search (pairs (i < j) by j, then i).  And, where q is
in the kernel of the star but the fan test fails, Lawson flips from the fan
(the library's fallback before the candidate search, restated here step by
step): they end on DT*(S - p + q) inside the star, listed in the search's
order."""
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


def _pack3(i, j, l):
    return (i << 16) | (j << 8) | l


def _lawson(P, ids, k, cap=32):
    """Flips from the fan over polygon 0..k-1 + q (index k); each triangle
    [v0, v1, v2, n0, n1, n2], n_e across the edge opposite v_e.  Returns the
    keys in candidate order, or None at the cap."""
    T = [[s, (s + 1) % k, k, (s + 1) % k, (s - 1) % k, -1] for s in range(k)]
    for it in range(cap + 1):
        hit = None
        for t in range(k):
            for e in range(3):
                u = T[t][3 + e]
                if u <= t:
                    continue
                c, a, b = T[t][e], T[t][(e + 1) % 3], T[t][(e + 2) % 3]
                d = next(v for v in T[u][:3] if v not in (a, b))
                if incircle_star(P[c], P[a], P[b], P[d], ids[c], ids[a], ids[b], ids[d]) > 0:
                    hit = (t, e)
                    break
            if hit:
                break
        if hit is None:
            break
        if it == cap:
            return None
        t, e = hit
        c, a, b = T[t][e], T[t][(e + 1) % 3], T[t][(e + 2) % 3]
        n_bc, n_ca, u = T[t][3 + (e + 1) % 3], T[t][3 + (e + 2) % 3], T[t][3 + e]
        f = next(i for i in range(3) if T[u][i] not in (a, b))
        d, n_ad, n_db = T[u][f], T[u][3 + (f + 1) % 3], T[u][3 + (f + 2) % 3]
        T[t] = [c, a, d, n_ad, u, n_ca]
        T[u] = [c, d, b, n_db, n_bc, t]
        if n_ad >= 0:
            T[n_ad][3:6] = [t if g == u else g for g in T[n_ad][3:6]]
        if n_bc >= 0:
            T[n_bc][3:6] = [u if g == t else g for g in T[n_bc][3:6]]
    ntrip = k * (k - 1) * (k - 2) // 6
    out = []
    for v0, v1, v2 in (r[:3] for r in T):
        if k in (v0, v1, v2):
            i = v0 if v2 == k else (v1 if v0 == k else v2)
            j = v1 if v2 == k else (v2 if v0 == k else v0)
            out.append((ntrip + max(i, j) * (max(i, j) - 1) // 2 + min(i, j), _pack3(i, j, k)))
        else:
            a, c = min(v0, v1, v2), max(v0, v1, v2)
            b = v0 + v1 + v2 - a - c
            out.append((c * (c - 1) * (c - 2) // 6 + b * (b - 1) // 2 + a, _pack3(a, b, c)))
    return [key for _, key in sorted(out)], T


def _search(P, ids, k):
    """The candidate search by its definition: link triples (colex), then
    pairs with q (colex, turned counter-clockwise), each kept when no other
    polygon vertex is inside or on its perturbed circle."""
    def empty(i, j, l):
        return all(incircle_star(P[i], P[j], P[l], P[m], ids[i], ids[j], ids[l], ids[m]) < 0
                   for m in range(k + 1) if m not in (i, j, l))
    keys = []
    for l in range(2, k):
        for j in range(1, l):
            for i in range(j):
                if orient(P[i], P[j], P[l]) > 0 and empty(i, j, l):
                    keys.append(_pack3(i, j, l))
    for j in range(1, k):
        for i in range(j):
            o = orient(P[i], P[j], P[k])
            if o != 0:
                a, b = (i, j) if o > 0 else (j, i)
                if empty(a, b, k):
                    keys.append(_pack3(a, b, k))
    return keys


@pytest.mark.parametrize("seed,n,side", [(1, 70, 24), (4, 120, 30), (5, 200, 5000)])
def test_lawson_from_the_fan_reaches_the_search_result(seed, n, side):
    rng = np.random.default_rng(seed)
    cells = rng.choice(side * side, size=n, replace=False)
    xy = np.stack([cells % side, cells // side], axis=1).astype(np.int64)
    T = _tris(xy)
    Pt = [tuple(v) for v in xy.tolist()]
    taken = set(Pt)
    checked = flipped = 0
    for p in range(n):
        link = _link(T, p)
        if link is None or len(link) > 15:
            continue
        k = len(link)
        star = {t for t in T if p in t}
        for _ in range(16):
            d = rng.integers(-6, 7, size=2)
            q = (int(xy[p, 0] + d[0]), int(xy[p, 1] + d[1]))
            if q in taken or not (0 <= q[0] < side and 0 <= q[1] < side):
                continue
            if any(incircle_star(Pt[t[0]], Pt[t[1]], Pt[t[2]], q, t[0], t[1], t[2], p) > 0
                   for t in T - star):
                continue
            if not all(orient(Pt[link[s]], Pt[link[(s + 1) % k]], q) > 0 for s in range(k)):
                continue
            P = [Pt[v] for v in link] + [q]
            ids = list(link) + [p]
            keys, tris = _lawson(P, ids, k)
            assert keys == _search(P, ids, k), (seed, p, q)
            xy2 = xy.copy()
            xy2[p] = q
            mine = {_canon(tuple(ids[v] for v in r[:3])) for r in tris}
            assert _tris(xy2) == (T - star) | mine, (seed, p, q)
            checked += 1
            flipped += any(k not in r[:3] for r in tris)
    assert checked >= 20 and flipped >= 5, (checked, flipped)
