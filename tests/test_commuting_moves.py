"""The reordering the concurrent launches rest on (several wavefronts per
block; the global mode's reservation rounds), checked against the move rule
applied in list order.  Reading: within a step, a move whose source and
target cells are named by no other move of the step commutes with every
other move -- its target's occupancy can change only by itself, and it
changes the occupancy of no cell another move names -- so such moves may run
first, in any order, and the others after them in list order, PROVIDED no
point moves twice in the step: a point's second move starts where its first
one ended, a cell the start-of-step positions do not name.  A step in which
a point moves twice runs wholly in list order.  This is a model of the
classification, in plain Python; the kernels' outcomes are compared with the
oracle by the GPU tests."""
import numpy as np

D = ((1, 0), (-1, 0), (0, 1), (0, -1))


def sequential(pos, frame, moves):
    """The move rule in list order; returns applied flags, updates pos."""
    x0, y0, x1, y1 = frame
    occ = {tuple(p) for p in pos}
    out = []
    for p, d, dist in moves:
        px, py = pos[p]
        q = (px + dist * D[d][0], py + dist * D[d][1])
        if not (x0 <= q[0] < x1 and y0 <= q[1] < y1) or q in occ:
            out.append(False)
            continue
        occ.discard((px, py))
        occ.add(q)
        pos[p] = q
        out.append(True)
    return out


def reordered(pos, frame, moves, repeat_rule=True, rng=None):
    """Commuting moves first (shuffled), the others in list order."""
    x0, y0, x1, y1 = frame
    pts = [m[0] for m in moves]
    if repeat_rule and len(set(pts)) < len(pts):
        return sequential(pos, frame, moves)
    src = [tuple(pos[p]) for p in pts]
    tgt = []
    for (p, d, dist), s in zip(moves, src):
        q = (s[0] + dist * D[d][0], s[1] + dist * D[d][1])
        tgt.append(q if (x0 <= q[0] < x1 and y0 <= q[1] < y1) else None)
    named = {}
    for s, t in zip(src, tgt):
        named[s] = named.get(s, 0) + 1
        if t is not None:
            named[t] = named.get(t, 0) + 1
    inter = [named[s] > 1 or (t is not None and named[t] > 1) or pts.count(pts[i]) > 1
             for i, (s, t) in enumerate(zip(src, tgt))]
    comm = [i for i in range(len(moves)) if not inter[i]]
    rest = [i for i in range(len(moves)) if inter[i]]
    if rng is not None:
        comm = list(rng.permutation(comm))
    out = [None] * len(moves)
    for i, a in zip(comm, sequential(pos, frame, [moves[i] for i in comm])):
        out[i] = a
    for i, a in zip(rest, sequential(pos, frame, [moves[i] for i in rest])):
        out[i] = a
    return out


def _dense_case(rng, side, k, repeats):
    full = [(x, y) for y in range(side) for x in range(side)]
    idx = rng.permutation(len(full))[: int(0.7 * len(full))]
    pos = [full[i] for i in idx]
    n = len(pos)
    who = rng.integers(0, n, size=k) if repeats else rng.permutation(n)[:k]
    moves = [(int(p), int(rng.integers(0, 4)), int(rng.integers(1, 3))) for p in who]
    return pos, (0, 0, side, side), moves


def test_reordering_equals_list_order_on_dense_lattices():
    rng = np.random.default_rng(0)
    for trial in range(3000):
        side = int(rng.integers(4, 12))
        pos, fr, moves = _dense_case(rng, side, int(rng.integers(2, 30)), repeats=trial % 2 == 0)
        a, b = list(pos), list(pos)
        want = sequential(a, fr, moves)
        got = reordered(b, fr, moves, rng=rng)
        assert got == want and a == b, trial


def test_repeated_points_need_list_order():
    """Without the repeated-point rule the reordering is wrong: point 0
    moves down, then left by 2; its second move's real target (2, 1) is the
    source of a later move that shares no start-of-step cell with anyone."""
    pos = [(4, 2), (2, 1), (7, 7)]
    fr = (0, 0, 10, 10)
    moves = [(0, 3, 1), (0, 1, 2), (1, 2, 3)]
    a, b, c = list(pos), list(pos), list(pos)
    want = sequential(a, fr, moves)
    assert want == [True, False, True]
    assert reordered(b, fr, moves, repeat_rule=False) != want
    assert reordered(c, fr, moves) == want and c == a
