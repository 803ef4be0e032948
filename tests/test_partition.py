"""kdt_partition (host code of the library, no GPU needed) against the
quad-tree division written out plainly from its description (Sec. III,
"Data structure"; Sec. IV, Quad-treeDvision): the smallest covering square,
cut into four equal squares until every square holds at most the
threshold number of points.  Readings shared by both: the square's side is
rounded up to a power of two, empty quarters are dropped, a square whose
cut would leave a quarter with fewer than 4 points or all of them on one
line is not cut."""
import numpy as np
import pytest

from paper_2308_06484_amd import kdt as K
from paper_2308_06484_amd import workloads as W


def _collinear(p):
    if len(p) < 3:
        return True
    a, b = p[0].astype(np.int64), p[1].astype(np.int64)
    c = p[2:].astype(np.int64)
    return bool(np.all((b[0] - a[0]) * (c[:, 1] - a[1]) - (b[1] - a[1]) * (c[:, 0] - a[0]) == 0))


def _square(xy):
    lo = xy.min(axis=0).astype(np.int64)
    ext = int((xy.max(axis=0).astype(np.int64) - lo).max()) + 1
    side = 1
    while side < ext:
        side *= 2
    return int(lo[0]), int(lo[1]), side


def quadtree_ref(xy, thr):
    x0, y0, side = _square(xy)
    out = []

    def node(idx, qx, qy, s):
        if len(idx) > thr and s > 1:
            h = s // 2
            parts = []
            for cx, cy in ((qx, qy), (qx + h, qy), (qx, qy + h), (qx + h, qy + h)):
                p = xy[idx]
                inside = (p[:, 0] >= cx) & (p[:, 0] < cx + h) & (p[:, 1] >= cy) & (p[:, 1] < cy + h)
                parts.append((idx[inside], cx, cy))
            if all(len(i) == 0 or (len(i) >= 4 and not _collinear(xy[i])) for i, _, _ in parts):
                for i, cx, cy in parts:
                    if len(i):
                        node(i, cx, cy, h)
                return
        out.append((np.sort(idx), qx, qy, s))

    node(np.arange(len(xy)), x0, y0, side)
    return out


def grid_ref(xy, cells):
    x0, y0, side = _square(xy)
    d = 0
    while 4 ** d < cells:
        d += 1
    side = max(side, 1 << d)
    cs = side >> d
    cx = (xy[:, 0].astype(np.int64) - x0) // cs
    cy = (xy[:, 1].astype(np.int64) - y0) // cs
    key = cy * (1 << d) + cx
    out = []
    for k in np.unique(key):
        idx = np.nonzero(key == k)[0]
        out.append((idx, x0 + int(k % (1 << d)) * cs, y0 + int(k // (1 << d)) * cs, cs))
    return out


def _compare(xy, scheme, param, ref):
    perm, off, fr = K.partition(xy, scheme, param)
    assert len(off) == len(ref) + 1
    assert sorted(perm.tolist()) == list(range(len(xy)))
    for b, (idx, qx, qy, s) in enumerate(ref):
        assert perm[off[b]:off[b + 1]].tolist() == idx.tolist(), b
        assert fr[b].tolist() == [qx, qy, min(qx + s, 1 << 24), min(qy + s, 1 << 24)], b
        p = xy[perm[off[b]:off[b + 1]]]
        assert np.all((p[:, 0] >= fr[b, 0]) & (p[:, 0] < fr[b, 2]) & (p[:, 1] >= fr[b, 1]) & (p[:, 1] < fr[b, 3]))
    return perm, off, fr


@pytest.mark.parametrize("thr", [4, 16, 100, 1000])
def test_quadtree_uniform_and_mixture(thr):
    rng = np.random.default_rng(thr)
    for xy in (W._distinct_uniform(rng, 3000, 100, 50, 5000, 7000),
               W._distinct_gmm(rng, 3000, 0, 65536)):
        ref = quadtree_ref(xy, thr)
        perm, off, fr = _compare(xy, "quadtree", thr, ref)
        sizes = np.diff(off)
        assert sizes.min() >= 4 or len(sizes) == 1
        # a block above the threshold is one whose cut was refused
        for b in np.nonzero(sizes > thr)[0]:
            assert fr[b, 2] - fr[b, 0] > 1


def test_quadtree_refuses_a_cut_that_leaves_three_points():
    # 8 points in the lower-left quarter, 3 in the upper-right: with threshold
    # 4 the root would be cut, but one quarter would hold only 3 points
    xy = np.array([(0, 0), (1, 0), (0, 1), (1, 1), (2, 0), (0, 2), (2, 2), (3, 1),
                   (14, 14), (15, 13), (13, 15)], np.int32)
    perm, off, fr = _compare(xy, "quadtree", 4, quadtree_ref(xy, 4))
    assert len(off) == 2 and fr[0].tolist() == [0, 0, 16, 16]


def test_quadtree_single_block_and_deep_split():
    rng = np.random.default_rng(3)
    xy = W._distinct_uniform(rng, 500, 0, 0, 1 << 20, 1 << 20)
    _compare(xy, "quadtree", 1000, quadtree_ref(xy, 1000))
    # a tight cluster far from a spread of points: many levels deep
    xy = np.concatenate([W._distinct_uniform(rng, 64, 1 << 22, 1 << 22, 64, 64),
                         W._distinct_uniform(rng, 200, 0, 0, 1 << 23, 1 << 23)])
    xy = np.unique(xy, axis=0)
    _compare(xy, "quadtree", 32, quadtree_ref(xy, 32))


@pytest.mark.parametrize("cells", [1, 4, 64, 1024])
def test_grid(cells):
    rng = np.random.default_rng(cells)
    xy = W._distinct_uniform(rng, 20000, 7, 3, 65536 - 7, 65536 - 3)
    _compare(xy, "grid", cells, grid_ref(xy, cells))


def test_partition_errors():
    import ctypes
    L = K.lib()
    xy = np.array([(0, 0), (5, 0), (0, 5), (5, 5)], np.int32)
    perm = np.zeros(4, np.int64)
    nb = ctypes.c_int32(0)

    def call(pts, scheme, param, cap=0, off=None, fr=None):
        pts = np.ascontiguousarray(pts, np.int32)
        return L.kdt_partition(K._ptr(pts), len(pts), scheme, param, K._ptr(perm), K._ptr(off), K._ptr(fr),
                               cap, ctypes.byref(nb))

    assert call(xy, 0, 3) == K.E_ARG          # not a power of four
    assert call(xy, 1, 3) == K.E_ARG          # threshold below 4
    assert call(xy, 7, 16) == K.E_ARG         # unknown scheme
    assert call([(0, 0), (5, 0), (5, 0), (0, 5)], 1, 16) == K.E_DUP
    assert call([(0, 0), (5, 0), (0, 1 << 24), (0, 5)], 1, 16) == K.E_RANGE
    assert call(xy, 0, 4) == K.E_CAPACITY and nb.value == 4  # four cells, no room given
    off = np.zeros(5, np.int64)
    fr = np.zeros((4, 4), np.int32)
    assert call(xy, 0, 4, 4, off, fr) == K.OK and off.tolist() == [0, 1, 2, 3, 4]
