"""Pins of the oracle's quad-tree (oracle/kinetic.py: quadtree,
quadtree_leaf) -- Sec. III, "Data structure"; Fig. 2, 3: a square holding
more than the threshold number of points is cut into four equal quarters.
Checked against a hand-worked case and against the definition's invariants
on random sets (the leaves tile the root without overlap, every leaf holds
at most the threshold unless it is one lattice cell wide, every inner node
holds more, a point's leaf is the one leaf that contains it)."""
import numpy as np
import pytest

from oracle.kinetic import quadtree, quadtree_leaf


def test_hand_worked_tree():
    # domain 8 x 8; threshold 1: the root (5 points) is cut; its low-x
    # low-y quarter holds two points and is cut again; the others hold one
    # point or none
    xy = [(0, 0), (3, 3), (5, 1), (1, 6), (6, 6)]
    nodes, cell = quadtree(xy, (0, 0, 8, 8), 1)
    assert nodes[0] == [0, 0, 8, 1]
    assert nodes[1] == [0, 0, 4, 5] and nodes[2] == [4, 0, 4, -1]
    assert nodes[3] == [0, 4, 4, -1] and nodes[4] == [4, 4, 4, -1]
    assert [n[:3] for n in nodes[5:9]] == [[0, 0, 2], [2, 0, 2], [0, 2, 2], [2, 2, 2]]
    assert list(cell) == [5, 8, 2, 3, 4]


def _contains(n, x, y):
    return n[0] <= x < n[0] + n[2] and n[1] <= y < n[1] + n[2]


@pytest.mark.parametrize("seed,thr", [(0, 1), (1, 4), (2, 16), (3, 64)])
def test_invariants_on_random_sets(seed, thr):
    rng = np.random.default_rng(seed)
    side = 256
    pts = np.unique(rng.integers(0, side, size=(400, 2)), axis=0)
    # clustered points too, so that some branches go deep
    pts = np.unique(np.concatenate([pts, rng.integers(100, 108, size=(60, 2))]), axis=0)
    nodes, cell = quadtree(pts, (0, 0, side, side), thr)
    leaves = [k for k, n in enumerate(nodes) if n[3] < 0]
    area = sum(nodes[k][2] ** 2 for k in leaves)
    assert area == nodes[0][2] ** 2  # the leaves tile the root
    for k, n in enumerate(nodes):
        inside = sum(_contains(n, x, y) for x, y in pts.tolist())
        if n[3] < 0:
            assert inside <= thr or n[2] == 1
        else:
            assert inside > thr
            for q in range(4):  # children are the four quarters, in order
                c = nodes[n[3] + q]
                h = n[2] // 2
                assert c[:3] == [n[0] + (q & 1) * h, n[1] + (q >> 1) * h, h]
    for i, (x, y) in enumerate(pts.tolist()):
        holders = [k for k in leaves if _contains(nodes[k], x, y)]
        assert holders == [cell[i]] == [quadtree_leaf(nodes, x, y)]
