"""Pins of the global-mode oracle (one DT* over all points, kd ownership).

The move rule is pinned by hand-made cases whose outcome follows from the
rule as stated (list order, occupancy at that moment, half-open domain); the
kd partition by hand on four points and by agreement with the workload
generator's own grouping; the triangulation by insertion-order independence
and the certificate of tests/certificate.py.
"""
import numpy as np

from oracle import dt_star
from oracle.kinetic import Kinetic, KineticGlobal, kd_cell, kd_splits
from paper_2308_06484_amd import workloads as W
from tests import certificate


def test_kd_split_by_hand():
    # level 0 orders by (x, y): (1,5) (2,0) | (2,3) (7,1); split key (2,3)
    xy = np.array([[7, 1], [2, 3], [1, 5], [2, 0]])
    sp = kd_splits(xy, 1)
    assert sp[1].tolist() == [2, 3]
    assert kd_cell(xy, sp, 1).tolist() == [1, 1, 0, 0]
    # level 1 orders each half by (y, x): left (2,0) | (1,5) -> key (5,1);
    # right (7,1) | (2,3) -> key (3,2)
    sp2 = kd_splits(xy, 2)
    assert sp2[2].tolist() == [5, 1] and sp2[3].tolist() == [3, 2]
    assert kd_cell(xy, sp2, 2).tolist() == [2, 3, 1, 0]
    # a position equal to a split key goes right; positions off the points too
    assert kd_cell([[2, 3], [2, 2], [0, 9]], sp, 1).tolist() == [1, 0, 0]


def test_kd_cells_match_generator_grouping():
    w = W.global_small(seed=3, steps=1)
    sp = kd_splits(w["xy"], w["depth"])
    own = kd_cell(w["xy"], sp, w["depth"])
    per = len(w["xy"]) >> w["depth"]
    assert np.array_equal(own, np.arange(len(own)) // per)


def test_move_rule_by_hand():
    xy = np.array([[0, 0], [5, 0], [0, 5], [5, 5]])
    K = KineticGlobal(xy, 8, 1)
    # p0 +x 5 onto p1: blocked; p1 -x 1: applied
    assert K.apply_step(np.array([[0, 0, 5, 0], [1, 1, 1, 0]])).tolist() == [False, True]
    assert K.xy.tolist() == [[0, 0], [4, 0], [0, 5], [5, 5]]
    # a cell vacated earlier in the step is free; later, it is not yet
    K2 = KineticGlobal(xy, 8, 1)
    assert K2.apply_step(np.array([[3, 0, 1, 0], [1, 2, 5, 0]])).tolist() == [True, True]
    assert K2.xy[1].tolist() == [5, 5] and K2.xy[3].tolist() == [6, 5]
    K3 = KineticGlobal(xy, 8, 1)
    assert K3.apply_step(np.array([[1, 2, 5, 0], [3, 0, 1, 0]])).tolist() == [False, True]
    # the half-open domain: x = 8 is outside, x = 7 inside, negatives outside
    K4 = KineticGlobal(xy, 8, 1)
    assert K4.apply_step(np.array([[3, 0, 3, 0], [3, 0, 2, 0], [0, 3, 1, 0]])).tolist() == [False, True, False]
    # a target taken earlier in the same step is held
    K5 = KineticGlobal(xy, 8, 1)
    assert K5.apply_step(np.array([[0, 2, 2, 0], [2, 3, 3, 0]])).tolist() == [True, False]


def test_one_cell_matches_block_oracle():
    w = W.global_small(seed=5, steps=10, n=1024, depth=0, side=1024)
    G = KineticGlobal(w["xy"], w["side"], 0)
    K = Kinetic(w["xy"], [0, len(w["xy"])], [[0, 0, w["side"], w["side"]]])
    for t in range(10):
        rows = w["mv"][w["step_off"][t]:w["step_off"][t + 1]]
        a = G.apply_step(rows)
        b = K.apply_step(rows, [0, len(rows)])
        assert np.array_equal(a, b)
    assert np.array_equal(G.xy, K.xy)
    assert np.array_equal(G.dt(), K.all_dt())


def test_global_dt_order_independent_and_certified():
    w = W.global_small(seed=2, steps=5, n=4096, depth=2, side=2048)
    G = KineticGlobal(w["xy"], w["side"], w["depth"])
    for t in range(5):
        G.apply_step(w["mv"][w["step_off"][t]:w["step_off"][t + 1]])
    d = G.dt()
    assert np.array_equal(d, dt_star(G.xy, np.arange(len(G.xy))))
    certificate.check(G.xy, np.arange(len(G.xy)), d)
    own = G.owner()
    assert own.min() >= 0 and own.max() < 4
