"""Seeded generators and the oracle's move rule (host-only)."""
import numpy as np

from oracle.kinetic import Kinetic
from paper_2308_06484_amd import workloads as W


def _check_workload(w):
    xy, pt_off, frame, mv, mv_off = w["xy"], w["pt_off"], w["frame"], w["mv"], w["mv_off"]
    B = len(pt_off) - 1
    assert xy.dtype == np.int32 and mv.dtype == np.int32 and mv_off.dtype == np.int32
    assert frame.shape == (B, 4) and mv.shape[1] == 4 and mv_off.shape[1] == B + 1
    for b in range(B):
        pts = xy[pt_off[b]:pt_off[b + 1]]
        assert len(np.unique(pts, axis=0)) == len(pts)
        assert (pts[:, 0] >= frame[b, 0]).all() and (pts[:, 0] < frame[b, 2]).all()
        assert (pts[:, 1] >= frame[b, 1]).all() and (pts[:, 1] < frame[b, 3]).all()
    assert (np.diff(mv_off, axis=1) >= 0).all()
    assert (mv_off[1:, 0] == mv_off[:-1, -1]).all()
    sizes = np.diff(pt_off)
    blk = np.repeat(np.tile(np.arange(B), mv_off.shape[0]), np.diff(mv_off, axis=1).reshape(-1))
    assert (mv[:, 0] >= 0).all() and (mv[:, 0] < sizes[blk]).all()
    assert ((mv[:, 1] >= 0) & (mv[:, 1] < 4)).all() and (mv[:, 2] >= 1).all()


def test_generators_are_seeded_and_well_formed():
    a, b = W.lattice256(seed=3), W.lattice256(seed=3)
    for k in ("xy", "pt_off", "frame", "mv", "mv_off"):
        assert np.array_equal(a[k], b[k])
    assert not np.array_equal(a["xy"], W.lattice256(seed=4)["xy"])
    _check_workload(a)
    g = W.grid1024(seed=1, steps=5, cells=4, per_block=256, cell=512)
    _check_workload(g)
    assert (g["mv"][:, 2] <= 8).all()
    u = W.uneven4096(seed=1, steps=3, blocks=12)
    _check_workload(u)
    m = W.multi2048(seed=1, steps=3, blocks=6, per_block=300, side=2048)
    _check_workload(m)
    # distinct movers per block and step
    for t in range(3):
        for bb in range(6):
            r = m["mv"][m["mv_off"][t, bb]:m["mv_off"][t, bb + 1], 0]
            assert len(np.unique(r)) == len(r) >= 1
    s = W.subset_blocks(g, [3, 7], steps=2)
    _check_workload(s)


def test_oracle_move_rule_closed_forms():
    xy = np.array([[0, 0], [1, 0], [0, 1], [2, 2]], np.int32)
    k = Kinetic(xy, [0, 4], [[0, 0, 3, 3]])
    mv = np.array([[0, 0, 1, 0],    # (0,0) -> (1,0): occupied, blocked
                   [0, 1, 1, 0],    # (0,0) -> (-1,0): outside the frame, blocked
                   [3, 0, 1, 0],    # (2,2) -> (3,2): outside (x1 = 3 is open), blocked
                   [3, 3, 2, 0],    # (2,2) -> (2,0): applied
                   [1, 0, 1, 0]],   # (1,0) -> (2,0): now occupied, blocked
                  np.int32)
    applied = k.apply_step(mv, np.array([0, 5]))
    assert applied.tolist() == [False, False, False, True, False]
    assert k.xy.tolist() == [[0, 0], [1, 0], [0, 1], [2, 0]]
    # a cell freed earlier in the step can be taken later in the same step
    mv2 = np.array([[3, 2, 1, 0], [1, 0, 1, 0]], np.int32)
    assert k.apply_step(mv2, np.array([0, 2])).tolist() == [True, True]
    assert k.xy.tolist() == [[0, 0], [2, 0], [0, 1], [2, 1]]
