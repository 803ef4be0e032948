"""Several wavefronts per block (kdt_set_block_waves 2 and 4): a block's
commuting moves in reservation rounds, the others afterwards in list order;
with the blocks taken most moves first and with size classes (only blocks
with at least `cut` moves get several wavefronts, the others one -- or two
from `mid` moves -- on separate streams at once) (kdt_set_block_order).  Every step against the oracle
(triangulations, applied flags, positions), on workloads with many moves per
block, dense lattices where moves share cells and are blocked, a point whose
degree exceeds the repair path's capacity, and under the rebuilding
policies."""
import numpy as np
import pytest
import torch

from oracle.kinetic import Kinetic
from paper_2308_06484_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)


def run_waves(w, waves, policy=None, tau=0.0, mlp_w=None, label="", order=0, cut=0, mid=0):
    from paper_2308_06484_amd.kdt import KineticDT
    T = w["mv_off"].shape[0]
    dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=DEV)
    dt.set_block_waves(waves)
    dt.set_block_order(order, cut, mid)
    label = f"{label} order {order} cut {cut} mid {mid}"
    if policy:
        dt.set_policy(policy, tau, mlp_w)
    ref = Kinetic(w["xy"], w["pt_off"], w["frame"])
    mv = torch.from_numpy(w["mv"]).to(DEV)
    off = torch.from_numpy(np.ascontiguousarray(w["mv_off"])).to(DEV)
    app = torch.full((max(1, len(w["mv"])),), -1, dtype=torch.int8, device=DEV)
    n_app = 0
    for t in range(T):
        dt.run(mv, off[t:t + 1].contiguous(), applied=app)
        a = ref.apply_step(w["mv"], w["mv_off"][t])
        lo, hi = int(w["mv_off"][t, 0]), int(w["mv_off"][t, -1])
        got = app[lo:hi].cpu().numpy()
        assert np.array_equal(got.astype(bool), a) and np.all(got >= 0), f"{label} waves {waves}: flags, step {t}"
        n_app += int(a.sum())
        assert np.array_equal(dt.query_canonical(), ref.all_dt(8)), f"{label} waves {waves}: DT* after step {t}"
    assert np.array_equal(dt.positions(), ref.xy)
    st = dt.stats()
    assert st["errors"] == 0 and st["applied"] == n_app, (label, waves, st)
    dt.close()
    return st


@pytest.mark.parametrize("waves,order,cut,mid", [(2, 0, 0, 0), (4, 0, 0, 0), (2, 1, 0, 0), (4, 1, 0, 0), (2, 1, 6, 0),
                                                 (4, 1, 6, 0), (4, 1, 20, 5)])
def test_many_moves_per_block(waves, order, cut, mid):
    _say(f"multi-move blocks, {waves} wavefronts per block, order {order}, cut {cut}, mid {mid}")
    w = W.multi2048(seed=9, steps=8, blocks=24, per_block=1024, side=4096, dcap=1024)
    st = run_waves(w, waves, label="multi", order=order, cut=cut, mid=mid)
    assert st["applied"] > 1000


@pytest.mark.parametrize("waves,order,cut,mid", [(2, 0, 0, 0), (4, 0, 0, 0), (2, 1, 16, 0), (4, 1, 20, 12)])
def test_dense_lattice_shared_cells(waves, order, cut, mid):
    """Nearly full small lattices, 8..30 moves per block per step of 1..2
    units: many moves share cells (they go to the rest list) or are blocked."""
    rng = np.random.default_rng(17 + waves)
    xy, off, frame = [], [0], []
    for b in range(8):
        side = 8 + b
        full = np.array([(x, y) for y in range(side) for x in range(side)])
        keep = full[rng.permutation(len(full))[: int(len(full) * 0.7)]]
        keep = keep[np.lexsort((keep[:, 0], keep[:, 1]))]
        xy.append(keep + np.array([100 * b, 0]))
        off.append(off[-1] + len(keep))
        frame.append([100 * b, 0, 100 * b + side, side])
    xy = np.concatenate(xy).astype(np.int32)
    sizes = np.diff(off)
    T = 25
    recs, offs, base = [], np.zeros((T, 9), np.int64), 0
    for t in range(T):
        offs[t, 0] = base
        for b in range(8):
            k = int(rng.integers(8, 31))
            r = np.zeros((k, 4), np.int32)
            r[:, 0] = rng.integers(0, sizes[b], size=k)  # repeated points too
            r[:, 1] = rng.integers(0, 4, size=k)
            r[:, 2] = rng.integers(1, 3, size=k)
            recs.append(r)
            base += k
            offs[t, b + 1] = base
    w = dict(xy=xy, pt_off=np.array(off, np.int64), frame=np.array(frame, np.int32),
             mv=np.concatenate(recs), mv_off=offs.astype(np.int32))
    _say(f"dense lattices, {waves} wavefronts per block, order {order}, cut {cut}, mid {mid}")
    run_waves(w, waves, label="dense", order=order, cut=cut, mid=mid)


def test_capacity_overflow_with_block_waves():
    """A centre point of degree above the repair path's capacity moves among
    other moves of its block: its plan fails, the rest list takes it (and the
    moves after it that the rounds did not apply), the sequential path
    rebuilds the block; the same DT* as the oracle after every step."""
    rng = np.random.default_rng(5)
    # the 108 lattice points of a circle of radius 1105 = 5 * 13 * 17 around
    # the centre, plus points outside it
    ang = []
    r = 1105
    for x in range(-r, r + 1):
        y2 = r * r - x * x
        y = int(round(np.sqrt(y2)))
        if y * y == y2:
            ang.append((x, y))
            ang.append((x, -y))
    circle = sorted(set(ang))
    c = (2048, 2048)
    pts = [c] + [(c[0] + x, c[1] + y) for x, y in circle]
    extra = set()
    while len(extra) < 200:
        x, y = int(rng.integers(0, 4096)), int(rng.integers(0, 4096))
        if (x - c[0]) ** 2 + (y - c[1]) ** 2 > (r + 50) ** 2:
            extra.add((x, y))
    blk = np.array(pts + sorted(extra), np.int32)
    n = len(blk)
    xy = np.concatenate([blk, blk + np.array([4096, 0], np.int32)])
    T = 6
    recs, offs, base = [], np.zeros((T, 3), np.int64), 0
    for t in range(T):
        offs[t, 0] = base
        for b in range(2):
            k = 12
            who = rng.choice(np.arange(1, n), size=k, replace=False)
            if b == 0 and t % 2 == 0:
                who[3] = 0  # the centre, in the middle of the step's list
            rr = np.zeros((k, 4), np.int32)
            rr[:, 0] = who
            rr[:, 1] = rng.integers(0, 4, size=k)
            rr[:, 2] = rng.integers(1, 4, size=k)
            recs.append(rr)
            base += k
            offs[t, b + 1] = base
    w = dict(xy=xy, pt_off=np.array([0, n, 2 * n], np.int64),
             frame=np.array([[0, 0, 4096, 4096], [4096, 0, 8192, 4096]], np.int32),
             mv=np.concatenate(recs), mv_off=offs.astype(np.int32))
    for order, cut in ((0, 0), (1, 12)):
        _say(f"capacity overflow with 4 wavefronts per block: degree {len(circle)} centre, order {order}, cut {cut}")
        st = run_waves(w, 4, label="capacity", order=order, cut=cut)
        assert st["rebuilt"] >= 1, st


@pytest.mark.parametrize("policy,cut,mid", [("rebuild", 0, 0), ("threshold", 0, 0), ("mlp", 0, 0), ("mlp", 4, 0),
                                            ("threshold", 4, 0), ("mlp", 6, 3)])
def test_block_waves_under_rebuilding_policies(policy, cut, mid):
    from paper_2308_06484_amd.kdt import MLP_PARAMS
    w = W.selector_mix(seed=4, steps=4, small=12, large=12)
    g = torch.Generator().manual_seed(9)
    wts = ((torch.rand(MLP_PARAMS, generator=g) - 0.5) * 0.5).to(DEV)
    kw = {"rebuild": {}, "threshold": {"tau": 50.0}, "mlp": {"mlp_w": wts}}[policy]
    _say(f"selector_mix subset, 4 wavefronts per block, policy {policy}, cut {cut}, mid {mid}")
    run_waves(w, 4, policy=policy, label=policy, order=1 if cut else 0, cut=cut, mid=mid, **kw)


def test_block_waves_full_size_multi2048_every_step():
    """multi2048 at full size, 40 steps, 4 wavefronts per block for the
    blocks with at least 32 moves and one for the others, at once: a
    rotating subset of 128 blocks against the oracle after every step, all
    blocks at the end; then 40 steps with a two-wavefront middle class."""
    from tests.test_gpu_fullsize import rotating_parity
    w = W.multi2048(seed=1, steps=40)
    rotating_parity(w, 40, waves=4, order=1, cut=32, label="multi2048 4 waves, cut 32")
    rotating_parity(w, 40, waves=4, order=1, cut=48, mid=16, seed=5, label="multi2048 4 waves, cut 48, mid 16")


@pytest.mark.parametrize("waves,cut", [(4, 0), (4, 6), (2, 0)])
def test_empty_steps_and_a_failed_block_under_the_schedules(waves, cut):
    """Steps in which no block moves, or only one does, pass through the
    ordered and split launches unchanged; a move with an out-of-range point
    fails its block (KDT_E_ARG) and every other block still matches the
    oracle after every later step."""
    K = __import__("paper_2308_06484_amd.kdt", fromlist=["KineticDT"])
    w = W.multi2048(seed=13, steps=6, blocks=16, per_block=512, side=2048, dcap=512)
    mv = w["mv"].copy()
    off = w["mv_off"].copy()
    B = len(w["pt_off"]) - 1
    # step 1: no moves at all; step 2: only block 5 moves
    base = int(off[1, 0])
    off[1, :] = base
    keep = off[2, 6] - off[2, 5]
    off[2, :6] = off[2, 5]
    off[2, 6:] = off[2, 5] + keep
    # step 4: block 9's first move names a point outside the block
    bad_b = 9
    mv[int(off[4, bad_b]), 0] = 10 ** 6
    # the oracle skips the failed block from step 4 on: compare the others
    ref = Kinetic(w["xy"], w["pt_off"], w["frame"])
    dt = K.KineticDT(w["xy"], w["pt_off"], w["frame"], device=DEV)
    dt.set_block_waves(waves)
    dt.set_block_order(1, cut, 0)
    mvt = torch.from_numpy(mv).to(DEV)
    offt = torch.from_numpy(np.ascontiguousarray(off)).to(DEV)
    others = np.array([b for b in range(B) if b != bad_b], np.int32)
    for t in range(4):  # every block, every step, until the failure
        dt.run(mvt, offt[t:t + 1].contiguous())
        ref.apply_step(mv, off[t])
        tris, _, bo = dt.query_blocks(np.arange(B, dtype=np.int32))
        for b in range(B):
            assert np.array_equal(tris[bo[b]:bo[b + 1]], ref.block_dt(b)), (waves, cut, t, b)
    # steps 4 and 5 in one call: the failure of step 4 is read afterwards
    dt.run(mvt, offt[4:6].contiguous())
    for t in (4, 5):  # the oracle without the failed block's moves
        lo, hi = int(off[t, bad_b]), int(off[t, bad_b + 1])
        mv_ref = np.delete(mv, np.arange(lo, hi), axis=0)
        row = off[t].copy()
        row[bad_b + 1:] -= hi - lo
        ref.apply_step(mv_ref, row)
    with pytest.raises(K.KDTError):
        dt.sync()
    tris, _, bo = dt.query_blocks(others)
    for i, b in enumerate(others):
        assert np.array_equal(tris[bo[i]:bo[i + 1]], ref.block_dt(b)), (waves, cut, b)
    st = dt.block_status()
    assert st[bad_b] == K.E_ARG and np.count_nonzero(st) == 1
    dt.close()
