"""Full-size runs of the benchmark workloads on the device, compared with the
oracle after EVERY step: each step a different seeded subset of blocks
(rotating through a permutation, so every block is compared every
B / subset steps) is queried with kdt_query_blocks and compared element by
element with the oracle's from-scratch DT* of the same blocks, together
with every move's applied flag; after the last step every block and every
position is compared.  The oracle rebuilds blocks on host threads."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

from oracle.kinetic import Kinetic, KineticGlobal
from paper_2308_06484_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
THREADS = max(1, min(16, len(os.sched_getaffinity(0))))
SUBSET = 128


def _say(*a):
    print(*a, flush=True)


def rotating_parity(w, T, mode="step", policy=None, tau=0.0, mlp_w=None, seed=0, label="", waves=1,
                    repair=None, order=0, cut=0, mid=0):
    """Run w's first T steps one step per call; after every step compare the
    applied flags and a rotating subset of SUBSET blocks; at the end, all."""
    from paper_2308_06484_amd.kdt import KineticDT
    B = len(w["pt_off"]) - 1
    dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=DEV)
    if policy:
        dt.set_policy(policy, tau, mlp_w)
    if waves > 1:
        dt.set_block_waves(waves)
    if order or cut:
        dt.set_block_order(order, cut, mid)
    if repair:
        dt.set_repair(repair)
    ref = Kinetic(w["xy"], w["pt_off"], w["frame"])
    perm = np.random.default_rng(seed).permutation(B).astype(np.int32)
    mv = torch.from_numpy(w["mv"]).to(DEV)
    off = torch.from_numpy(np.ascontiguousarray(w["mv_off"][:T])).to(DEV)
    app = torch.zeros(max(1, len(w["mv"])), dtype=torch.int8, device=DEV)
    n_app = 0
    k = min(SUBSET, B)
    for t in range(T):
        dt.run(mv, off[t:t + 1].contiguous(), applied=app, mode=mode)
        a = ref.apply_step(w["mv"], w["mv_off"][t])
        lo, hi = int(w["mv_off"][t, 0]), int(w["mv_off"][t, -1])
        got = app[lo:hi].cpu().numpy().astype(bool)
        assert np.array_equal(got, a), f"{label}: applied flags differ in step {t}"
        n_app += int(a.sum())
        blocks = perm[(t * k + np.arange(k)) % B]
        tris, _, boff = dt.query_blocks(blocks)
        want = ref.blocks_dt(blocks, THREADS)
        for i, b in enumerate(blocks):
            assert np.array_equal(tris[boff[i]:boff[i + 1]], want[i]), f"{label}: block {b} differs after step {t}"
        if t % 50 == 0:
            _say(f"{label}: step {t} ok")
    assert np.array_equal(dt.positions(), ref.xy), label
    assert np.array_equal(dt.query_canonical(), ref.all_dt(THREADS)), f"{label}: final DT* differs"
    st = dt.stats()
    assert st["errors"] == 0 and st["applied"] == n_app, (label, st)
    dt.close()
    return st


@pytest.mark.timeout(900)
def test_grid1024_full_size_every_step():
    _say("grid1024 full size (1024 blocks x 1024 points), 1000 steps, per-step launch")
    w = W.grid1024(seed=1, steps=1000)
    rotating_parity(w, 1000, label="grid1024")


@pytest.mark.timeout(900)
def test_uneven4096_full_size_every_step():
    _say("uneven4096 full size (4096 blocks, lognormal sizes 64..16384), 500 steps")
    w = W.uneven4096(seed=1, steps=500)
    # the first steps in the fused form, the rest per step: both compared
    rotating_parity(w, 500, label="uneven4096 per step")
    rotating_parity(w, 60, mode="fused", seed=1, label="uneven4096 fused")
    rotating_parity(w, 60, mode="persistent", seed=2, label="uneven4096 persistent")


@pytest.mark.timeout(900)
def test_multi2048_full_size_every_step_all_policies():
    """multi2048 at full size for its 100 steps under the repair rule, the
    threshold rule (tau calibrated on another seed) and the network trained
    on the device on another seed; rebuild-only for 10 steps."""
    from paper_2308_06484_amd import selector as S
    _say("multi2048: calibration (seed 101, 6 steps, forced repair and forced rebuild)")
    cal = W.multi2048(seed=101, steps=6)
    X, Y = S.collect(cal, 6, DEV)
    del cal
    wts = torch.from_numpy(S.train(X, Y, epochs=200, batch=2048, lr=0.02, device=DEV)).to(DEV)
    tau = S.calibrate_threshold(X, Y)
    # a tau low enough that the rule also takes the rebuild branch
    tau_lo = float(np.quantile(X[:, 3], 0.9))
    _say(f"multi2048 full size (2048 blocks x 4096 points), 100 steps; tau {tau:.2f}, low tau {tau_lo:.2f}")
    w = W.multi2048(seed=1, steps=100)
    rotating_parity(w, 100, label="multi2048 repair")
    rotating_parity(w, 100, policy="mlp", mlp_w=wts, seed=1, label="multi2048 mlp")
    # the benchmark's launch shape: four wavefronts per block, most moves first
    rotating_parity(w, 100, policy="mlp", mlp_w=wts, seed=4, waves=4, order=1,
                    label="multi2048 mlp, 4 waves, ordered")
    st = rotating_parity(w, 100, policy="threshold", tau=tau_lo, seed=2, label="multi2048 threshold")
    assert st["rebuilt"] > 0
    st = rotating_parity(w, 10, policy="rebuild", seed=3, label="multi2048 rebuild")
    assert st["rebuilt"] > 0


@pytest.mark.timeout(900)
def test_global4m_twenty_steps_every_step():
    """Global mode at full size (4,194,304 points, 4096 kd cells): 20
    consecutive steps, the whole triangulation against the oracle's
    from-scratch DT* after every step (the oracle rebuilds the 20 states on
    host threads), plus the kd cells and positions."""
    from paper_2308_06484_amd.kdt import GlobalDT
    T = 20
    _say("global4m full size: generating")
    w = W.global4m(seed=1, steps=T)
    G = GlobalDT(w["xy"], [0, 0, w["side"], w["side"]], w["depth"], 1 << w["depth"], device=DEV)
    K = KineticGlobal(w["xy"], w["side"], w["depth"])
    mv = torch.from_numpy(np.ascontiguousarray(w["mv"])).to(DEV)
    app = torch.zeros(len(w["mv"]), dtype=torch.int8, device=DEV)
    snaps, got = [], []
    for t in range(T):
        G.run(mv, w["step_off"][t:t + 2], applied=app)
        lo, hi = int(w["step_off"][t]), int(w["step_off"][t + 1])
        a = K.apply_step(w["mv"][lo:hi])
        assert np.array_equal(app[lo:hi].cpu().numpy().astype(bool), a), f"applied flags differ in step {t}"
        snaps.append(K.xy.copy())
        tris, _, _ = G.query_blocks(np.array([0], np.int32))
        got.append(tris)
        _say(f"global4m: step {t} run and queried")
    assert np.array_equal(G.positions(), K.xy)
    assert np.array_equal(G.owner(), K.owner())

    def oracle_dt(xy):
        k = KineticGlobal.__new__(KineticGlobal)
        k.xy = xy
        return k.dt()

    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        for t, want in enumerate(ex.map(oracle_dt, snaps)):
            assert np.array_equal(got[t], want), f"global DT* differs after step {t}"
            got[t] = None
    _say("global4m: 20 steps equal")
    G.close()
