"""Full-size runs of the batched and the selection workloads on the device,
against the oracle: every move's applied flag, every position and every
block's DT* after the last step (the oracle rebuilds each block from
scratch on host threads)."""
import numpy as np
import pytest
import torch

from oracle.kinetic import Kinetic
from paper_2308_06484_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)


def _run(w, mode="step", policy=None):
    from paper_2308_06484_amd.kdt import KineticDT
    dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=DEV)
    if policy:
        dt.set_policy(policy)
    mv = torch.from_numpy(w["mv"]).to(DEV)
    off = torch.from_numpy(np.ascontiguousarray(w["mv_off"])).to(DEV)
    applied = torch.zeros(w["mv"].shape[0], dtype=torch.int8, device=DEV)
    dt.run(mv, off, applied=applied, mode=mode)
    dt.sync()
    return dt, applied.cpu().numpy().astype(bool)


def _oracle(w):
    ref = Kinetic(w["xy"], w["pt_off"], w["frame"])
    app = np.concatenate([ref.apply_step(w["mv"], w["mv_off"][t]) for t in range(w["mv_off"].shape[0])])
    return ref, app


@pytest.mark.timeout(900)
def test_uneven4096_full_size_fused_and_per_step():
    _say("uneven4096 full size (4096 blocks, lognormal sizes 64..16384), 100 steps: generating")
    w = W.uneven4096(seed=1, steps=100)
    ref, app = _oracle(w)
    want = ref.all_dt(16)
    for mode in ("fused", "step"):
        _say(f"uneven4096 full size: {mode} launch")
        dt, got = _run(w, mode)
        assert np.array_equal(got, app), mode
        assert np.array_equal(dt.positions(), ref.xy), mode
        assert np.array_equal(dt.query_canonical(), want), mode
        st = dt.stats()
        assert st["errors"] == 0 and st["applied"] == int(app.sum())
        dt.close()


@pytest.mark.timeout(900)
def test_multi2048_full_size_repair_and_rebuild():
    _say("multi2048 full size (2048 blocks x 4096 points, 1..64 heavy-tailed moves per block), 3 steps")
    w = W.multi2048(seed=1, steps=3)
    ref, app = _oracle(w)
    want = ref.all_dt(16)
    for policy in ("repair", "rebuild"):
        _say(f"multi2048 full size: policy {policy}")
        dt, got = _run(w, "step", policy)
        assert np.array_equal(got, app), policy
        assert np.array_equal(dt.positions(), ref.xy), policy
        assert np.array_equal(dt.query_canonical(), want), policy
        st = dt.stats()
        assert st["errors"] == 0 and st["applied"] == int(app.sum())
        if policy == "rebuild":
            assert st["rebuilt"] > 0
        dt.close()


@pytest.mark.timeout(900)
def test_selector_mix_full_size_mlp_and_threshold():
    """The selection workload at full size (512 blocks, half of them with most
    points moving far every step): the network (random weights: any choice
    of branch must give the same DT*) and the threshold rule both take both
    branches; every block against the oracle after the last step."""
    _say("selector_mix full size, 12 steps")
    from paper_2308_06484_amd.kdt import MLP_PARAMS
    w = W.selector_mix(seed=1)
    ref, app = _oracle(w)
    want = ref.all_dt(16)
    g = torch.Generator().manual_seed(5)
    wts = ((torch.rand(MLP_PARAMS, generator=g) - 0.5) * 0.5).to(DEV)
    for policy, kw in (("mlp", dict(mlp_w=wts)), ("threshold", dict(tau=50.0))):
        _say(f"selector_mix full size: policy {policy}")
        from paper_2308_06484_amd.kdt import KineticDT
        dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=DEV)
        dt.set_policy(policy, **kw)
        mv = torch.from_numpy(w["mv"]).to(DEV)
        off = torch.from_numpy(np.ascontiguousarray(w["mv_off"])).to(DEV)
        applied = torch.zeros(w["mv"].shape[0], dtype=torch.int8, device=DEV)
        dt.run(mv, off, applied=applied)
        dt.sync()
        assert np.array_equal(applied.cpu().numpy().astype(bool), app), policy
        assert np.array_equal(dt.positions(), ref.xy), policy
        assert np.array_equal(dt.query_canonical(), want), policy
        st = dt.stats()
        assert st["errors"] == 0 and st["applied"] == int(app.sum())
        if policy == "threshold":
            assert 0 < st["rebuilt"] < 12 * 512, st
        dt.close()
