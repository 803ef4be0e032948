"""kdt_dcalc (the d-calculation of Sec. III / IV on the device) against the
brute-force oracle: per-block mindistance^2 and diameter^2, the minimum over
blocks, d^2 over the steps and every block's running N-spread, on uniform,
lattice (ties everywhere) and mixture blocks, after moves; N from 1 to 8."""
import numpy as np
import pytest
import torch

from oracle.dcalc import NONE, DTracker, dcalc
from oracle.kinetic import Kinetic
from paper_2308_06484_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _blocks(rng):
    parts, frames = [], []
    x0 = 0
    for kind, n, side in (("u", 700, 3000), ("l", 150, 14), ("g", 1200, 8192), ("u", 5, 50), ("l", 90, 10),
                          ("u", 2000, 20000), ("g", 64, 1024)):
        if kind == "u":
            p = W._distinct_uniform(rng, n, 0, 0, side, side)
        elif kind == "l":
            full = np.array([(x, y) for y in range(side) for x in range(side)])
            p = full[rng.permutation(len(full))[:n]]
        else:
            p = W._distinct_gmm(rng, n, 0, side)
        parts.append(np.asarray(p) + np.array([x0, 0]))
        frames.append([x0, 0, x0 + side, side])
        x0 += side
    xy = np.concatenate(parts).astype(np.int32)
    off = np.concatenate([[0], np.cumsum([len(p) for p in parts])]).astype(np.int64)
    return xy, off, np.array(frames, np.int32)


@pytest.mark.parametrize("N", [1, 3, 8])
def test_dcalc_matches_brute_force_over_steps(N):
    from paper_2308_06484_amd.kdt import KineticDT
    rng = np.random.default_rng(N)
    xy, off, fr = _blocks(rng)
    B = len(off) - 1
    mv, mv_off = W._one_move_per_block(rng, 6, np.diff(off), 1, 6)
    dt = KineticDT(xy, off, fr, device=DEV)
    ref = Kinetic(xy, off, fr)
    tr = DTracker(B)
    mvd, offd = torch.from_numpy(mv).to(DEV), torch.from_numpy(mv_off).to(DEV)
    for t in range(7):
        if t > 0:
            dt.run(mvd, offd[t - 1:t].contiguous())
            ref.apply_step(mv, mv_off[t - 1])
        got = dt.dcalc(N)
        m, d, g = dcalc(ref.xy, off, N)
        assert np.array_equal(got["mind2"], m), (N, t)
        assert np.array_equal(got["diam2"], d), (N, t)
        assert got["d2_now"] == g, (N, t)
        d2, sp = tr.update(m, d, g)
        assert got["d2"] == d2
        assert np.allclose(got["spread"], sp, rtol=1e-12, atol=0), (N, t)
    assert got["mind2"][3] == (NONE if N >= 5 else got["mind2"][3])
    dt.close()


def test_dcalc_full_size_multi2048_and_arguments():
    """multi2048's 2048 blocks of 4096 points: every block against the
    oracle (brute force on host threads), then argument errors."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle.dcalc import block_values
    from paper_2308_06484_amd.kdt import KDTError, KineticDT
    w = W.multi2048(seed=3, steps=1)
    dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=DEV)
    got = dt.dcalc(4)
    off = w["pt_off"]
    sample = np.arange(0, 2048, 16)
    with ThreadPoolExecutor(max_workers=8) as ex:
        want = list(ex.map(lambda b: block_values(w["xy"][off[b]:off[b + 1]], 4), sample))
    for b, (m, d) in zip(sample, want):
        assert got["mind2"][b] == m and got["diam2"][b] == d, b
    assert got["d2_now"] == got["mind2"].min()
    for bad in (0, 9):
        with pytest.raises(KDTError):
            dt.dcalc(bad)
    dt.close()


def test_dlimit_policy_bit_exact():
    """The d-limit rule (rebuild a block whose move goes farther than d, the
    d of the latest d-calculation): both branches taken, every step equal
    to the oracle."""
    from paper_2308_06484_amd.kdt import KineticDT
    w = W.multi2048(seed=5, steps=6, blocks=16, per_block=512, side=2048, dcap=1024)
    dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=DEV)
    d = dt.dcalc(2)
    assert 0 < d["d2"] < NONE
    dt.set_policy("dlimit", tau=1.0)
    ref = Kinetic(w["xy"], w["pt_off"], w["frame"])
    mv, off = torch.from_numpy(w["mv"]).to(DEV), torch.from_numpy(w["mv_off"]).to(DEV)
    for t in range(6):
        dt.run(mv, off[t:t + 1].contiguous())
        ref.apply_step(w["mv"], w["mv_off"][t])
        assert np.array_equal(dt.query_canonical(), ref.all_dt(8)), t
    st = dt.stats()
    assert 0 < st["rebuilt"] < 6 * 16, st
    dt.close()
