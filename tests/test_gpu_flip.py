"""Move-and-flip repair (kdt_set_repair "flip"): the point moves in place
inside the kernel of its star and Lawson flips restore DT*; other moves
delete and insert.  Every step against the oracle (canonical triangles,
applied flags, positions), with the flip path taken and flipping."""
import numpy as np
import pytest
import torch

from oracle.kinetic import Kinetic
from paper_2308_06484_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def run_flip(w, waves=1, label=""):
    from paper_2308_06484_amd.kdt import KineticDT
    T = w["mv_off"].shape[0]
    dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=DEV)
    dt.set_repair("flip")
    if waves > 1:
        dt.set_block_waves(waves)
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
        assert np.array_equal(got.astype(bool), a) and np.all(got >= 0), f"{label}: flags, step {t}"
        n_app += int(a.sum())
        assert np.array_equal(dt.query_canonical(), ref.all_dt(8)), f"{label}: DT* after step {t}"
    assert np.array_equal(dt.positions(), ref.xy), label
    st = dt.stats()
    assert st["errors"] == 0 and st["applied"] == n_app, (label, st)
    dt.close()
    print(label, {k: st[k] for k in ("applied", "flipped", "flips", "fast", "rebuilt")}, flush=True)
    return st


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_flip_unit_moves(seed):
    # unit moves on a sparse set: mostly inside the kernel, flips are rare
    st = run_flip(W.lattice256(seed=seed, steps=100), label=f"lattice256 seed {seed}")
    assert st["flipped"] > 20


def test_flip_grid_blocks_and_waves():
    w = W.subset_blocks(W.grid1024(seed=4, steps=40), np.arange(0, 1024, 41), steps=40)
    st = run_flip(w, label="grid1024 subset")
    assert st["flipped"] > 0 and st["flips"] > 0
    st = run_flip(w, waves=4, label="grid1024 subset, 4 waves")
    assert st["flipped"] > 0


def test_flip_dense_cocircular_lattices():
    """Nearly full lattices: cocircular quadruples everywhere, so the flips
    are decided by the perturbation."""
    rng = np.random.default_rng(11)
    xy, off, frame = [], [0], []
    for b in range(6):
        side = 7 + b
        full = np.array([(x, y) for y in range(side) for x in range(side)])
        keep = full[rng.permutation(len(full))[: int(len(full) * 0.75)]]
        keep = keep[np.lexsort((keep[:, 0], keep[:, 1]))]
        xy.append(keep * 4 + np.array([200 * b, 0]))  # spacing 4: unit moves stay inside stars
        off.append(off[-1] + len(keep))
        frame.append([200 * b, 0, 200 * b + 4 * side, 4 * side])
    xy = np.concatenate(xy).astype(np.int32)
    sizes = np.diff(off)
    T = 50
    recs, offs, base = [], np.zeros((T, 7), np.int64), 0
    for t in range(T):
        offs[t, 0] = base
        for b in range(6):
            k = int(rng.integers(1, 6))
            r = np.zeros((k, 4), np.int32)
            r[:, 0] = rng.choice(sizes[b], size=k, replace=False)
            r[:, 1] = rng.integers(0, 4, size=k)
            r[:, 2] = rng.integers(1, 4, size=k)
            recs.append(r)
            base += k
            offs[t, b + 1] = base
    w = dict(xy=xy, pt_off=np.array(off, np.int64), frame=np.array(frame, np.int32),
             mv=np.concatenate(recs), mv_off=offs.astype(np.int32))
    st = run_flip(w, label="dense lattices")
    assert st["flipped"] > 0 and st["flips"] > 0


def test_flip_multi_moves_full_size_multi2048():
    """multi2048 at full size, 30 steps, move-and-flip: a rotating subset of
    blocks every step, every block at the end."""
    from tests.test_gpu_fullsize import rotating_parity
    w = W.multi2048(seed=2, steps=30)
    st = rotating_parity(w, 30, label="multi2048 flip", repair="flip")
    assert st["flipped"] > 0.5 * st["applied"], st
