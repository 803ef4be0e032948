"""Launch forms (one kernel per step, persistent, fused, HIP graph replay,
several wavefronts per block, blocks most moves first, size classes on two
streams, the star prefetch off) and the autotuner: every form gives the same
triangulations, bit for bit, as the oracle, under the repair and the rebuild
policies."""
import numpy as np
import pytest
import torch

from oracle.kinetic import Kinetic
from paper_2308_06484_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _run(w, mode, graph=False, per_cu=None, repeat=1, policy=None, shape=None):
    from paper_2308_06484_amd.autotune import apply_form
    from paper_2308_06484_amd.kdt import KineticDT
    stream = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(stream):
        dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=DEV)
        if per_cu:
            dt.set_launch(per_cu)
        if shape:
            apply_form(dt, shape)
        if policy:
            dt.set_policy(policy)
        mv = torch.from_numpy(w["mv"]).to(DEV)
        off = torch.from_numpy(w["mv_off"]).to(DEV)
        applied = torch.zeros(w["mv"].shape[0], dtype=torch.int8, device=DEV)
        if graph:
            g = dt.graph(mv, off, applied=applied, mode=mode)
            for _ in range(repeat):
                g.launch()
        else:
            for _ in range(repeat):
                dt.run(mv, off, applied=applied, mode=mode)
        stream.synchronize()
        out = (dt.query_canonical(), dt.positions(), applied.cpu().numpy(), dt.stats())
        if graph:
            g.close()
        dt.close()
    return out


@pytest.fixture(scope="module")
def uneven():
    return W.uneven4096(seed=21, steps=25, blocks=24, nmax=3000)


def test_launch_forms_bit_identical(uneven):
    w = uneven
    ref = _run(w, "step")
    oracle = Kinetic(w["xy"], w["pt_off"], w["frame"])
    app = np.concatenate([oracle.apply_step(w["mv"], w["mv_off"][t]) for t in range(w["mv_off"].shape[0])])
    assert np.array_equal(ref[0], oracle.all_dt(8))
    assert np.array_equal(ref[1], oracle.xy)
    assert np.array_equal(ref[2].astype(bool), app)
    for mode, graph, per_cu in [("persistent", False, 1), ("persistent", False, 3), ("fused", False, None),
                                ("step", True, None), ("persistent", True, 2)]:
        got = _run(w, mode, graph, per_cu)
        assert np.array_equal(got[0], ref[0]), (mode, graph, per_cu)
        assert np.array_equal(got[1], ref[1]), (mode, graph, per_cu)
        assert np.array_equal(got[2], ref[2]), (mode, graph, per_cu)
        assert got[3]["applied"] == ref[3]["applied"] and got[3]["errors"] == 0
    for graph, shape in [(False, {"order": 1}), (True, {"waves": 2, "order": 1}), (False, {"waves": 4, "order": 1}),
                         (True, {"waves": 4, "order": 1, "cut": 3}), (False, {"waves": 2, "order": 1, "cut": 2}),
                         (True, {"order": 1, "prefetch": 0}), (False, {"waves": 2, "order": 1, "prefetch": 2}),
                         (True, {"waves": 4, "order": 1, "cut": 4, "mid": 2})]:
        got = _run(w, "step", graph, shape=shape)
        for i in range(3):
            assert np.array_equal(got[i], ref[i]), (graph, shape, i)
        assert got[3]["applied"] == ref[3]["applied"] and got[3]["errors"] == 0


def test_graph_replays_apply_the_stream_again(uneven):
    w = uneven
    a = _run(w, "step", repeat=2)
    b = _run(w, "persistent", graph=True, per_cu=2, repeat=2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # the split launch's fork and join replayed
    c = _run(w, "step", graph=True, repeat=2, shape={"waves": 2, "order": 1, "cut": 3})
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    c = _run(w, "step", graph=True, repeat=2, shape={"waves": 4, "order": 1, "cut": 3, "mid": 2})
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    oracle = Kinetic(w["xy"], w["pt_off"], w["frame"])
    for _ in range(2):
        for t in range(w["mv_off"].shape[0]):
            oracle.apply_step(w["mv"], w["mv_off"][t])
    assert np.array_equal(a[0], oracle.all_dt(8))


def test_autotune_returns_a_timed_candidate(tmp_path, monkeypatch):
    from paper_2308_06484_amd import autotune as A
    monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path))
    w = W.grid1024(seed=101, steps=12, cells=8, per_block=512, cell=1024)
    best = A.autotune(w, steps=10)
    assert best["mode"] in ("step", "persistent", "fused") and best["s_per_step"] > 0
    assert len(best["table"]) == len(A.DEFAULT_CANDIDATES)
    again = A.autotune(w, steps=10)  # served from the cache
    assert again["mode"] == best["mode"] and again["s_per_step"] == best["s_per_step"]


def test_rebuild_policy_in_every_launch_form(uneven):
    """Blocks of 64..3000 points: the small ones are rebuilt inside the step
    kernel, the large ones by the build kernel launched after it (recorded
    in the graph too); every form matches the oracle."""
    w = uneven
    oracle = Kinetic(w["xy"], w["pt_off"], w["frame"])
    app = np.concatenate([oracle.apply_step(w["mv"], w["mv_off"][t]) for t in range(w["mv_off"].shape[0])])
    for mode, graph, per_cu in [("step", False, None), ("step", True, None), ("persistent", True, 2),
                                ("fused", False, None)]:
        got = _run(w, mode, graph, per_cu, policy="rebuild")
        assert np.array_equal(got[0], oracle.all_dt(8)), (mode, graph)
        assert np.array_equal(got[1], oracle.xy), (mode, graph)
        assert np.array_equal(got[2].astype(bool), app), (mode, graph)
        assert got[3]["errors"] == 0 and got[3]["rebuilt"] > 0


def test_timing_pairs_span_runs_of_launches(uneven):
    """kdt_timing(P): event pairs over runs of P consecutive launches; a run
    cut short is closed by the read, and every launch is counted once."""
    from paper_2308_06484_amd.kdt import KineticDT
    w = uneven
    stream = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(stream):
        dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=DEV)
        mv = torch.from_numpy(w["mv"]).to(DEV)
        off = torch.from_numpy(w["mv_off"]).to(DEV)
        T = w["mv_off"].shape[0]
        for period in (1, 4, T + 3):
            dt.timing(True, period=period)
            dt.run(mv, off)
            ms, n = dt.timing_read()
            assert n == T and ms > 0, (period, n, ms)
        dt.timing(False)
        dt.close()
