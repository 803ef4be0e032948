"""Launch-shape autotuner for the per-step paths of libkdt.

Candidates are the launch forms of `kdt_run` and `kdt_graph_build`:
one kernel per step with 1, 2 or 4 wavefronts per block (the workgroup
size), the blocks taken in index order or most moves first, size classes
(only the blocks with at least `cut` moves get several wavefronts, the
others one -- or, with `mid`, two for the blocks from `mid` moves -- at once
on separate streams), the staging depth of the star
prefetch (0, 1 or 2 rings), the
persistent launch with 1..8 workgroups per compute unit (the LDS of an
MI355X compute unit holds 5), each either launched step by step or
captured as a HIP graph, and the fused multi-step launch.  Every candidate computes the same
triangulations (tests check this bit for bit), so the choice only changes
speed.  Each candidate is timed on its own fresh context built from a
calibration workload (a different seed from the measured one), the fastest
is returned, and the choice is cached in a JSON file keyed by the device
name and a signature of the workload's shape.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from .kdt import KineticDT

PER_STEP_CANDIDATES = (
    *({"mode": "step", "graph": g, "order": o} for o in (0, 1) for g in (False, True)),
    *({"mode": "step", "graph": g, "waves": 2, "order": 1} for g in (False, True)),
    *({"mode": "step", "graph": True, "waves": nw, "order": 0} for nw in (2, 4)),
    *({"mode": "step", "graph": g, "waves": 4, "order": 1} for g in (False, True)),
    *({"mode": "step", "graph": True, "waves": 2, "order": 1, "cut": c} for c in (24, 40)),
    *({"mode": "step", "graph": True, "waves": 4, "order": 1, "cut": c} for c in (32, 40, 48)),
    *({"mode": "step", "graph": True, "waves": 4, "order": 1, "cut": c, "mid": m} for c, m in ((40, 16), (40, 24),
                                                                                              (48, 16), (48, 24))),
    *({"mode": "step", "graph": True, "waves": w, "order": 1, "prefetch": d} for w in (2, 4) for d in (0, 2)),
)
DEFAULT_CANDIDATES = (
    *PER_STEP_CANDIDATES,
    *({"mode": "persistent", "graph": g, "per_cu": pc} for pc in (1, 2, 4, 5, 8) for g in (False, True)),
    {"mode": "fused", "graph": False},
)


def apply_form(dt, form):
    """Set a context's launch shape from a candidate's keys."""
    if form.get("per_cu"):
        dt.set_launch(form["per_cu"])
    if form.get("waves", 1) > 1:
        dt.set_block_waves(form["waves"])
    if form.get("order") or form.get("cut"):
        dt.set_block_order(form.get("order", 0), form.get("cut", 0), form.get("mid", 0))
    if "prefetch" in form:
        dt.set_prefetch(form["prefetch"])
    if form.get("repair"):
        dt.set_repair(form["repair"])


def cache_path():
    root = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(root, "paper_2308_06484_amd", "autotune.json")


def signature(w):
    sizes = np.diff(w["pt_off"])
    mps = float(w["mv_off"][0, -1] - w["mv_off"][0, 0]) if w["mv_off"].shape[0] else 0.0
    return (f"B={len(sizes)}|n_med={int(np.median(sizes))}|n_max={int(sizes.max())}"
            f"|moves_per_step={mps:.0f}")


def time_candidate(w, cand, steps, device="cuda:0", policy=None):
    """Seconds per time step of one candidate on a fresh context (policy:
    None, or (name, tau, mlp_w) as for KineticDT.set_policy)."""
    stream = torch.cuda.Stream(device=device)
    with torch.cuda.stream(stream):
        dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=device)
        if policy is not None:
            from .selector import DCALC_N
            dt.dcalc(DCALC_N)  # as in the runs the selector was trained on
            dt.set_policy(*policy)
        apply_form(dt, cand)
        mv = torch.from_numpy(w["mv"]).to(device)
        off = torch.from_numpy(np.ascontiguousarray(w["mv_off"][:steps])).to(device)
        g = dt.graph(mv, off, mode=cand["mode"]) if cand["graph"] else None
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if g is not None:
            g.launch()
        else:
            dt.run(mv, off, mode=cand["mode"])
        e1.record(stream)
        stream.synchronize()
        dt.sync()
        if g is not None:
            g.close()
        dt.close()
    return e0.elapsed_time(e1) / 1e3 / steps


def autotune(w, steps=100, candidates=DEFAULT_CANDIDATES, device="cuda:0", use_cache=True, policy=None):
    """Best launch form for workloads shaped like `w` (a calibration
    workload), under `policy` (None: repair; else (name, tau, mlp_w)).
    Returns {"mode", "graph", "per_cu"?, "s_per_step", "table"}."""
    name = torch.cuda.get_device_name(torch.device(device))
    key = f"{name}|{signature(w)}|steps={steps}|policy={policy[0] if policy else 'repair'}"
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return cache[key]
    table = []
    for cand in candidates:
        table.append(dict(cand, s_per_step=time_candidate(w, cand, steps, device, policy)))
    best = dict(min(table, key=lambda r: r["s_per_step"]))
    best["table"] = table
    if use_cache:
        cache[key] = best
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(path + ".tmp", path)
    return best
