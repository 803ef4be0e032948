"""Benchmark: point moves per second of the kinetic Delaunay repair on one GPU.

Measured configuration (the largest single-GPU workload): multi2048 --
2048 blocks of 4096 distinct uniform lattice points on [0,16384)^2
(8,388,608 points); in every time step each block moves
k = clip(Poisson(lambda_b), 1, 64) distinct points (lambda_b log-uniform
on [1, 64], fixed per block) by Pareto(1.2) distances capped at 4096
units, in one of four directions.  Per block and step the learned FP32
selector (trained on the device on another seed) picks repair (delete +
reinsert of every moved point) or rebuild; the launch form is the
autotuner's pick on that calibration workload.  Inputs (points,
triangulations, the whole move stream) are resident in device memory
before the timed region.

A "step" is one time step of Fig. 4 over all blocks.  `value` counts
applied moves (blocked moves are not counted) per second of the timed
region.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
    python bench.py --copy-probe          # plain copy kernel for counter scaling
    python bench.py --workload grid1024   # secondary reports (also lattice256,
                                          # uneven4096, selector_mix, global4m)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "point moves/sec (delete+reinsert, bit-exact) at 1 MI355X; % HBM roofline"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kdt.hip", "kdt_device.hpp", "kdt_pbuild.hpp", "kdt_mlp.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2308_06484_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(form, workload):
    """HBM bytes per time step of a launch form (summed over the step's
    kernels) from the committed rocprofv3 counter summary, or None if that
    form was not profiled or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"step_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_sha256_16") != source_hash():
        return None
    # a graph replays the same kernels: the form's traffic with or without one
    want = form_name(dict(form, graph=False))
    for name, rec in d.get("forms", {}).items():
        if name.removesuffix("_graph") == want:
            return rec["traffic_bytes_per_step"]
    return None


def step_kernels(form, policy):
    """The kernels one time step of a launch form runs, in launch order
    (the two size classes of a split launch run at the same time)."""
    if form["mode"] == "fused":
        return ["k_run_fused"]
    ks = []
    if form["mode"] == "persistent":
        ks = ["k_step_persist"]
    else:
        w = form.get("waves", 1)
        if form.get("order") or form.get("cut"):
            ks.append("k_order")
        if w > 1:
            ks.append(f"k_step_mw<{w}>")
        if form.get("mid"):
            ks.append("k_step_mw<2>")
        if w == 1 or form.get("cut"):
            ks.append("k_step")
        if w > 1:
            ks.append("k_step_rest")
    if policy[0] != "repair":
        ks.append("k_build_listed")
    return ks


def copy_probe():
    """A plain device copy of known size (256 MiB read + 256 MiB written),
    used to scale the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 256 << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": n, "launches": 3}), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, threads, budget_s=12.0, max_steps=16, blocks=None):
    """The CPU oracle as it stands: apply the same moves, rebuild every block
    (or every listed block) whose points changed from scratch, on `threads`
    host threads; applied moves per second of the listed blocks."""
    from oracle.kinetic import Kinetic
    from paper_2308_06484_amd import workloads as W
    if blocks is not None:
        w = W.subset_blocks(w, blocks, steps=max_steps)
    ref = Kinetic(w["xy"], w["pt_off"], w["frame"])
    t0 = time.perf_counter()
    applied, steps = 0, 0
    T = w["mv_off"].shape[0]
    while steps < min(max_steps, T) and time.perf_counter() - t0 < budget_s:
        a = ref.apply_step(w["mv"], w["mv_off"][steps])
        ref.all_dt(threads)
        applied += int(a.sum())
        steps += 1
    dt = time.perf_counter() - t0
    B = len(w["pt_off"]) - 1
    return dict(value=applied / dt, unit="point moves/s", cores=threads, kind="oracle",
                sample=f"first {steps} time steps of the same stream on {B} blocks ({applied} applied moves), "
                       f"every block rebuilt from scratch by Bowyer-Watson after each step, "
                       f"{threads} host thread{'s' if threads > 1 else ''} over blocks",
                cpu_model=cpu_model())


def time_form(w, steps, mode, graph, per_cu, dev, shape=None):
    """Seconds and applied moves of `steps` steps of w from its initial
    state under one launch form (fresh context, own stream; shape: an
    autotuner candidate's other keys)."""
    import numpy as np
    import torch

    from paper_2308_06484_amd import autotune as A
    from paper_2308_06484_amd.kdt import KineticDT
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=dev)
        if per_cu:
            dt.set_launch(per_cu)
        if shape:
            A.apply_form(dt, shape)
        mv = torch.from_numpy(w["mv"]).to(dev)
        off = torch.from_numpy(np.ascontiguousarray(w["mv_off"][:steps])).to(dev)
        g = dt.graph(mv, off, mode=mode) if graph else None
        stream.synchronize()
        a0 = dt.stats()["applied"]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if g is not None:
            g.launch()
        else:
            dt.run(mv, off, mode=mode)
        e1.record(stream)
        stream.synchronize()
        dt.sync()
        st = dt.stats()
        if g is not None:
            g.close()
        dt.close()
    return e0.elapsed_time(e1) / 1e3, st["applied"] - a0, st


def other_workload(args):
    """Secondary reports: launch forms on lattice256 / uneven4096 (with the
    autotuner's pick), the repair-or-rebuild selector on multi2048."""
    import numpy as np
    import torch

    from paper_2308_06484_amd import autotune as A
    from paper_2308_06484_amd import selector as S
    from paper_2308_06484_amd import workloads as W
    dev = "cuda:0"
    name = args.workload
    if name == "global4m":
        global_report(args)
        return
    if name == "selector_mix":
        gen = W.multi2048 if name == "multi2048" else W.selector_mix
        cal_steps = 8
        ev_steps = args.other_steps or 10
        log(f"{name}: calibration workload (seed {100 + args.seed})")
        calib = gen(seed=100 + args.seed, steps=cal_steps)
        X, Y, cal_step, cal_after = S.collect_steps(calib, cal_steps, dev)
        del calib
        wts = S.train(X, Y, epochs=300, batch=2048, lr=0.02, device=dev)
        tau = S.calibrate_threshold_cp(X, Y, cal_step, cal_after)
        log(f"trained on {len(X)} samples, tau = {tau:.3f}; evaluation workload (seed {args.seed})")
        evalw = gen(seed=args.seed, steps=ev_steps)
        res = S.evaluate(evalw, ev_steps, torch.from_numpy(wts).to(dev), tau, dev)
        desc = {"multi2048": "multi2048: 2048 blocks x 4096 uniform points on [0,16384)^2, "
                             "k ~ clip(Poisson(lambda_b),1,64) moves per block per step, Pareto(1.2) "
                             "distances capped at 4096",
                "selector_mix": "selector_mix: 256 blocks of 256 points on 1024^2 with n/2..n moves of "
                                "side/8..side/2 units per step, 256 blocks of 4096 points on 16384^2 with "
                                "1..8 moves of 1..8 units"}[name]
        out = {"workload": desc, "steps": ev_steps, "train_samples": int(len(X)), "tau": tau, "policies": res}
        for pol, r in res.items():
            log(f"{name} {pol}: {r['seconds'] * 1e3:.2f} ms, rebuilt fraction {r['rebuild_fraction']:.3f}, "
                f"chosen/best ticks {r['chosen_ticks'] / max(r['best_ticks'], 1):.3f}, "
                f"critical path chosen/best {r['cp_ticks'] / max(r['cp_best_ticks'], 1):.3f}")
        print(json.dumps(out), flush=True)
        return
    if name == "lattice256":
        w = W.lattice256(seed=args.seed, steps=args.other_steps or 100)
    else:
        w = W.uneven4096(seed=args.seed, steps=args.other_steps or 500)
    T = w["mv_off"].shape[0]
    forms = [("per_step", "step", False, None, None), ("graph_per_step", "step", True, None, None),
             ("persistent_lpt", "persistent", False, None, None),
             ("graph_persistent_lpt", "persistent", True, None, None), ("fused", "fused", False, None, None)]
    res = {}
    if name == "uneven4096":
        cal = W.uneven4096(seed=100 + args.seed, steps=60)
        best = A.autotune(cal, steps=50, use_cache=False)
        log("autotuner: " + json.dumps({k: v for k, v in best.items() if k != "table"}))
        shape = {k: best[k] for k in ("waves", "order", "cut", "mid", "prefetch") if k in best}
        forms.append(("autotuned", best["mode"], best["graph"], best.get("per_cu"), shape))
        res["autotune_table"] = best["table"]
    for fname, mode, graph, per_cu, shape in forms:
        secs, napp, st = time_form(w, T, mode, graph, per_cu, dev, shape)
        res[fname] = {"moves_per_s": napp / secs, "ms_per_step": secs * 1e3 / T, "mode": mode,
                      "graph": graph, "per_cu": per_cu, "shape": shape, "errors": st["errors"]}
        log(f"{name} {fname}: {napp / secs:.3e} moves/s, {secs * 1e3 / T:.3f} ms/step")
    sizes = np.diff(w["pt_off"])
    print(json.dumps({"workload": name, "blocks": int(len(sizes)), "points": int(sizes.sum()),
                      "steps": T, "forms": res}), flush=True)


def global_report(args):
    """Global mode on 4,194,304 points in 4096 kd cells: moves/s of the
    reservation-round repair, against rebuilding the whole DT* with the
    device builder (one rebuild per step would be the alternative)."""
    import numpy as np
    import torch

    from paper_2308_06484_amd import workloads as W
    from paper_2308_06484_amd.kdt import GlobalDT
    dev = "cuda:0"
    steps = args.other_steps or 200
    warm = min(10, steps - 1)
    t0 = time.perf_counter()
    w = W.global4m(seed=args.seed, steps=steps)
    log(f"global4m: generated in {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        G = GlobalDT(w["xy"], [0, 0, w["side"], w["side"]], w["depth"], 1 << w["depth"], device=dev)
        init_s = time.perf_counter() - t0
        mv = torch.from_numpy(np.ascontiguousarray(w["mv"])).to(dev)
        G.run(mv, w["step_off"][:warm + 1])
        stream.synchronize()
        st0 = G.stats()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        G.run(mv, w["step_off"][warm:])
        e1.record(stream)
        stream.synchronize()
        secs = e0.elapsed_time(e1) / 1e3
        st = G.stats()
        gs = G.gstats()
        applied = st["applied"] - st0["applied"]
        timed = steps - warm
        rb = []
        for _ in range(3):
            t0 = time.perf_counter()
            G.rebuild()
            rb.append(time.perf_counter() - t0)
        G.close()
        # the same timed steps replayed from a HIP graph on a fresh context
        G = GlobalDT(w["xy"], [0, 0, w["side"], w["side"]], w["depth"], 1 << w["depth"], device=dev,
                     stream=stream)
        G.run(mv, w["step_off"][:warm + 1])
        g = G.graph(mv, w["step_off"][warm:])
        stream.synchronize()
        sg0 = G.stats()
        e0.record(stream)
        g.launch()
        e1.record(stream)
        stream.synchronize()
        secs_g = e0.elapsed_time(e1) / 1e3
        applied_g = G.stats()["applied"] - sg0["applied"]
        g.close()
        G.close()
    moves_per_step = int(w["step_off"][1] - w["step_off"][0])
    out = {"workload": "global4m: one DT* of 4,194,304 uniform points on [0,65536)^2, 4096 kd cells "
                       "(median splits), one move per cell per step of 1..16 units",
           "steps_timed": timed, "warmup": warm, "moves_per_s": applied / secs,
           "ms_per_step": secs * 1e3 / timed, "applied": int(applied),
           "graph_moves_per_s": applied_g / secs_g, "graph_ms_per_step": secs_g * 1e3 / timed,
           "blocked": int(st["blocked"] - st0["blocked"]), "init_build_s": init_s,
           "full_rebuild_s": min(rb), "full_rebuild_moves_per_s": moves_per_step / min(rb),
           "speedup_vs_rebuild_per_step": (applied / secs) / (moves_per_step / min(rb)),
           "global_counters": gs}
    log(f"global4m: {applied / secs:.3e} moves/s ({secs * 1e3 / timed:.3f} ms/step), from a graph "
        f"{applied_g / secs_g:.3e} ({secs_g * 1e3 / timed:.3f} ms/step); full rebuild "
        f"{min(rb) * 1e3:.1f} ms; init {init_s:.2f} s; counters {gs}")
    print(json.dumps(out), flush=True)


def grid_report(args):
    """grid1024 (1024 blocks x 1024 points, one move per block per step): the
    launch forms, one kernel launch per step by default (secondary report)."""
    import numpy as np
    import torch

    from paper_2308_06484_amd import workloads as W
    from paper_2308_06484_amd.kdt import KineticDT

    K, Wu = args.other_steps or 980, args.warmup
    log(f"generating grid1024 with {K + Wu} steps")
    w = W.grid1024(seed=args.seed, steps=K + Wu)
    dev = torch.device("cuda:0")
    mv = torch.from_numpy(w["mv"]).to(dev)
    off_all = torch.from_numpy(w["mv_off"]).to(dev)
    off_warm = off_all[:Wu].contiguous()
    off_timed = off_all[Wu:Wu + K].contiguous()

    def fresh(stream):
        with torch.cuda.stream(stream):
            dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=dev)
            if Wu:
                dt.run(mv, off_warm)
            dt.sync()
        return dt

    # headline: one plain kernel launch per time step; HIP events around the
    # whole timed region and, for the average launch duration, pairs each
    # spanning 8 consecutive launches (kdt_timing; a pair around every launch
    # would cost the stream ~16 % of its throughput)
    stream = torch.cuda.Stream(device=dev)
    mode = "fused" if args.fused else "step"
    dt = fresh(stream)
    s0 = dt.stats()
    dt.timing(True, period=1 if mode == "fused" else 8)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        t_host = time.perf_counter()
        e0.record(stream)
        dt.run(mv, off_timed, mode=mode)
        e1.record(stream)
        stream.synchronize()
        t_host = time.perf_counter() - t_host
    ms = e0.elapsed_time(e1)
    kern_ms, launches = dt.timing_read()
    dt.timing(False)
    dt.sync()
    s1 = dt.stats()
    dt.close()

    # the other launch forms on fresh contexts, same stream of moves
    variants = {}
    for name, vmode, graph, per_cu in [] if args.no_variants else [("graph_per_step", "step", True, None),
                                       ("persistent_lpt", "persistent", False, None),
                                       ("graph_persistent_lpt", "persistent", True, None),
                                       ("fused", "fused", False, None)]:
        d2 = fresh(stream)
        if per_cu:
            d2.set_launch(per_cu)
        a0 = d2.stats()["applied"]
        with torch.cuda.stream(stream):
            g = d2.graph(mv, off_timed, mode=vmode) if graph else None
            stream.synchronize()
            f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            f0.record(stream)
            if g is not None:
                g.launch()
            else:
                d2.run(mv, off_timed, mode=vmode)
            f1.record(stream)
            stream.synchronize()
        vms = f0.elapsed_time(f1)
        d2.sync()
        napp = d2.stats()["applied"] - a0
        variants[name] = {"moves_per_s": napp / (vms / 1e3), "ms_per_step": vms / K}
        log(f"variant {name}: {vms:.2f} ms, {napp / (vms / 1e3):.3e} moves/s")
        if g is not None:
            g.close()
        d2.close()

    # the alternative the paper weighs against updating (Sec. I): rebuild
    # every block from scratch after each step, on the first steps of the
    # same stream
    if not args.no_variants:
        R = min(20, K)
        d2 = fresh(stream)
        d2.set_policy("rebuild")
        a0 = d2.stats()["applied"]
        off_r = off_timed[:R].contiguous()
        with torch.cuda.stream(stream):
            f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            f0.record(stream)
            d2.run(mv, off_r)
            f1.record(stream)
            stream.synchronize()
        vms = f0.elapsed_time(f1)
        d2.sync()
        napp = d2.stats()["applied"] - a0
        variants["full_rebuild_per_step"] = {"moves_per_s": napp / (vms / 1e3), "ms_per_step": vms / R,
                                             "steps": R}
        log(f"variant full_rebuild_per_step: {vms:.2f} ms for {R} steps, {napp / (vms / 1e3):.3e} moves/s")
        d2.close()

    applied = s1["applied"] - s0["applied"]
    blocked = s1["blocked"] - s0["blocked"]
    alg = s1["alg_bytes"] - s0["alg_bytes"]
    touched = s1["tri_touched"] - s0["tri_touched"]
    value = applied / (ms / 1e3)
    n_launch = 1 if mode == "fused" else K  # kernel launches in the timed region
    avg_launch_s = kern_ms / 1e3 / max(1, launches)  # over the launches the pairs span
    achieved = alg / n_launch / avg_launch_s / 1e9
    log(f"timed {K} steps: {ms:.2f} ms (host {t_host * 1e3:.1f} ms), kernels {kern_ms:.2f} ms over "
        f"{launches} launches in event pairs of 8 ({avg_launch_s * 1e6:.2f} us each), applied {applied}, blocked {blocked}")
    khz = max(1, s1["clock_khz"])
    phases = {ph: (s1["t_" + ph] - s0["t_" + ph]) / khz * 1e3 / max(1, applied)
              for ph in ("star", "locate", "hole", "insert")}
    log("per applied move, us of one wavefront: " + ", ".join(f"{k} {v:.2f}" for k, v in phases.items())
        + f"; mean degree {(s1['star_sum'] - s0['star_sum']) / max(1, applied):.2f}"
        + f", mean cavity {(s1['cavity_sum'] - s0['cavity_sum']) / max(1, applied):.2f}"
        + f", mean walk {(s1['walk_sum'] - s0['walk_sum']) / max(1, applied + blocked):.2f}"
        + f", star-only path {(s1['fast'] - s0['fast']) / max(1, applied):.3f}")
    hist = [a - b for a, b in zip(s1["hist"], s0["hist"])]
    log("move time histogram (us upper edge: count): " + ", ".join(
        f"{(2 ** (i + 1)) / khz * 1e3:.2f}: {c}" for i, c in enumerate(hist) if c))
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "point moves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wu,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": "grid1024: 1024 blocks = 32x32 cells of 2048^2 over [0,65536)^2, "
                        "1024 distinct uniform lattice points per block, one move per block per "
                        "time step of 1-8 units in one of 4 directions, "
                        + ("all steps in one fused launch" if args.fused else "one kernel launch per time step"),
            "blocks": 1024,
            "points_per_block": 1024,
            "moves_per_step": 1024,
            "seed": args.seed,
        },
        "applied_moves": applied,
        "variants": variants,
        "phase_us_per_move": phases,
        "move_time_hist": {f"<{(2 ** (i + 1)) / khz * 1e3:.2f}us": c
                           for i, c in enumerate([a - b for a, b in zip(s1["hist"], s0["hist"])]) if c},
        "blocked_moves": blocked,
        "mtri_touched_per_s": touched / (ms / 1e3) / 1e6,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic({"mode": "fused" if args.fused else "step", "graph": False}, "grid1024"),
            "kernel": "k_run_fused" if args.fused else "k_step",
            "avg_launch_us": avg_launch_s * 1e6,
            "alg_bytes_per_launch": alg / n_launch,
            "timed_launches": launches,
        },
    }
    if not args.no_cpu_baseline:
        threads = min(16, len(os.sched_getaffinity(0)))
        log(f"cpu baseline (oracle) on {threads} threads")
        res["cpu_baseline"] = cpu_baseline(w, threads)
    print(json.dumps(res), flush=True)



def headline_forms():
    from paper_2308_06484_amd import autotune as A
    return (
        *A.PER_STEP_CANDIDATES,
        *({"mode": "persistent", "graph": False, "per_cu": pc} for pc in (2, 4, 8)),
        {"mode": "fused", "graph": False},
    )
CAL_STEPS = 6


def form_name(f):
    n = {"step": "per_step", "persistent": "persistent", "fused": "fused"}[f["mode"]]
    if f.get("per_cu"):
        n += f"_{f['per_cu']}wg"
    if f.get("waves", 1) > 1:
        n += f"_{f['waves']}waves"
    if f.get("order"):
        n += "_ordered"
    if f.get("cut"):
        n += f"_cut{f['cut']}"
    if f.get("mid"):
        n += f"_mid{f['mid']}"
    if "prefetch" in f:
        n += f"_depth{f['prefetch']}"
    if f.get("repair"):
        n += "_" + f["repair"]
    return n + ("_graph" if f.get("graph") else "")


def timed_run(w, mv, off_warm, off_timed, form, policy, dev, period=0):
    """One fresh context: warm-up steps, then the timed steps under one
    launch form and policy ((name, tau, mlp_w)), HIP events on the
    library's stream around the timed region.  Returns the region's
    milliseconds and the counters before and after."""
    import torch

    from paper_2308_06484_amd import autotune as A
    from paper_2308_06484_amd import selector as S
    from paper_2308_06484_amd.kdt import KineticDT
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=dev, stream=stream)
        dt.dcalc(S.DCALC_N)  # d of the initial positions: the selector's feature 15, the d-limit rule
        dt.set_policy(*policy)
        A.apply_form(dt, form)
        if off_warm is not None and off_warm.shape[0]:
            dt.run(mv, off_warm, mode=form["mode"])
        dt.sync()
        g = dt.graph(mv, off_timed, mode=form["mode"]) if form.get("graph") else None
        stream.synchronize()
        s0 = dt.stats()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if g is not None:
            g.launch()
        else:
            dt.run(mv, off_timed, mode=form["mode"])
        e1.record(stream)
        stream.synchronize()
        dt.sync()
        s1 = dt.stats()
        if g is not None:
            g.close()
        dt.close()
    return e0.elapsed_time(e1), s0, s1


def headline(args):
    import numpy as np
    import torch

    from paper_2308_06484_amd import autotune as A
    from paper_2308_06484_amd import selector as S
    from paper_2308_06484_amd import workloads as W
    dev = "cuda:0"
    K, Wu = args.steps, args.warmup
    # the selector: trained on the device on a calibration workload of
    # another seed (forced-repair and forced-rebuild runs give both costs)
    t0 = time.perf_counter()
    cal = W.multi2048(seed=100 + args.seed, steps=CAL_STEPS)
    X, Y, cal_step, cal_after = S.collect_steps(cal, CAL_STEPS, dev)
    mlp = torch.from_numpy(S.train(X, Y, epochs=200, batch=2048, lr=0.02, device=dev)).to(dev)
    tau = S.calibrate_threshold_cp(X, Y, cal_step, cal_after)  # on the step's critical path
    tau_d = S.calibrate_threshold_cp(X, Y, cal_step, cal_after, feature=15)  # the d-limit rule's
    tau_sum = S.calibrate_threshold(X, Y)           # on summed block costs, for comparison
    log(f"selector trained on {len(X)} block-steps of seed {100 + args.seed} "
        f"({time.perf_counter() - t0:.1f} s); threshold tau = {tau:.3g} on the critical path, "
        f"{tau_sum:.3g} on summed costs; d-limit tau = {tau_d:.3g} (3e+38: never rebuild)")
    pol_mlp = ("mlp", 0.0, mlp)
    if args.form:  # a fixed launch form (profiling runs): a candidate's name
        forms = {form_name(f): f for f in headline_forms()}
        forms.update(step={"mode": "step", "graph": False}, step_graph={"mode": "step", "graph": True},
                     fused={"mode": "fused", "graph": False})
        if args.form not in forms:
            sys.exit(f"--form: one of {', '.join(sorted(forms))}")
        form = forms[args.form]
        autotune_table = None
    else:
        best = A.autotune(cal, steps=CAL_STEPS, candidates=headline_forms(), device=dev, use_cache=False,
                          policy=pol_mlp)
        form = {k: best[k] for k in ("mode", "graph", "per_cu", "waves", "order", "cut", "mid", "prefetch")
                if k in best}
        autotune_table = {form_name(r): r["s_per_step"] * 1e3 for r in best["table"]}
        log("autotuner (calibration workload, MLP policy): " + ", ".join(
            f"{form_name(r)} {r['s_per_step'] * 1e3:.3f} ms" for r in best["table"]) + f" -> {form_name(form)}")
    del cal
    t0 = time.perf_counter()
    w = W.multi2048(seed=args.seed, steps=Wu + K)
    log(f"multi2048 seed {args.seed}, {Wu} warm-up + {K} timed steps generated in {time.perf_counter() - t0:.1f} s")
    mv = torch.from_numpy(w["mv"]).to(dev)
    off_all = torch.from_numpy(w["mv_off"]).to(dev)
    off_warm = off_all[:Wu].contiguous()
    off_timed = off_all[Wu:Wu + K].contiguous()

    ms, s0, s1 = timed_run(w, mv, off_warm, off_timed, form, pol_mlp, dev)
    applied = s1["applied"] - s0["applied"]
    blocked = s1["blocked"] - s0["blocked"]
    alg = s1["alg_bytes"] - s0["alg_bytes"]
    touched = s1["tri_touched"] - s0["tri_touched"]
    rebuilt = s1["rebuilt"] - s0["rebuilt"]
    value = applied / (ms / 1e3)
    log(f"headline ({form_name(form)}, MLP): {ms:.2f} ms for {K} steps, {value:.4e} moves/s, "
        f"{applied} applied, {blocked} blocked, {rebuilt} block-steps rebuilt")

    variants = {}
    if not args.no_variants:
        # the other launch forms the schedule is built from, one per idea (the
        # autotuner's table above times every candidate on the calibration
        # workload)
        shown = [{"mode": "step", "graph": False}, {"mode": "step", "graph": False, "order": 1},
                 {"mode": "step", "graph": False, "waves": 2, "order": 1},
                 {"mode": "step", "graph": True, "waves": 4, "order": 0},
                 {"mode": "step", "graph": False, "waves": 4, "order": 1},
                 {"mode": "step", "graph": True, "waves": 4, "order": 1},
                 {"mode": "step", "graph": True, "waves": 4, "order": 1, "cut": 32},
                 {"mode": "step", "graph": True, "waves": 4, "order": 1, "cut": 40, "mid": 16},
                 {"mode": "step", "graph": True, "waves": 4, "order": 1, "prefetch": 0},
                 {"mode": "persistent", "graph": False, "per_cu": 8}, {"mode": "fused", "graph": False}]
        runs = [(form_name(f) + "_mlp", f, pol_mlp, K) for f in shown if f != form]
        runs += [(form_name(form) + "_repair_only", form, ("repair", 0.0, None), K),
                 ("per_step_repair_only", {"mode": "step", "graph": False}, ("repair", 0.0, None), K),
                 (form_name(form) + "_threshold", form, ("threshold", tau, None), K),
                 (form_name(form) + "_threshold_summed_tau", form, ("threshold", tau_sum, None), K),
                 (form_name(form) + "_dlimit", form, ("dlimit", tau_d, None), K),
                 (form_name(form) + "_dlimit_tau1", form, ("dlimit", 1.0, None), K),
                (form_name(dict(form, repair="flip")) + "_mlp", dict(form, repair="flip"), pol_mlp, K),
                 ("per_step_rebuild_only", {"mode": "step", "graph": False}, ("rebuild", 0.0, None), min(10, K))]
        for name, f, pol, steps in runs:
            if name in variants:
                continue
            vms, a0, a1 = timed_run(w, mv, off_warm, off_timed[:steps].contiguous(), f, pol, dev)
            napp = a1["applied"] - a0["applied"]
            variants[name] = {"moves_per_s": napp / (vms / 1e3), "ms_per_step": vms / steps, "steps": steps,
                              "rebuilt_block_steps": a1["rebuilt"] - a0["rebuilt"]}
            log(f"variant {name}: {vms / steps:.3f} ms/step, {napp / (vms / 1e3):.4e} moves/s")

    # the paper's d-calculation and N-spread (Sec. III) of the evaluation
    # workload's initial and final positions, with the kernel's time
    dcal = {}
    if not args.no_variants:
        from paper_2308_06484_amd.kdt import KineticDT
        stream = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(stream):
            dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=dev, stream=stream)
            first = dt.dcalc(S.DCALC_N)
            dt.run(mv, off_all)
            t0 = time.perf_counter()
            last = dt.dcalc(S.DCALC_N)
            secs = time.perf_counter() - t0
            dt.close()
        dcal = {"N": S.DCALC_N, "mindistance_start": float(np.sqrt(first["d2_now"])),
                "mindistance_end": float(np.sqrt(last["d2_now"])), "d": float(np.sqrt(last["d2"])),
                "max_n_spread": float(last["spread"].max()), "median_n_spread": float(np.median(last["spread"])),
                "dcalc_ms": secs * 1e3}
        log(f"d-calculation (N = {S.DCALC_N}): mindistance {dcal['mindistance_start']:.2f} at the start, "
            f"{dcal['mindistance_end']:.2f} after {Wu + K} steps, d = {dcal['d']:.2f}, N-spread up to "
            f"{dcal['max_n_spread']:.1f}; {secs * 1e3:.2f} ms per call")

    # roofline of the step: the timed region spans K launches of the form's
    # step kernel (one launch in the fused form), so its average duration is
    # the region over the launches, gaps and the selector's follow-up
    # launches included: an upper bound of the kernel's own duration
    n_launch = 1 if form["mode"] == "fused" else K
    kernels = step_kernels(form, pol_mlp)
    avg_launch_s = ms / 1e3 / n_launch
    achieved = alg / n_launch / avg_launch_s / 1e9
    khz = max(1, s1["clock_khz"])
    phases = {ph: (s1["t_" + ph] - s0["t_" + ph]) / khz * 1e3 / max(1, applied)
              for ph in ("star", "locate", "hole", "insert")}
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "point moves/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wu,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": "multi2048: 2048 blocks x 4096 distinct uniform lattice points on [0,16384)^2, "
                        "per block and time step k = clip(Poisson(lambda_b), 1, 64) movers (lambda_b "
                        "log-uniform on [1,64]) by Pareto(1.2) distances capped at 4096, 4 directions; "
                        "per-block repair-or-rebuild choice by the FP32 MLP 16-32-32-2 trained on the "
                        f"device on seed {100 + args.seed}; launch form {form_name(form)} (autotuner)",
            "blocks": 2048,
            "points_per_block": 4096,
            "moves_per_step": round((applied + blocked) / K),
            "seed": args.seed,
        },
        "applied_moves": applied,
        "blocked_moves": blocked,
        "rebuilt_block_steps": rebuilt,
        "variants": variants,
        "selector_taus": {"threshold_critical_path": tau, "threshold_summed": tau_sum, "dlimit": tau_d},
        "autotune_ms_per_step": autotune_table,
        "d_calculation": dcal,
        "phase_us_per_move": phases,
        "mtri_touched_per_s": touched / (ms / 1e3) / 1e6,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (measured_traffic(form, "multi2048") * K / n_launch
                        if measured_traffic(form, "multi2048") is not None else None),
            # the unit is one time step: its kernels (the size classes of a
            # split launch at the same time), gaps between them included
            "kernel": " + ".join(kernels),
            "avg_launch_us": avg_launch_s * 1e6,
            "alg_bytes_per_launch": alg / n_launch,
            "timed_launches": n_launch,
        },
    }
    if not args.no_cpu_baseline:
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        log(f"cpu baseline (oracle) on {threads} threads, all blocks")
        res["cpu_baseline"] = cpu_baseline(w, threads, budget_s=12.0, max_steps=16)
        # the paper's comparison with the serial form: one thread against
        # all of them, on the same 64 blocks
        sub = np.arange(0, 2048, 32)
        log("cpu baseline: serial form (1 thread) and all threads on 64 blocks")
        ser = cpu_baseline(w, 1, budget_s=6.0, max_steps=16, blocks=sub)
        par = cpu_baseline(w, threads, budget_s=6.0, max_steps=16, blocks=sub)
        res["cpu_baseline"]["serial_form"] = {"value": ser["value"], "cores": 1, "sample": ser["sample"]}
        res["cpu_baseline"]["parallel_same_sample"] = {"value": par["value"], "cores": threads,
                                                       "sample": par["sample"]}
        log(f"cpu: {res['cpu_baseline']['value']:.4e} moves/s on {threads} threads; serial form "
            f"{ser['value']:.4e}, {threads} threads {par['value']:.4e} on 64 blocks")
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fused", action="store_true", help="grid1024 report: time the fused launch instead")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the other launch forms and policies")
    ap.add_argument("--workload", default="multi2048",
                    choices=["multi2048", "grid1024", "lattice256", "uneven4096", "selector_mix", "global4m"],
                    help="multi2048 is the measured configuration; the others print a secondary report")
    ap.add_argument("--other-steps", type=int, default=0, help="steps for the secondary reports")
    ap.add_argument("--form", default=None,
                    help="headline: this launch form (step, step_graph, fused or an autotuner "
                         "candidate's name such as per_step_2waves_ordered_graph) instead of the "
                         "autotuner's pick (profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(blocks are independent: sharding them over GPUs needs no exchange)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.workload == "multi2048":
        headline(args)
    elif args.workload == "grid1024":
        grid_report(args)
    else:
        other_workload(args)


if __name__ == "__main__":
    main()
