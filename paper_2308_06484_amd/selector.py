"""Training and evaluation driver of the repair-or-rebuild selector.

The paper weighs updating the triangulation against rebuilding it when
points move far (Sec. I, abstract).  Here that choice is made per block and
time step by a small network (16 -> 32 -> 32 -> 2) that predicts the log2
device-clock cost of each branch from the block's features; a threshold on
the summed move distance (in units of the block's point spacing), or on the
longest move against d of the d-calculation, is the fallback.  Every block of
a step runs at once, so a step lasts as long as its slowest block: choosing
the cheaper branch for every block also minimises each step's slowest block,
so the network predicts per-block costs, while the thresholds are calibrated
and the choices are judged on that critical path (the sum over steps of the
slowest block's cost, plus the slowest rebuild too large for the step's
kernel, which runs after it).  Features, costs and branch choices are
produced by the library's kernels (the per-step log), and the network is
trained by the library's own forward/backward/SGD kernels; this module only
arranges the runs, the feature normalisation (folded into the first layer
afterwards) and the bookkeeping of the regret.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from .kdt import LOG_FIELDS, MLP_NOALLOC_BATCH, MLP_PARAMS, KineticDT, mlp_train, mlp_train_noalloc

H, IN = 32, 16


DCALC_N = 4  # N of the d-calculation whose d feeds feature 15 and the d-limit rule


def run_policy(w, steps, policy, device="cuda:0", tau=0.0, mlp_w=None, log=True):
    """Run the workload's first `steps` steps under one policy from its
    initial state (after one d-calculation of the initial positions).
    Returns (log [steps, B, LOG_FIELDS] numpy or None, seconds, stats)."""
    dt = KineticDT(w["xy"], w["pt_off"], w["frame"], device=device)
    dt.dcalc(DCALC_N)
    dt.set_policy(policy, tau, mlp_w)
    lg = dt.set_log(steps) if log else None
    mv = torch.from_numpy(w["mv"]).to(device)
    off = torch.from_numpy(np.ascontiguousarray(w["mv_off"][:steps])).to(device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dt.run(mv, off)
    dt.sync()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    st = dt.stats()
    out = lg.cpu().numpy() if lg is not None else None
    dt.close()
    return out, secs, st


def collect_steps(w, steps, device="cuda:0"):
    """Training samples: features and the log2 cost of both branches for
    every (step, block) with moves, from a forced-repair and a forced-rebuild
    run of the same workload (identical states: DT* is unique), the step of
    each sample, and whether its rebuild would run after the step's kernel."""
    lr_, _, _ = run_policy(w, steps, "repair", device)
    lb_, _, _ = run_policy(w, steps, "rebuild", device)
    # block-steps with moves; a repair that hit the repair path's capacity
    # and finished by rebuilding (branch 2) has no clean cost: left out
    valid = (lr_[..., 18] > 0) & (lr_[..., 16] != 2)
    X = lr_[..., :IN][valid].astype(np.float32)
    Y = np.stack([np.log2(np.maximum(lr_[..., 17][valid], 1.0)),
                  np.log2(np.maximum(lb_[..., 17][valid], 1.0))], axis=1).astype(np.float32)
    step = np.nonzero(valid)[0]
    after = lb_[..., 19][valid] > 0.5
    return X, Y, step, after


def collect(w, steps, device="cuda:0"):
    X, Y, _, _ = collect_steps(w, steps, device)
    return X, Y


def init_weights(seed=0):
    """He-uniform initialisation, zero biases (float32 [MLP_PARAMS])."""
    rng = np.random.default_rng(seed)
    w = np.zeros(MLP_PARAMS, dtype=np.float32)
    o = 0
    for fan_in, fan_out in ((IN, H), (H, H), (H, 2)):
        lim = np.sqrt(6.0 / fan_in)
        w[o:o + fan_in * fan_out] = rng.uniform(-lim, lim, fan_in * fan_out)
        o += fan_in * fan_out + fan_out
    return w


def fold_normalisation(w, mu, sd):
    """Weights for raw features from weights trained on (x - mu) / sd."""
    w = w.astype(np.float64).copy()
    W1 = w[:H * IN].reshape(H, IN)
    b1 = w[H * IN:H * IN + H]
    W1n = W1 / sd[None, :]
    b1n = b1 - W1n @ mu
    w[:H * IN] = W1n.reshape(-1)
    w[H * IN:H * IN + H] = b1n
    return w.astype(np.float32)


# Features the network does not see: 15 (max d over d of the d-calculation)
# divides by a minimum over the whole point set, an extreme value that
# changes from one data set to the next (on selector_mix, d = 17 for one seed
# and 7.6 for another): a network trained on one set would read the other's
# blocks as moving more than twice as far.  The d-limit rule uses it.
NET_DROP = (15,)


def train(X, Y, epochs=200, batch=4096, lr=0.02, seed=0, device="cuda:0", drop=NET_DROP):
    """Train on the device (the library's kernels) and return float32
    weights for raw features.  The features in `drop` are held at zero
    during training and their first-layer weights set to zero, so the
    network ignores them."""
    mu = X.mean(axis=0).astype(np.float64)
    sd = X.std(axis=0).astype(np.float64)
    sd[sd < 1e-6] = 1.0  # constant features: centred to zero, left unscaled
    Xn = ((X - mu) / sd).astype(np.float32)
    drop = list(drop)
    Xn[:, drop] = 0.0
    ym = Y.mean(axis=0)
    Yc = (Y - ym).astype(np.float32)
    w0 = init_weights(seed)
    w0[-2:] = 0.0
    w0[:H * IN].reshape(H, IN)[:, drop] = 0.0
    wt = torch.from_numpy(w0).to(device)
    xt = torch.from_numpy(Xn).to(device)
    yt = torch.from_numpy(Yc).to(device)
    # the same floats either way; the no-alloc path spreads a batch over
    # one workgroup per 64 samples
    (mlp_train_noalloc if batch <= MLP_NOALLOC_BATCH else mlp_train)(wt, xt, yt, epochs, batch, lr)
    torch.cuda.synchronize()
    w = wt.cpu().numpy()
    w[-2:] += ym.astype(np.float32)  # output bias back to the label scale
    w[:H * IN].reshape(H, IN)[:, drop] = 0.0  # (their gradient was zero: still zero)
    return fold_normalisation(w, mu, sd)


def step_time(cost, step, after=None):
    """The blocks of a step run at once, so the step's kernel lasts as long
    as its slowest block; rebuilds too large for that kernel run after it
    (at once too): the sum over steps of the slowest block's cost in the
    kernel plus the slowest of those after it.  after: bool per sample, or
    None (all in the kernel)."""
    n = int(step.max()) + 1 if len(step) else 0
    during, later = np.zeros(n), np.zeros(n)
    late = np.zeros(len(cost), dtype=bool) if after is None else np.asarray(after, dtype=bool)
    np.maximum.at(during, step[~late], cost[~late])
    np.maximum.at(later, step[late], cost[late])
    return float(during.sum() + later.sum())


NEVER = 3.0e38  # a threshold no feature value exceeds: the rule never rebuilds


def calibrate_threshold_cp(X, Y, step, after=None, candidates=256, feature=3):
    """tau for "rebuild iff feature > tau" (feature 3: sum d/s, the threshold
    rule; 15: max d / d, the d-limit rule) that minimises the step time of
    step_time -- the critical path -- on the samples (candidates: quantiles
    of the observed values, rebuild everything, rebuild nothing).  A choice
    that makes one block of a step slower costs the whole step; per-block
    sums would not see it.  after: per sample, whether its rebuild would run
    after the step's kernel (None: none would).  Of equally good candidates
    the largest is kept: on unseen blocks it rebuilds least, and a needless
    rebuild costs far more than a missed one; when rebuilding no sample is
    best, no rebuild paid on the samples and the rule never rebuilds
    (NEVER), rather than rebuilding the first unseen larger value."""
    f = X[:, feature].astype(np.float64)
    cr, cb = np.exp2(Y[:, 0].astype(np.float64)), np.exp2(Y[:, 1].astype(np.float64))
    late = np.zeros(len(f), dtype=bool) if after is None else np.asarray(after, dtype=bool)
    cand = np.unique(np.concatenate([np.quantile(f, np.linspace(0, 1, candidates)), [f.min() - 1.0, f.max() + 1.0]]))
    best_tau, best = float(f.max() + 1.0), np.inf
    for tau in cand[::-1]:
        rb = f > tau
        t = step_time(np.where(rb, cb, cr), step, rb & late)
        if t < best:
            best, best_tau = t, float(tau)
    return NEVER if best_tau >= f.max() else best_tau


def calibrate_threshold(X, Y):
    """tau for the rule "rebuild iff sum d/s > tau" that minimises the
    summed cost on the samples (candidates: the observed values)."""
    f = X[:, 3].astype(np.float64)
    cr, cb = np.exp2(Y[:, 0].astype(np.float64)), np.exp2(Y[:, 1].astype(np.float64))
    order = np.argsort(f)
    fs, crs, cbs = f[order], cr[order], cb[order]
    # choose the split index i: repair for the first i samples, rebuild after
    cum_r = np.concatenate([[0.0], np.cumsum(crs)])
    cum_b = np.concatenate([[0.0], np.cumsum(cbs[::-1])])[::-1]
    total = cum_r + cum_b
    i = int(np.argmin(total))
    if i >= len(fs):
        return float(fs[-1] + 1.0) if len(fs) else 0.0
    return float(fs[i - 1] if i > 0 else fs[0] - 1.0)


def regret(branch_log, cost_repair, cost_rebuild, valid):
    """Sum over (step, block) of the chosen branch's cost minus the cheaper
    one's (device ticks), and the total cost of the choices."""
    cr, cb = cost_repair[valid], cost_rebuild[valid]
    ch = branch_log[valid]
    chosen = np.where(ch == 1, cb, cr)  # 2: a repair that fell back (no clean cost): counted as repair
    best = np.minimum(cr, cb)
    return float((chosen - best).sum()), float(chosen.sum()), float(best.sum())


def evaluate(w, steps, mlp_w, tau, device="cuda:0"):
    """Wall time and regret of every policy on the workload: the summed
    regret over block-steps and the critical-path regret (the sum over steps
    of the slowest block's cost under the policy's choices, minus the same
    under the cheaper branch of every block, from the forced runs' costs)."""
    res = {}
    logs = {}
    for pol in ("repair", "rebuild", "threshold", "mlp"):
        lg, secs, st = run_policy(w, steps, pol, device, tau=tau, mlp_w=mlp_w)
        logs[pol] = lg
        res[pol] = {"seconds": secs, "applied": st["applied"], "rebuilt_block_steps": st["rebuilt"],
                    "moves_per_s": st["applied"] / secs}
    valid = logs["repair"][..., 18] > 0
    step = np.nonzero(valid)[0]
    cr, cb = logs["repair"][..., 17], logs["rebuild"][..., 17]
    late = logs["rebuild"][..., 19][valid] > 0.5
    # the per-block cheaper branch (not exactly the fastest step once
    # deferred rebuilds add to it, but the reference the regret is taken to)
    rb_best = cb[valid] < cr[valid]
    best_cp = step_time(np.minimum(cr[valid], cb[valid]).astype(np.float64), step, rb_best & late)
    for pol in res:
        r, tot, best = regret(logs[pol][..., 16], cr, cb, valid)
        took = logs[pol][..., 16][valid] == 1
        chosen = np.where(took, cb[valid], cr[valid]).astype(np.float64)
        cp = step_time(chosen, step, took & late)
        res[pol].update(regret_ticks=r, chosen_ticks=tot, best_ticks=best,
                        cp_ticks=cp, cp_best_ticks=best_cp, cp_regret_ticks=cp - best_cp,
                        rebuild_fraction=float((logs[pol][..., 16][valid] == 1).mean()))
    return res
