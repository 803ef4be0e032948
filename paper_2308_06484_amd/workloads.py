"""Seeded synthetic workloads: point sets, block partitions and move streams.

This module only draws random numbers.  It holds none of the method's
arithmetic (no predicate, no triangulation, no move-blocking rule): the GPU
path and the CPU oracle each apply the moves it emits with their own code.

Shapes follow the paper's setting (Sec. III, "Notation and definitions";
Fig. 4): points on an integer lattice, a partition into blocks, and at every
time step a randomly chosen point per block that moves in one of four
directions (Lemma 1 of Sec. V).  The sizes are the workloads this project is
measured on:

  lattice256   1 block, 256 uniform points on [0,4096)^2, 100 steps,
               one move of 1 unit per step.
  grid1024     32x32 square cells of 2048^2 over [0,65536)^2 (a depth-5
               quad-tree), 1024 uniform points per cell, 1000 steps,
               one move per block of 1..8 units.
  uneven4096   4096 blocks, lognormal sizes (median 1024, clipped to
               64..16384), 4-component Gaussian mixture per block snapped to
               [0,65536)^2, 500 steps, one move per block of 1..8 units.
  multi2048    2048 blocks x 4096 uniform points on [0,16384)^2, per step
               k ~ clip(Poisson(lambda_b), 1, 64) distinct movers per block
               with Pareto(1.2) distances capped at 4096.

  global4m     one triangulation of 4,194,304 uniform points on
               [0,65536)^2; the points are grouped into 4096 cells of 1024
               by alternating median splits (x first), and every step moves
               one point drawn from each cell by 1..16 units (200 steps).

A workload is a dict of numpy arrays:
  xy      int32 [N, 2]   point coordinates, grouped by block
  pt_off  int64 [B + 1]  block b owns points pt_off[b] .. pt_off[b+1]-1;
                         the global id of a point is its row in xy
  frame   int32 [B, 4]   (x0, y0, x1, y1): half-open domain of block b
  mv      int32 [M, 4]   (local point, direction, distance, 0)
  mv_off  int32 [T, B+1] moves of step t for block b are rows
                         mv_off[t, b] .. mv_off[t, b+1]-1 of mv
Directions: 0 = +x (right), 1 = -x (left), 2 = +y (up), 3 = -y (down).

The global-mode workload (global4m) is a dict of:
  xy        int32 [N, 2]  points, ordered cell by cell (cell c holds rows
                          c * N / C .. (c + 1) * N / C - 1)
  side      int           the domain is [0, side)^2
  depth     int           C = 2^depth cells
  mv        int32 [M, 4]  (global point id, direction, distance, 0)
  step_off  int64 [T + 1] moves of step t are rows step_off[t] .. step_off[t+1]-1
"""
from __future__ import annotations

import numpy as np

DIRS = np.array([[1, 0], [-1, 0], [0, 1], [0, -1]], dtype=np.int64)


def _distinct_uniform(rng, n, x0, y0, w, h):
    """n distinct lattice points uniform on [x0,x0+w) x [y0,y0+h)."""
    if n > w * h:
        raise ValueError("more points than lattice cells")
    got = np.empty((0,), dtype=np.int64)
    while got.size < n:
        need = n - got.size
        cand = rng.integers(0, w * h, size=need + need // 8 + 8, dtype=np.int64)
        got = np.concatenate([got, cand])
        _, first = np.unique(got, return_index=True)
        got = got[np.sort(first)]
    got = got[:n]
    return np.stack([x0 + got % w, y0 + got // w], axis=1).astype(np.int32)


def _distinct_gmm(rng, n, lo, hi):
    """n distinct lattice points from a 4-component isotropic Gaussian
    mixture on [lo,hi)^2: weights ~ Dirichlet(1,1,1,1), means uniform,
    standard deviations log-uniform on [256, 8192].  Samples are rounded;
    samples outside the domain and repeated cells are drawn again."""
    w = rng.dirichlet(np.ones(4))
    mu = rng.uniform(lo, hi, size=(4, 2))
    sd = np.exp(rng.uniform(np.log(256.0), np.log(8192.0), size=4))
    have = np.empty((0,), dtype=np.int64)
    span = hi - lo
    while have.size < n:
        m = (n - have.size) * 2 + 16
        comp = rng.choice(4, size=m, p=w)
        pts = np.rint(mu[comp] + rng.standard_normal((m, 2)) * sd[comp, None])
        ok = np.all((pts >= lo) & (pts < hi), axis=1)
        pts = pts[ok].astype(np.int64) - lo
        key = pts[:, 1] * span + pts[:, 0]
        have = np.concatenate([have, key])
        _, first = np.unique(have, return_index=True)
        have = have[np.sort(first)]
    have = have[:n]
    return np.stack([lo + have % span, lo + have // span], axis=1).astype(np.int32)


def _one_move_per_block(rng, T, sizes, dmin, dmax):
    B = len(sizes)
    pt = (rng.random((T, B)) * sizes[None, :]).astype(np.int64)
    d = rng.integers(0, 4, size=(T, B))
    dist = rng.integers(dmin, dmax + 1, size=(T, B))
    mv = np.zeros((T * B, 4), dtype=np.int32)
    mv[:, 0] = pt.reshape(-1)
    mv[:, 1] = d.reshape(-1)
    mv[:, 2] = dist.reshape(-1)
    mv_off = (np.arange(T, dtype=np.int64)[:, None] * B
              + np.arange(B + 1, dtype=np.int64)[None, :]).astype(np.int32)
    return mv, mv_off


def lattice256(seed=1, steps=100, n=256):
    rng = np.random.default_rng(seed)
    xy = _distinct_uniform(rng, n, 0, 0, 4096, 4096)
    mv, mv_off = _one_move_per_block(rng, steps, np.array([n]), 1, 1)
    return dict(name="lattice256", xy=xy, pt_off=np.array([0, n], dtype=np.int64),
                frame=np.array([[0, 0, 4096, 4096]], dtype=np.int32),
                mv=mv, mv_off=mv_off)


def grid1024(seed=1, steps=1000, cells=32, per_block=1024, cell=2048):
    """Square cells of side `cell`; block b = (row b // cells, column b % cells)."""
    rng = np.random.default_rng(seed)
    B = cells * cells
    xy = np.empty((B * per_block, 2), dtype=np.int32)
    frame = np.empty((B, 4), dtype=np.int32)
    for b in range(B):
        x0, y0 = (b % cells) * cell, (b // cells) * cell
        frame[b] = (x0, y0, x0 + cell, y0 + cell)
        xy[b * per_block:(b + 1) * per_block] = _distinct_uniform(rng, per_block, x0, y0, cell, cell)
    pt_off = np.arange(B + 1, dtype=np.int64) * per_block
    mv, mv_off = _one_move_per_block(rng, steps, np.full(B, per_block), 1, 8)
    return dict(name="grid1024", xy=xy, pt_off=pt_off, frame=frame, mv=mv, mv_off=mv_off)


def uneven4096(seed=1, steps=500, blocks=4096, sigma=1.0, nmin=64, nmax=16384, median=1024):
    rng = np.random.default_rng(seed)
    sizes = np.clip(np.rint(np.exp(np.log(median) + sigma * rng.standard_normal(blocks))),
                    nmin, nmax).astype(np.int64)
    pt_off = np.zeros(blocks + 1, dtype=np.int64)
    pt_off[1:] = np.cumsum(sizes)
    xy = np.empty((int(pt_off[-1]), 2), dtype=np.int32)
    for b in range(blocks):
        xy[pt_off[b]:pt_off[b + 1]] = _distinct_gmm(rng, int(sizes[b]), 0, 65536)
    frame = np.tile(np.array([[0, 0, 65536, 65536]], dtype=np.int32), (blocks, 1))
    mv, mv_off = _one_move_per_block(rng, steps, sizes, 1, 8)
    return dict(name="uneven4096", xy=xy, pt_off=pt_off, frame=frame, mv=mv, mv_off=mv_off)


def multi2048(seed=1, steps=100, blocks=2048, per_block=4096, side=16384,
              kmax=64, alpha=1.2, dcap=4096):
    rng = np.random.default_rng(seed)
    xy = np.concatenate([_distinct_uniform(rng, per_block, 0, 0, side, side)
                         for _ in range(blocks)])
    pt_off = np.arange(blocks + 1, dtype=np.int64) * per_block
    frame = np.tile(np.array([[0, 0, side, side]], dtype=np.int32), (blocks, 1))
    lam = np.exp(rng.uniform(0.0, np.log(kmax), size=blocks))
    recs, offs, base = [], np.zeros((steps, blocks + 1), dtype=np.int64), 0
    for t in range(steps):
        k = np.clip(rng.poisson(lam), 1, kmax)
        offs[t, 0] = base
        for b in range(blocks):
            who = rng.choice(per_block, size=int(k[b]), replace=False)
            d = rng.integers(0, 4, size=k[b])
            u = 1.0 - rng.random(k[b])
            dist = np.minimum(dcap, np.floor(u ** (-1.0 / alpha))).astype(np.int64)
            recs.append(np.stack([who, d, dist, np.zeros_like(who)], axis=1))
            base += int(k[b])
            offs[t, b + 1] = base
    mv = np.concatenate(recs).astype(np.int32)
    return dict(name="multi2048", xy=xy, pt_off=pt_off, frame=frame, mv=mv,
                mv_off=offs.astype(np.int32))


def selector_mix(seed=1, steps=12, small=256, large=256, n_small=256, n_large=4096,
                 side_small=1024, side_large=16384):
    """Blocks where either branch of the repair-or-rebuild choice can be the
    cheaper one: `small` blocks of n_small points most of which move far
    every step (k ~ U{n/2..n} distinct movers, distances U{side/8..side/2})
    and `large` blocks of n_large points with a few short moves (k ~
    U{1..8}, distances U{1..8}); the two kinds are interleaved at random.
    Every block has its own frame, side by side along x."""
    rng = np.random.default_rng(seed)
    kinds = np.zeros(small + large, dtype=np.int64)
    kinds[rng.permutation(small + large)[:large]] = 1
    B = len(kinds)
    sizes = np.where(kinds == 1, n_large, n_small).astype(np.int64)
    sides = np.where(kinds == 1, side_large, side_small).astype(np.int64)
    x0 = np.concatenate([[0], np.cumsum(sides)[:-1]])
    if x0[-1] + sides[-1] > (1 << 24):
        raise ValueError("frames do not fit the lattice")
    pt_off = np.zeros(B + 1, dtype=np.int64)
    pt_off[1:] = np.cumsum(sizes)
    xy = np.concatenate([_distinct_uniform(rng, int(sizes[b]), int(x0[b]), 0, int(sides[b]), int(sides[b]))
                         for b in range(B)])
    frame = np.stack([x0, np.zeros(B, np.int64), x0 + sides, sides], axis=1).astype(np.int32)
    recs, offs, base = [], np.zeros((steps, B + 1), dtype=np.int64), 0
    for t in range(steps):
        offs[t, 0] = base
        for b in range(B):
            n, sd = int(sizes[b]), int(sides[b])
            if kinds[b] == 0:
                k = int(rng.integers(n // 2, n + 1))
                dist = rng.integers(sd // 8, sd // 2 + 1, size=k)
            else:
                k = int(rng.integers(1, 9))
                dist = rng.integers(1, 9, size=k)
            r = np.zeros((k, 4), dtype=np.int32)
            r[:, 0] = rng.choice(n, size=k, replace=False)
            r[:, 1] = rng.integers(0, 4, size=k)
            r[:, 2] = dist
            recs.append(r)
            base += k
            offs[t, b + 1] = base
    return dict(name="selector_mix", xy=xy, pt_off=pt_off, frame=frame, mv=np.concatenate(recs),
                mv_off=offs.astype(np.int32), kind=kinds)


def subset_blocks(w, blocks, steps=None):
    """Restrict a per-block workload to the listed blocks (and first steps).
    Global ids are renumbered to rows of the new xy, block by block."""
    blocks = np.asarray(blocks, dtype=np.int64)
    T = w["mv_off"].shape[0] if steps is None else steps
    sizes = w["pt_off"][blocks + 1] - w["pt_off"][blocks]
    pt_off = np.zeros(len(blocks) + 1, dtype=np.int64)
    pt_off[1:] = np.cumsum(sizes)
    xy = np.concatenate([w["xy"][w["pt_off"][b]:w["pt_off"][b + 1]] for b in blocks])
    recs, offs, base = [], np.zeros((T, len(blocks) + 1), dtype=np.int64), 0
    for t in range(T):
        offs[t, 0] = base
        for j, b in enumerate(blocks):
            lo, hi = w["mv_off"][t, b], w["mv_off"][t, b + 1]
            recs.append(w["mv"][lo:hi])
            base += int(hi - lo)
            offs[t, j + 1] = base
    mv = np.concatenate(recs) if recs else np.zeros((0, 4), np.int32)
    return dict(name=w["name"] + "_subset", xy=xy, pt_off=pt_off,
                frame=w["frame"][blocks].copy(), mv=mv.astype(np.int32),
                mv_off=offs.astype(np.int32))


def _median_groups(xy, depth):
    """Row order that groups the points into 2^depth cells of equal size by
    alternating median splits: at level l every group is sorted by
    (x, y) (l even) or (y, x) (l odd) and cut in half.  Used to pick one
    mover per cell; requires N divisible by 2^depth."""
    n = len(xy)
    if n % (1 << depth):
        raise ValueError("point count must be divisible by the cell count")
    order = np.arange(n, dtype=np.int64)
    x = xy[:, 0].astype(np.int64)
    y = xy[:, 1].astype(np.int64)
    for level in range(depth):
        group = np.arange(n, dtype=np.int64) // (n >> level)
        a, b = (x, y) if level % 2 == 0 else (y, x)
        key = (group << 48) | (a[order] << 24) | b[order]
        order = order[np.argsort(key, kind="stable")]
    return order


def global_mode(seed=1, steps=200, n=1 << 22, depth=12, side=65536, dmax=16, name="global4m"):
    """One triangulation over all points (see the module notes)."""
    rng = np.random.default_rng(seed)
    xy = _distinct_uniform(rng, n, 0, 0, side, side)
    xy = xy[_median_groups(xy, depth)]
    cells = 1 << depth
    per = n // cells
    pt = (np.arange(cells, dtype=np.int64)[None, :] * per
          + rng.integers(0, per, size=(steps, cells)))
    mv = np.zeros((steps * cells, 4), dtype=np.int32)
    mv[:, 0] = pt.reshape(-1)
    mv[:, 1] = rng.integers(0, 4, size=steps * cells)
    mv[:, 2] = rng.integers(1, dmax + 1, size=steps * cells)
    step_off = np.arange(steps + 1, dtype=np.int64) * cells
    return dict(name=name, xy=xy, side=side, depth=depth, mv=mv, step_off=step_off)


def global4m(seed=1, steps=200):
    return global_mode(seed=seed, steps=steps)


def global_small(seed=1, steps=20, n=16384, depth=4, side=4096, dmax=16):
    """The global mode at the density of global4m (one point per 1024
    lattice cells), small enough for the oracle at every step."""
    return global_mode(seed=seed, steps=steps, n=n, depth=depth, side=side, dmax=dmax,
                       name="global_small")
