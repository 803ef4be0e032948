"""Kinetic driver of the oracle: applies a move stream, rebuilds from scratch.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper's main loop (Fig. 4) moves, in every time step, a chosen point of
every block in one of four directions (Lemma 1, Sec. V) and requires the
triangulation to be Delaunay again after the step (Sec. III).  Rather than
repairing anything, the oracle keeps only the point positions and recomputes
each block's DT* from scratch (the "rebuild" alternative of Sec. I) with the
Bowyer-Watson code in dt_oracle.c.

Move rule (the paper leaves it open; this project's reading): the moves of a
block in one step are applied one after the other in list order; a move of
point p by `dist` lattice units in direction `dir` (0 +x, 1 -x, 2 +y, 3 -y)
jumps p to its target cell, and is blocked (no change) when that cell lies
outside the block's half-open frame or is held by a point of the block.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import dt_star

_DIR = ((1, 0), (-1, 0), (0, 1), (0, -1))


class Kinetic:
    def __init__(self, xy, pt_off, frame):
        self.xy = np.array(xy, dtype=np.int32).reshape(-1, 2)
        self.pt_off = np.asarray(pt_off, dtype=np.int64)
        self.frame = np.asarray(frame, dtype=np.int64).reshape(-1, 4)
        self.B = len(self.pt_off) - 1
        self.occ = []
        for b in range(self.B):
            lo, hi = self.pt_off[b], self.pt_off[b + 1]
            self.occ.append({(int(x), int(y)) for x, y in self.xy[lo:hi]})

    def apply_step(self, mv, mv_off_row):
        """Apply one step's moves; returns a bool array (applied) per move row
        of this step, in order."""
        applied = []
        for b in range(self.B):
            lo_m, hi_m = int(mv_off_row[b]), int(mv_off_row[b + 1])
            base = int(self.pt_off[b])
            x0, y0, x1, y1 = (int(v) for v in self.frame[b])
            occ = self.occ[b]
            for r in range(lo_m, hi_m):
                p, d, dist = int(mv[r, 0]), int(mv[r, 1]), int(mv[r, 2])
                px, py = int(self.xy[base + p, 0]), int(self.xy[base + p, 1])
                qx, qy = px + dist * _DIR[d][0], py + dist * _DIR[d][1]
                if not (x0 <= qx < x1 and y0 <= qy < y1) or (qx, qy) in occ:
                    applied.append(False)
                    continue
                occ.discard((px, py))
                occ.add((qx, qy))
                self.xy[base + p] = (qx, qy)
                applied.append(True)
        return np.array(applied, dtype=bool)

    def block_dt(self, b):
        lo, hi = int(self.pt_off[b]), int(self.pt_off[b + 1])
        return dt_star(self.xy[lo:hi], np.arange(lo, hi, dtype=np.int64))

    def blocks_dt(self, blocks=None, threads=None):
        """Canonical DT* of the listed blocks (default: all), rebuilt from
        scratch, on a pool of `threads` host threads (ctypes drops the GIL)."""
        blocks = range(self.B) if blocks is None else list(blocks)
        if threads is None or threads <= 1:
            return [self.block_dt(b) for b in blocks]
        with ThreadPoolExecutor(max_workers=threads) as ex:
            return list(ex.map(self.block_dt, blocks))

    def all_dt(self, threads=None):
        """Canonical list of every block's triangles, concatenated in block
        order (ids are global, so this is the sorted union)."""
        parts = self.blocks_dt(None, threads)
        return np.concatenate(parts) if parts else np.zeros((0, 3), np.int64)


def kd_splits(xy, depth):
    """The kd partition of a point set into 2^depth cells, by definition:
    the root holds every point; a node at level l orders its points by the
    key (x, y) if l is even, (y, x) if l is odd, keeps the first half (n // 2
    points) on the left and the rest on the right, and its split key is the
    key of the first right point.  Nodes are numbered as a heap (root 1,
    children 2k and 2k + 1).  Returns int64 [2^depth, 2]: the split key of
    node k in row k (row 0 unused)."""
    xy = np.asarray(xy, dtype=np.int64)
    splits = np.zeros((1 << depth, 2), dtype=np.int64)
    if depth == 0:
        return splits

    def node(k, idx, level):
        a = xy[idx, level % 2]
        b = xy[idx, 1 - level % 2]
        idx = idx[np.lexsort((b, a))]
        h = len(idx) // 2
        splits[k] = (xy[idx[h], level % 2], xy[idx[h], 1 - level % 2])
        if level + 1 < depth:
            node(2 * k, idx[:h], level + 1)
            node(2 * k + 1, idx[h:], level + 1)

    node(1, np.arange(len(xy)), 0)
    return splits


def kd_cell(xy, splits, depth):
    """Cell (0 .. 2^depth - 1) of each position: from the root, go right iff
    the position's key is >= the node's split key (lexicographically)."""
    xy = np.asarray(xy, dtype=np.int64).reshape(-1, 2)
    k = np.ones(len(xy), dtype=np.int64)
    for level in range(depth):
        a = xy[:, level % 2]
        b = xy[:, 1 - level % 2]
        sa, sb = splits[k, 0], splits[k, 1]
        right = (a > sa) | ((a == sa) & (b >= sb))
        k = 2 * k + right
    return k - (1 << depth)


class KineticGlobal:
    """Global mode: one DT* over every point of the domain [0, side)^2.

    Move rule (this project's reading, as in the per-block mode but with one
    domain): the moves of a step are applied one after the other in list
    order; a move of point p by `dist` units in direction `dir` jumps p to
    its target cell and is blocked when that cell lies outside the domain or
    is held by any point at that moment.  Points belong to the kd cell that
    holds their current position (cells fixed by the initial points)."""

    def __init__(self, xy, side, depth):
        self.xy = np.array(xy, dtype=np.int32).reshape(-1, 2)
        self.side = int(side)
        self.depth = int(depth)
        self.occ = set((self.xy[:, 0].astype(np.int64) << 24 | self.xy[:, 1]).tolist())
        self.splits = kd_splits(self.xy, self.depth)

    def apply_step(self, mv_rows):
        """Apply one step's moves (rows (point, dir, dist, _)) in order;
        returns a bool array: applied."""
        out = np.zeros(len(mv_rows), dtype=bool)
        for r, (p, d, dist) in enumerate(np.asarray(mv_rows)[:, :3].tolist()):
            px, py = int(self.xy[p, 0]), int(self.xy[p, 1])
            qx, qy = px + dist * _DIR[d][0], py + dist * _DIR[d][1]
            key = qx << 24 | qy
            if not (0 <= qx < self.side and 0 <= qy < self.side) or key in self.occ:
                continue
            self.occ.discard(px << 24 | py)
            self.occ.add(key)
            self.xy[p] = (qx, qy)
            out[r] = True
        return out

    def owner(self):
        return kd_cell(self.xy, self.splits, self.depth)

    def dt(self):
        """Canonical DT* of all points (global ids = rows).  The points are
        handed to the builder in strips of 64 columns, alternately upward and
        downward, so that consecutive insertions are close; the order never
        changes DT*."""
        x = self.xy[:, 0].astype(np.int64)
        y = self.xy[:, 1].astype(np.int64)
        strip = x >> 6
        yy = np.where(strip % 2 == 0, y, (1 << 24) - 1 - y)
        order = np.lexsort((x, yy, strip))
        return dt_star(self.xy[order], order.astype(np.int64))


def quadtree(xy, domain, thr):
    """Quad-tree of a point set (Sec. III, "Data structure"), by its
    definition: the root is the smallest power-of-two square at the domain's
    lower-left corner that covers the domain; a square holding more than
    `thr` points (and wider than one lattice cell) is cut into its four
    quarters -- (low x, low y), (high x, low y), (low x, high y), (high x,
    high y), empty ones kept.  Nodes are numbered depth first (a node's four
    children get the next numbers when it is cut).  Returns the nodes as
    [x0, y0, side, first child or -1] and the leaf of every point."""
    xy = np.asarray(xy, dtype=np.int64).reshape(-1, 2)
    x0, y0, x1, y1 = (int(v) for v in domain)
    side = 1
    while side < max(x1 - x0, y1 - y0):
        side *= 2
    nodes = [[x0, y0, side, -1]]
    cell = np.zeros(len(xy), dtype=np.int64)

    def node(k, idx):
        nx, ny, s, _ = nodes[k]
        if len(idx) <= thr or s == 1:
            cell[idx] = k
            return
        h = s // 2
        c0 = len(nodes)
        nodes[k][3] = c0
        for q in range(4):
            nodes.append([nx + (q & 1) * h, ny + (q >> 1) * h, h, -1])
        p = xy[idx]
        quarter = (p[:, 0] >= nx + h).astype(np.int64) + 2 * (p[:, 1] >= ny + h)
        for q in range(4):
            node(c0 + q, idx[quarter == q])

    node(0, np.arange(len(xy)))
    return nodes, cell


def quadtree_leaf(nodes, x, y):
    """The leaf holding the lattice point (x, y)."""
    k = 0
    while nodes[k][3] >= 0:
        nx, ny, s, c = nodes[k]
        h = s // 2
        k = c + (1 if x >= nx + h else 0) + (2 if y >= ny + h else 0)
    return k


class KineticGlobalQT(KineticGlobal):
    """Global mode with quad-tree cells (fixed by the initial points): the
    same triangulation and move rule, a point's cell is the leaf holding
    its current position."""

    def __init__(self, xy, side, thr):
        super().__init__(xy, side, 0)
        self.thr = thr
        self.nodes, _ = quadtree(self.xy, (0, 0, side, side), thr)

    def owner(self):
        return np.array([quadtree_leaf(self.nodes, int(x), int(y)) for x, y in self.xy.tolist()], dtype=np.int64)

    def repartition(self):
        """Quad-treeDvision of the current positions (Fig. 4): the tree made
        again, by the same definition."""
        self.nodes, _ = quadtree(self.xy, (0, 0, self.side, self.side), self.thr)
