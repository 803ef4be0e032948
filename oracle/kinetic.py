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
