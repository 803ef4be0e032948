"""d-calculation and N-spread by their definitions (TEST INFRASTRUCTURE ONLY;
see oracle/__init__.py).

Sec. III ("Notation and definitions"): for a constant N, dist_p is the
distance from p to its N-th nearest neighbour; mindistance(P) is the
minimum of dist_p over the points; d is the minimum of mindistance(P_t)
over the time steps t.  Sec. IV: each block computes its value locally and
the minimum over the blocks is taken.  The N-spread of a block is
diam(P_i) / mindistance(P), kept at its largest over the time steps.

Readings: the neighbours of a point are the other points of its block (the
blocks are independent triangulations); distances are compared through
their exact squares (integers); a block with at most N points has no N-th
nearest neighbour and takes no part in the minimum.  Plain brute force over
all pairs, with numpy.
"""
from __future__ import annotations

import numpy as np

NONE = np.iinfo(np.int64).max


def block_values(xy, N):
    """(mindistance^2, diam^2) of one block: exact int64, brute force."""
    p = np.asarray(xy, dtype=np.int64).reshape(-1, 2)
    n = len(p)
    dx = p[:, None, 0] - p[None, :, 0]
    dy = p[:, None, 1] - p[None, :, 1]
    d2 = dx * dx + dy * dy
    diam2 = int(d2.max()) if n > 1 else 0
    if n <= N:
        return NONE, diam2
    # the N-th smallest distance to another point: row minus the zero to itself
    nth = np.partition(d2, N, axis=1)[:, N]
    return int(nth.min()), diam2


def dcalc(xy, pt_off, N):
    """Per-block (mindistance^2, diam^2) arrays and mindistance(P)^2."""
    B = len(pt_off) - 1
    mind2 = np.empty(B, dtype=np.int64)
    diam2 = np.empty(B, dtype=np.int64)
    for b in range(B):
        mind2[b], diam2[b] = block_values(xy[pt_off[b]:pt_off[b + 1]], N)
    return mind2, diam2, int(mind2.min())


class DTracker:
    """d over time (running minimum of mindistance(P_t)) and every block's
    N-spread (running maximum of diam(P_i) / mindistance(P_t))."""

    def __init__(self, B):
        self.d2 = NONE
        self.spread = np.zeros(B, dtype=np.float64)

    def update(self, mind2, diam2, g2):
        self.d2 = min(self.d2, g2)
        if g2 != NONE:
            self.spread = np.maximum(self.spread, np.sqrt(diam2.astype(np.float64) / float(g2)))
        return self.d2, self.spread
