"""CPU oracle for the kinetic Delaunay method.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product path (the HIP
library and its Python binding) never does, and shares no code with it.

  dt_star(xy, ids)        DT*(S) of one point set by from-scratch
                          Bowyer-Watson (dt_oracle.c), canonical list
  definition.dt_star_bf   the same set by the O(n^4) empty-circle definition
  kinetic.Kinetic         applies a move stream block by block and rebuilds
                          every block's DT* from scratch after each step
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "dt_oracle.c")

ERRORS = {-1: "bad arguments", -2: "coordinate out of range", -3: "duplicate point",
          -4: "fewer than 3 points or all collinear", -5: "out of memory",
          -8: "internal failure"}


def build(force: bool = True) -> str:
    """Compile dt_oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        i64, i32p, i64p = ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
        L.oracle_dt.restype = ctypes.c_long
        L.oracle_dt.argtypes = [i32p, i64p, ctypes.c_long, i64p, ctypes.c_long]
        L.oracle_orient.restype = i64
        L.oracle_orient.argtypes = [i64] * 6
        L.oracle_incircle_sign.restype = ctypes.c_int
        L.oracle_incircle_sign.argtypes = [i64] * 8
        L.oracle_incircle_star.restype = ctypes.c_int
        L.oracle_incircle_star.argtypes = [i64] * 12
        L.oracle_ghost_conflict.restype = ctypes.c_int
        L.oracle_ghost_conflict.argtypes = [i64] * 6
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle_dt failed: {ERRORS.get(code, code)}")
        self.code = code


def dt_star(xy, ids=None) -> np.ndarray:
    """Canonical DT*(S): int64 [T, 3] global ids, counter-clockwise, each row
    rotated to start at its smallest id, rows sorted lexicographically."""
    xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
    n = xy.shape[0]
    ids = np.arange(n, dtype=np.int64) if ids is None else np.ascontiguousarray(ids, dtype=np.int64)
    cap = max(2 * n, 1)
    out = np.empty((cap, 3), dtype=np.int64)
    L = lib()
    r = L.oracle_dt(xy.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n,
                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), cap)
    if r < 0:
        raise OracleError(r)
    return out[:r].copy()
