"""The C-ABI library loads, exports every declared symbol, and validates its
arguments on the host (no GPU needed: every case here returns before any
HIP call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2308_06484_amd import kdt as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_declared_symbol_is_exported():
    hdr = open(os.path.join(ROOT, "include", "kdt.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(kdt_\w+)\s*\(", hdr, re.M))
    assert declared == set(K.EXPORTS)
    L = ctypes.CDLL(K.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name


def test_strerror():
    L = K.lib()
    assert L.kdt_strerror(0) == b"ok"
    assert b"duplicate" in L.kdt_strerror(K.E_DUP)


def test_workspace_size_formula_grows_with_points():
    a = K.workspace_size(1024, [0, 1024])
    b = K.workspace_size(2048, [0, 1024, 2048])
    # one 64-byte record per triangle dominates: 2n - 2B records
    assert b - a >= 64 * (2 * 2048 - 4 - (2 * 1024 - 2)) and a > 64 * 2046
    with pytest.raises(K.KDTError):
        K.workspace_size(10, [0, 5, 9])


def _init(xy, off, frames=None, ws=1 << 20):
    L = K.lib()
    xy = np.ascontiguousarray(xy, np.int32)
    off = np.ascontiguousarray(off, np.int64)
    fr = None if frames is None else np.ascontiguousarray(frames, np.int32)
    ctx = ctypes.c_void_p()
    # a non-null, 256-byte aligned fake address: validation fails before use
    return L.kdt_init(ctypes.byref(ctx), xy.ctypes.data, len(xy), len(off) - 1, off.ctypes.data,
                      None if fr is None else fr.ctypes.data, 0, ctypes.c_void_p(1 << 20), ws, None)


def test_init_validation_errors():
    sq = [[0, 0], [4, 0], [4, 4], [0, 4], [2, 1]]
    assert _init(sq[:3], [0, 3]) == K.E_DEGEN                      # fewer than 4 points
    assert _init([[0, 0], [1, 1], [2, 2], [3, 3]], [0, 4]) == K.E_DEGEN  # collinear
    assert _init([[0, 0], [4, 0], [4, 0], [0, 4]], [0, 4]) == K.E_DUP
    assert _init([[0, 0], [4, 0], [4, 4], [0, 1 << 24]], [0, 4]) == K.E_RANGE
    assert _init([[0, 0], [4, 0], [4, 4], [-1, 4]], [0, 4]) == K.E_RANGE
    assert _init(sq, [0, 5], frames=[[0, 0, 4, 5]]) == K.E_RANGE    # x = 4 outside [0, 4)
    assert _init(sq, [0, 5], frames=[[3, 0, 2, 5]]) == K.E_RANGE    # empty frame
    assert _init(sq, [0, 4]) == K.E_ARG                              # offsets do not end at n
    assert _init(sq, [0, 5], ws=64) == K.E_CAPACITY                  # workspace too small


def test_null_context_is_rejected():
    L = K.lib()
    assert L.kdt_step(None) == K.E_ARG
    assert L.kdt_sync(None) == K.E_ARG
    assert L.kdt_move(None, 0, 0, 0, 1) == K.E_ARG
    L.kdt_destroy(None)
