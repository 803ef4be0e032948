"""Python binding of libkdt (include/kdt.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libkdt.so; this module
only allocates the device workspace with torch, passes pointers and sizes,
and turns status codes into exceptions.  It fails loudly if the library has
not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libkdt.so")

OK, E_ARG, E_RANGE, E_DUP, E_DEGEN, E_CAPACITY, E_DEVICE, E_STATE, E_INTERNAL = 0, -1, -2, -3, -4, -5, -6, -7, -8
RUN_PER_STEP, RUN_FUSED, RUN_PERSISTENT = 0, 1, 2

EXPORTS = ("kdt_workspace_size", "kdt_init", "kdt_move", "kdt_step", "kdt_run", "kdt_query",
           "kdt_query_canonical", "kdt_positions", "kdt_stats", "kdt_block_status", "kdt_sync",
           "kdt_destroy", "kdt_strerror", "kdt_timing", "kdt_timing_read", "kdt_set_launch",
           "kdt_graph_build", "kdt_graph_launch", "kdt_graph_destroy")


class KDTError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__(f"{where}: {_lib().kdt_strerror(code).decode()} ({code})")


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("applied", "blocked", "star_sum", "cavity_sum", "walk_sum", "tri_touched",
                 "alg_bytes", "errors", "t_star", "t_locate", "t_hole", "t_insert", "clock_khz")] + \
               [("hist", ctypes.c_int64 * 16), ("fast", ctypes.c_int64)]

    def as_dict(self):
        d = {n: int(getattr(self, n)) for n, _ in self._fields_ if n != "hist"}
        d["hist"] = [int(v) for v in self.hist]
        return d


_L = None


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2308_06484_amd.build.build_lib()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.kdt_workspace_size.argtypes = [i64, i32, vp, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.kdt_init.argtypes = [ctypes.POINTER(vp), vp, i64, i32, vp, vp, i32, vp, ctypes.c_size_t, vp]
        L.kdt_move.argtypes = [vp, i32, i64, i32, i32]
        L.kdt_step.argtypes = [vp]
        L.kdt_run.argtypes = [vp, vp, vp, i32, vp, i32]
        L.kdt_query.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(i64)]
        L.kdt_query_canonical.argtypes = [vp, vp, i64, ctypes.POINTER(i64)]
        L.kdt_positions.argtypes = [vp, vp]
        L.kdt_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.kdt_block_status.argtypes = [vp, vp]
        L.kdt_sync.argtypes = [vp]
        L.kdt_destroy.argtypes = [vp]
        L.kdt_destroy.restype = None
        L.kdt_timing.argtypes = [vp, i32]
        L.kdt_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        L.kdt_set_launch.argtypes = [vp, i32]
        L.kdt_graph_build.argtypes = [vp, vp, vp, i32, vp, i32, ctypes.POINTER(vp)]
        L.kdt_graph_launch.argtypes = [vp, vp]
        L.kdt_graph_destroy.argtypes = [vp]
        L.kdt_graph_destroy.restype = None
        L.kdt_strerror.argtypes = [ctypes.c_int]
        L.kdt_strerror.restype = ctypes.c_char_p
        _L = L
    return _L


def lib():
    return _lib()


def _check(rc, where):
    if rc != OK:
        raise KDTError(rc, where)


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def workspace_size(n, pt_off, max_staged=0):
    pt_off = np.ascontiguousarray(pt_off, dtype=np.int64)
    out = ctypes.c_size_t(0)
    _check(_lib().kdt_workspace_size(int(n), len(pt_off) - 1, _ptr(pt_off), int(max_staged),
                                     ctypes.byref(out)), "kdt_workspace_size")
    return int(out.value)


class Graph:
    """A captured multi-step launch; keeps the tensors it records alive."""

    def __init__(self, dt, handle, keep):
        self.dt, self.handle, self.keep = dt, handle, keep

    def launch(self):
        _check(_lib().kdt_graph_launch(self.dt.ctx, self.handle), "kdt_graph_launch")

    def close(self):
        if self.handle:
            _lib().kdt_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class KineticDT:
    """One context of the library: the per-block DT* of a partitioned point
    set, kept on the device.  `xy` int32 [N, 2], `pt_off` int64 [B + 1],
    `frame` int32 [B, 4] (x0, y0, x1, y1) or None."""

    def __init__(self, xy, pt_off, frame=None, max_staged=0, device="cuda:0", stream=None):
        L = _lib()
        self.xy0 = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
        self.pt_off = np.ascontiguousarray(pt_off, dtype=np.int64)
        self.frame = None if frame is None else np.ascontiguousarray(frame, dtype=np.int32).reshape(-1, 4)
        self.n = self.xy0.shape[0]
        self.B = len(self.pt_off) - 1
        self.device = torch.device(device)
        ws = workspace_size(self.n, self.pt_off, max_staged)
        self.ws = torch.empty(ws, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        rc = L.kdt_init(ctypes.byref(ctx), _ptr(self.xy0), self.n, self.B, _ptr(self.pt_off),
                        _ptr(self.frame), int(max_staged), ctypes.c_void_p(self.ws.data_ptr()),
                        ws, ctypes.c_void_p(self.stream.cuda_stream))
        _check(rc, "kdt_init")
        self.ctx = ctx

    # ---- moves
    def move(self, block, point, direction, dist):
        _check(_lib().kdt_move(self.ctx, int(block), int(point), int(direction), int(dist)), "kdt_move")

    def step(self):
        _check(_lib().kdt_step(self.ctx), "kdt_step")

    def _check_stream(self, moves, step_off, applied):
        assert moves.dtype == torch.int32 and moves.is_cuda and moves.is_contiguous()
        assert step_off.dtype == torch.int32 and step_off.is_cuda and step_off.is_contiguous()
        assert step_off.shape[-1] == self.B + 1
        if applied is not None:
            assert applied.dtype == torch.int8 and applied.is_cuda and applied.numel() >= moves.shape[0]

    def run(self, moves, step_off, n_steps=None, applied=None, fused=False, mode=None):
        """moves: int32 device tensor [M, 4]; step_off: int32 device tensor
        [T, B + 1]; applied: optional int8 device tensor [M].
        mode: "step" (default), "fused" or "persistent"."""
        if mode is None:
            mode = "fused" if fused else "step"
        flags = {"step": RUN_PER_STEP, "fused": RUN_FUSED, "persistent": RUN_PERSISTENT}[mode]
        assert moves.dtype == torch.int32 and moves.is_cuda and moves.is_contiguous()
        assert step_off.dtype == torch.int32 and step_off.is_cuda and step_off.is_contiguous()
        assert step_off.shape[-1] == self.B + 1
        T = step_off.shape[0] if n_steps is None else int(n_steps)
        assert T <= step_off.shape[0]
        if applied is not None:
            assert applied.dtype == torch.int8 and applied.is_cuda and applied.numel() >= moves.shape[0]
        rc = _lib().kdt_run(self.ctx, ctypes.c_void_p(moves.data_ptr()), ctypes.c_void_p(step_off.data_ptr()),
                            T, None if applied is None else ctypes.c_void_p(applied.data_ptr()), flags)
        _check(rc, "kdt_run")

    def set_launch(self, persist_per_cu):
        _check(_lib().kdt_set_launch(self.ctx, int(persist_per_cu)), "kdt_set_launch")

    def graph(self, moves, step_off, applied=None, mode="step"):
        """Capture the move stream's steps as a HIP graph (needs a non-null
        stream); returns a Graph with launch() and close()."""
        self._check_stream(moves, step_off, applied)
        flags = {"step": RUN_PER_STEP, "fused": RUN_FUSED, "persistent": RUN_PERSISTENT}[mode]
        g = ctypes.c_void_p()
        _check(_lib().kdt_graph_build(self.ctx, ctypes.c_void_p(moves.data_ptr()),
                                      ctypes.c_void_p(step_off.data_ptr()), step_off.shape[0],
                                      None if applied is None else ctypes.c_void_p(applied.data_ptr()),
                                      flags, ctypes.byref(g)), "kdt_graph_build")
        return Graph(self, g, (moves, step_off, applied))

    # ---- results
    def sync(self):
        _check(_lib().kdt_sync(self.ctx), "kdt_sync")

    def query(self):
        """(tris int32 [T, 3], adj int32 [T, 3], blk_off int64 [B + 1]) on the host."""
        L = _lib()
        cap = 2 * self.n
        tris = torch.empty((cap, 3), dtype=torch.int32, device=self.device)
        adj = torch.empty((cap, 3), dtype=torch.int32, device=self.device)
        off = np.zeros(self.B + 1, dtype=np.int64)
        nt = ctypes.c_int64(0)
        _check(L.kdt_query(self.ctx, ctypes.c_void_p(tris.data_ptr()), ctypes.c_void_p(adj.data_ptr()),
                           _ptr(off), cap, ctypes.byref(nt)), "kdt_query")
        k = int(nt.value)
        return tris[:k].cpu().numpy(), adj[:k].cpu().numpy(), off

    def query_canonical(self):
        cap = 2 * self.n
        out = np.empty((cap, 3), dtype=np.int32)
        nt = ctypes.c_int64(0)
        _check(_lib().kdt_query_canonical(self.ctx, _ptr(out), cap, ctypes.byref(nt)), "kdt_query_canonical")
        return out[:int(nt.value)].copy()

    def positions(self):
        out = np.empty((self.n, 2), dtype=np.int32)
        _check(_lib().kdt_positions(self.ctx, _ptr(out)), "kdt_positions")
        return out

    def stats(self):
        s = Stats()
        _check(_lib().kdt_stats(self.ctx, ctypes.byref(s)), "kdt_stats")
        return s.as_dict()

    def block_status(self):
        out = np.zeros(self.B, dtype=np.int32)
        _check(_lib().kdt_block_status(self.ctx, _ptr(out)), "kdt_block_status")
        return out

    def timing(self, enable=True):
        """Record a HIP event pair around every launch (see kdt_timing)."""
        _check(_lib().kdt_timing(self.ctx, 1 if enable else 0), "kdt_timing")

    def timing_read(self):
        """(summed kernel milliseconds, launches) since timing was enabled."""
        ms, n = ctypes.c_double(0), ctypes.c_int64(0)
        _check(_lib().kdt_timing_read(self.ctx, ctypes.byref(ms), ctypes.byref(n)), "kdt_timing_read")
        return float(ms.value), int(n.value)

    def close(self):
        if getattr(self, "ctx", None):
            _lib().kdt_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
