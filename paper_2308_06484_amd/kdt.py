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

BLOCKED = 1
OK, E_ARG, E_RANGE, E_DUP, E_DEGEN, E_CAPACITY, E_DEVICE, E_STATE, E_INTERNAL = 0, -1, -2, -3, -4, -5, -6, -7, -8
RUN_PER_STEP, RUN_FUSED, RUN_PERSISTENT = 0, 1, 2
POLICY = {"repair": 0, "rebuild": 1, "threshold": 2, "mlp": 3, "dlimit": 4}
MLP_PARAMS = 1666
LOG_FIELDS = 20

EXPORTS = ("kdt_workspace_size", "kdt_init", "kdt_move", "kdt_step", "kdt_run", "kdt_query",
           "kdt_query_canonical", "kdt_positions", "kdt_stats", "kdt_block_status", "kdt_sync",
           "kdt_destroy", "kdt_strerror", "kdt_timing", "kdt_timing_read", "kdt_set_launch",
           "kdt_graph_build", "kdt_graph_launch", "kdt_graph_destroy", "kdt_digest",
           "kdt_set_policy", "kdt_set_log", "kdt_mlp_forward", "kdt_mlp_grad", "kdt_mlp_train",
           "kdt_workspace_size_global", "kdt_init_global", "kdt_run_global", "kdt_rebuild_global",
           "kdt_owner", "kdt_global_stats", "kdt_moves", "kdt_step_status", "kdt_query_blocks",
           "kdt_partition", "kdt_mlp_train_noalloc", "kdt_set_block_waves", "kdt_dcalc", "kdt_set_repair",
           "kdt_set_prefetch", "kdt_set_block_order", "kdt_graph_build_global",
           "kdt_workspace_size_global_qt", "kdt_init_global_qt", "kdt_quadtree", "kdt_repartition",
           "kdt_set_repartition")
REPAIR = {"delins": 0, "flip": 1}
MLP_NOALLOC_BATCH = 4096
PART = {"grid": 0, "quadtree": 1}

# kdt_global_stats counters, in order
GSTATS = ("interacting", "serial", "lost", "transfers", "overflow", "build_rounds", "link", "tree")
GSTAT_N = 8


class KDTError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__(f"{where}: {_lib().kdt_strerror(code).decode()} ({code})")


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("applied", "blocked", "star_sum", "cavity_sum", "walk_sum", "tri_touched",
                 "alg_bytes", "errors", "t_star", "t_locate", "t_hole", "t_insert", "clock_khz")] + \
               [("hist", ctypes.c_int64 * 16), ("fast", ctypes.c_int64), ("rebuilt", ctypes.c_int64),
                ("flipped", ctypes.c_int64), ("flips", ctypes.c_int64)]

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
        L.kdt_moves.argtypes = [vp, vp, vp, i64, vp]
        L.kdt_step_status.argtypes = [vp, vp]
        L.kdt_query_blocks.argtypes = [vp, vp, i32, vp, vp, i64, vp]
        L.kdt_partition.argtypes = [vp, i64, i32, i64, vp, vp, vp, i32, ctypes.POINTER(i32)]
        L.kdt_run.argtypes = [vp, vp, vp, i32, vp, i32]
        L.kdt_query.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(i64)]
        L.kdt_query_canonical.argtypes = [vp, vp, i64, ctypes.POINTER(i64)]
        L.kdt_positions.argtypes = [vp, vp]
        L.kdt_digest.argtypes = [vp, vp]
        L.kdt_set_policy.argtypes = [vp, i32, ctypes.c_float, vp]
        L.kdt_set_log.argtypes = [vp, vp, i64]
        L.kdt_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.kdt_mlp_grad.argtypes = [vp, vp, vp, i64, vp, vp]
        L.kdt_mlp_train.argtypes = [vp, vp, vp, i64, i32, i32, ctypes.c_float, vp, vp]
        L.kdt_mlp_train_noalloc.argtypes = [vp, vp, vp, i64, i32, i32, ctypes.c_float, vp]
        L.kdt_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.kdt_block_status.argtypes = [vp, vp]
        L.kdt_sync.argtypes = [vp]
        L.kdt_destroy.argtypes = [vp]
        L.kdt_destroy.restype = None
        L.kdt_timing.argtypes = [vp, i32]
        L.kdt_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        L.kdt_set_launch.argtypes = [vp, i32]
        L.kdt_set_block_waves.argtypes = [vp, i32]
        L.kdt_set_repair.argtypes = [vp, i32]
        L.kdt_set_prefetch.argtypes = [vp, i32]
        L.kdt_set_block_order.argtypes = [vp, i32, i32, i32]
        L.kdt_workspace_size_global_qt.argtypes = [vp, i64, vp, i64, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.kdt_init_global_qt.argtypes = [ctypes.POINTER(vp), vp, i64, vp, i64, i32, vp, ctypes.c_size_t, vp]
        L.kdt_quadtree.argtypes = [vp, vp, i32, ctypes.POINTER(i32)]
        L.kdt_repartition.argtypes = [vp]
        L.kdt_set_repartition.argtypes = [vp, i32]
        L.kdt_dcalc.argtypes = [vp, i32, vp, vp, ctypes.POINTER(i64), ctypes.POINTER(i64), vp]
        L.kdt_graph_build.argtypes = [vp, vp, vp, i32, vp, i32, ctypes.POINTER(vp)]
        L.kdt_graph_launch.argtypes = [vp, vp]
        L.kdt_graph_build_global.argtypes = [vp, vp, vp, i32, vp, ctypes.POINTER(vp)]
        L.kdt_graph_destroy.argtypes = [vp]
        L.kdt_graph_destroy.restype = None
        L.kdt_workspace_size_global.argtypes = [i64, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.kdt_init_global.argtypes = [ctypes.POINTER(vp), vp, i64, i32, vp, i32, vp, ctypes.c_size_t, vp]
        L.kdt_run_global.argtypes = [vp, vp, vp, i32, vp]
        L.kdt_rebuild_global.argtypes = [vp]
        L.kdt_owner.argtypes = [vp, vp]
        L.kdt_global_stats.argtypes = [vp, vp]
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


def partition(xy, scheme, param):
    """Library-side partition (kdt_partition): scheme "grid" (param = number
    of cells, a power of four) or "quadtree" (param = threshold).  Returns
    (perm int64 [N], pt_off int64 [B + 1], frame int32 [B, 4]); row i of the
    partitioned set is input point perm[i]."""
    xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
    n = xy.shape[0]
    perm = np.empty(n, dtype=np.int64)
    nb = ctypes.c_int32(0)
    L = _lib()
    rc = L.kdt_partition(_ptr(xy), n, PART[scheme], int(param), _ptr(perm), None, None, 0, ctypes.byref(nb))
    if rc not in (OK, E_CAPACITY):
        _check(rc, "kdt_partition")
    cap = int(nb.value)
    off = np.zeros(cap + 1, dtype=np.int64)
    fr = np.zeros((max(cap, 1), 4), dtype=np.int32)
    _check(L.kdt_partition(_ptr(xy), n, PART[scheme], int(param), _ptr(perm), _ptr(off), _ptr(fr), cap,
                           ctypes.byref(nb)), "kdt_partition")
    return perm, off, fr[:cap]


def _stream_arg(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def mlp_forward(w, x, stream=None):
    """Device tensors: w [MLP_PARAMS], x [n, 16] -> out [n, 2] (float32)."""
    n = x.shape[0]
    out = torch.empty((n, 2), dtype=torch.float32, device=x.device)
    _check(_lib().kdt_mlp_forward(ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(x.data_ptr()), n,
                                  ctypes.c_void_p(out.data_ptr()), _stream_arg(stream)), "kdt_mlp_forward")
    return out


def mlp_grad(w, x, y, stream=None):
    """Summed gradient [MLP_PARAMS] and summed loss of 0.5 |f(x) - y|^2."""
    g = torch.empty(MLP_PARAMS + 1, dtype=torch.float32, device=x.device)
    _check(_lib().kdt_mlp_grad(ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                               ctypes.c_void_p(y.data_ptr()), x.shape[0], ctypes.c_void_p(g.data_ptr()),
                               _stream_arg(stream)), "kdt_mlp_grad")
    return g[:MLP_PARAMS], g[MLP_PARAMS]


def mlp_train(w, x, y, epochs, batch, lr, stream=None):
    """Mini-batch gradient descent on the device; w updated in place."""
    scratch = torch.empty(MLP_PARAMS + 1, dtype=torch.float32, device=x.device)
    _check(_lib().kdt_mlp_train(ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                ctypes.c_void_p(y.data_ptr()), x.shape[0], int(epochs), int(batch),
                                float(lr), ctypes.c_void_p(scratch.data_ptr()), _stream_arg(stream)),
           "kdt_mlp_train")
    return w


def mlp_train_noalloc(w, x, y, epochs, batch, lr, stream=None):
    """mlp_train with no device allocation (the library's fixed scratch;
    batch <= MLP_NOALLOC_BATCH); w updated in place."""
    _check(_lib().kdt_mlp_train_noalloc(ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(y.data_ptr()), x.shape[0], int(epochs), int(batch),
                                        float(lr), _stream_arg(stream)), "kdt_mlp_train_noalloc")
    return w


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

    def moves(self, blocks, moves):
        """Stage a batch: blocks int32 [M], moves int32 [M, 4] (local point,
        dir, dist, 0).  Returns the per-move staging status (int32 [M])."""
        blocks = np.ascontiguousarray(blocks, dtype=np.int32)
        moves = np.ascontiguousarray(moves, dtype=np.int32).reshape(-1, 4)
        st = np.zeros(len(blocks), dtype=np.int32)
        rc = _lib().kdt_moves(self.ctx, _ptr(blocks), _ptr(moves), len(blocks), _ptr(st))
        if rc not in (OK, E_ARG, E_CAPACITY):
            _check(rc, "kdt_moves")
        return st

    def step_status(self, n_staged):
        """Apply the staged step; per staged move OK (0) or BLOCKED (1)."""
        st = np.full(max(1, n_staged), -100, dtype=np.int32)
        _check(_lib().kdt_step_status(self.ctx, _ptr(st)), "kdt_step_status")
        return st[:n_staged]

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

    def set_policy(self, policy, tau=0.0, mlp_w=None):
        """policy: "repair", "rebuild", "threshold" (tau) or "mlp" (mlp_w: a
        float32 device tensor of MLP_PARAMS, kept alive by this object)."""
        if mlp_w is not None:
            assert mlp_w.dtype == torch.float32 and mlp_w.is_cuda and mlp_w.numel() == MLP_PARAMS
        self._mlp_w = mlp_w
        _check(_lib().kdt_set_policy(self.ctx, POLICY[policy], float(tau),
                                     None if mlp_w is None else ctypes.c_void_p(mlp_w.data_ptr())),
               "kdt_set_policy")

    def set_log(self, cap_steps):
        """Log features, branch and cost per step and block into a device
        tensor [cap_steps, B, LOG_FIELDS] (returned; None turns it off)."""
        if not cap_steps:
            _check(_lib().kdt_set_log(self.ctx, None, 0), "kdt_set_log")
            self._log = None
            return None
        self._log = torch.zeros((cap_steps, self.B, LOG_FIELDS), dtype=torch.float32, device=self.device)
        _check(_lib().kdt_set_log(self.ctx, ctypes.c_void_p(self._log.data_ptr()), cap_steps), "kdt_set_log")
        return self._log

    def set_launch(self, persist_per_cu):
        _check(_lib().kdt_set_launch(self.ctx, int(persist_per_cu)), "kdt_set_launch")

    def set_repair(self, variant):
        """Repair variant: "delins" (delete + insert) or "flip" (move-and-flip)."""
        _check(_lib().kdt_set_repair(self.ctx, REPAIR[variant]), "kdt_set_repair")

    def set_prefetch(self, depth):
        """Staging depth of the star prefetch before a block's moves: 0 off,
        1 (default) star and the ring beyond it, 2 one ring more; same results."""
        _check(_lib().kdt_set_prefetch(self.ctx, int(depth)), "kdt_set_prefetch")

    def set_block_order(self, order, heavy_cut=0, mid_cut=0):
        """Per-step launch schedule: blocks most moves first (order=1) and,
        with several wavefronts per block, size classes split at heavy_cut
        moves (and, with four wavefronts, a two-wavefront middle class from
        mid_cut moves), run at once on separate streams."""
        _check(_lib().kdt_set_block_order(self.ctx, int(order), int(heavy_cut), int(mid_cut)),
               "kdt_set_block_order")

    def set_block_waves(self, waves):
        """Wavefronts per block of the per-step launch (1, 2 or 4)."""
        _check(_lib().kdt_set_block_waves(self.ctx, int(waves)), "kdt_set_block_waves")

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

    def query_blocks(self, blocks, adjacency=False):
        """Canonical triangles of the listed blocks (kdt_query_blocks):
        (tris int32 [T, 3], adj int32 [T, 3] or None, off int64 [len + 1]);
        block blocks[i] holds rows off[i] .. off[i+1]-1."""
        blocks = np.ascontiguousarray(blocks, dtype=np.int32)
        off = np.zeros(len(blocks) + 1, dtype=np.int64)
        L = _lib()
        rc = L.kdt_query_blocks(self.ctx, _ptr(blocks), len(blocks), None, None, 0, _ptr(off))
        if rc not in (OK, E_CAPACITY):
            _check(rc, "kdt_query_blocks")
        cap = int(off[-1])
        tris = np.empty((max(cap, 1), 3), dtype=np.int32)
        adj = np.empty((max(cap, 1), 3), dtype=np.int32) if adjacency else None
        _check(L.kdt_query_blocks(self.ctx, _ptr(blocks), len(blocks), _ptr(tris), _ptr(adj), cap, _ptr(off)),
               "kdt_query_blocks")
        return tris[:cap], (adj[:cap] if adjacency else None), off

    def digest(self):
        """uint64 [B]: order-independent digest of each block's triangulation."""
        out = np.zeros(self.B, dtype=np.uint64)
        _check(_lib().kdt_digest(self.ctx, _ptr(out)), "kdt_digest")
        return out

    def dcalc(self, N):
        """d-calculation (kdt_dcalc): dict of per-block mindistance^2 and
        diameter^2, mindistance(P_t)^2 now, d^2 over the calls so far, and
        every block's running N-spread."""
        mind2 = np.zeros(self.B, dtype=np.int64)
        diam2 = np.zeros(self.B, dtype=np.int64)
        spread = np.zeros(self.B, dtype=np.float64)
        now, dmin = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(_lib().kdt_dcalc(self.ctx, int(N), _ptr(mind2), _ptr(diam2), ctypes.byref(now), ctypes.byref(dmin),
                                _ptr(spread)), "kdt_dcalc")
        return dict(mind2=mind2, diam2=diam2, d2_now=int(now.value), d2=int(dmin.value), spread=spread)

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

    def timing(self, enable=True, period=1):
        """Record a HIP event pair around every period-th step's launch (see
        kdt_timing); enable=False stops."""
        _check(_lib().kdt_timing(self.ctx, int(period) if enable else 0), "kdt_timing")

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


def workspace_size_global(n, depth, max_moves):
    out = ctypes.c_size_t(0)
    _check(_lib().kdt_workspace_size_global(int(n), int(depth), int(max_moves), ctypes.byref(out)),
           "kdt_workspace_size_global")
    return int(out.value)


class GlobalDT(KineticDT):
    """A global-mode context: one DT* over every point of the domain
    (x0, y0, x1, y1), kd cells of depth `depth` -- or, with `quadtree` =
    threshold, the leaves of the quad-tree of the initial points -- and at
    most `max_moves` moves per step.  Query, digest, positions and stats as
    for one block."""

    def __init__(self, xy, domain, depth, max_moves, device="cuda:0", stream=None, quadtree=None):
        L = _lib()
        self.xy0 = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
        self.domain = np.ascontiguousarray(domain, dtype=np.int32).reshape(4)
        self.depth = int(depth)
        self.max_moves = int(max_moves)
        self.n = self.xy0.shape[0]
        self.B = 1
        self.pt_off = np.array([0, self.n], dtype=np.int64)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        if quadtree:
            out = ctypes.c_size_t(0)
            _check(L.kdt_workspace_size_global_qt(_ptr(self.xy0), self.n, _ptr(self.domain), int(quadtree),
                                                  self.max_moves, ctypes.byref(out)), "kdt_workspace_size_global_qt")
            ws = int(out.value)
            self.ws = torch.empty(ws, dtype=torch.uint8, device=self.device)
            rc = L.kdt_init_global_qt(ctypes.byref(ctx), _ptr(self.xy0), self.n, _ptr(self.domain), int(quadtree),
                                      self.max_moves, ctypes.c_void_p(self.ws.data_ptr()), ws,
                                      ctypes.c_void_p(self.stream.cuda_stream))
            _check(rc, "kdt_init_global_qt")
        else:
            ws = workspace_size_global(self.n, self.depth, self.max_moves)
            self.ws = torch.empty(ws, dtype=torch.uint8, device=self.device)
            rc = L.kdt_init_global(ctypes.byref(ctx), _ptr(self.xy0), self.n, self.depth, _ptr(self.domain),
                                   self.max_moves, ctypes.c_void_p(self.ws.data_ptr()), ws,
                                   ctypes.c_void_p(self.stream.cuda_stream))
            _check(rc, "kdt_init_global")
        self.ctx = ctx

    def repartition(self):
        """Quad-treeDvision of the current positions (kdt_repartition)."""
        _check(_lib().kdt_repartition(self.ctx), "kdt_repartition")

    def set_repartition(self, every_step=True):
        _check(_lib().kdt_set_repartition(self.ctx, 1 if every_step else 0), "kdt_set_repartition")

    def quadtree(self):
        """int32 [nodes, 8]: (x0, y0, side, first child, links +x, -x, +y, -y
        of a leaf)."""
        L = _lib()
        nn = ctypes.c_int32(0)
        rc = L.kdt_quadtree(self.ctx, None, 0, ctypes.byref(nn))
        if rc not in (OK, E_CAPACITY):
            _check(rc, "kdt_quadtree")
        out = np.zeros((max(1, nn.value), 8), dtype=np.int32)
        _check(L.kdt_quadtree(self.ctx, _ptr(out), nn.value, ctypes.byref(nn)), "kdt_quadtree")
        return out[:nn.value]

    def run(self, moves, step_off, applied=None):
        """moves: device int32 [M, 4] (global point id, dir, dist, 0);
        step_off: host int64 [T + 1]; applied: device int8 [M] or None."""
        assert moves.dtype == torch.int32 and moves.is_cuda and moves.is_contiguous()
        step_off = np.ascontiguousarray(step_off, dtype=np.int64)
        if applied is not None:
            assert applied.dtype == torch.int8 and applied.is_cuda
        _check(_lib().kdt_run_global(self.ctx, ctypes.c_void_p(moves.data_ptr()), _ptr(step_off),
                                     len(step_off) - 1,
                                     ctypes.c_void_p(applied.data_ptr()) if applied is not None else None),
               "kdt_run_global")

    def graph(self, moves, step_off, applied=None):
        """The steps captured once as a HIP graph (needs a non-null stream;
        not with re-partition every step); returns a Graph with launch() and
        close()."""
        assert moves.dtype == torch.int32 and moves.is_cuda and moves.is_contiguous()
        step_off = np.ascontiguousarray(step_off, dtype=np.int64)
        if applied is not None:
            assert applied.dtype == torch.int8 and applied.is_cuda
        g = ctypes.c_void_p()
        _check(_lib().kdt_graph_build_global(self.ctx, ctypes.c_void_p(moves.data_ptr()), _ptr(step_off),
                                             len(step_off) - 1,
                                             ctypes.c_void_p(applied.data_ptr()) if applied is not None else None,
                                             ctypes.byref(g)), "kdt_graph_build_global")
        return Graph(self, g, (moves, step_off, applied))

    def rebuild(self):
        _check(_lib().kdt_rebuild_global(self.ctx), "kdt_rebuild_global")

    def owner(self):
        out = np.empty(self.n, dtype=np.int32)
        _check(_lib().kdt_owner(self.ctx, _ptr(out)), "kdt_owner")
        return out

    def gstats(self):
        out = np.zeros(GSTAT_N, dtype=np.uint64)
        _check(_lib().kdt_global_stats(self.ctx, _ptr(out)), "kdt_global_stats")
        return {k: int(out[i]) for i, k in enumerate(GSTATS)}
