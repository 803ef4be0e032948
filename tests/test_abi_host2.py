"""More host-side checks of the C-ABI (no GPU needed)."""
from paper_2308_06484_amd import kdt as K


def test_graph_and_launch_calls_reject_null_context():
    L = K.lib()
    assert L.kdt_set_launch(None, 4) == K.E_ARG
    assert L.kdt_graph_launch(None, None) == K.E_ARG
    L.kdt_graph_destroy(None)


def test_global_mode_validation_without_device():
    """Argument and input checks of the global-mode calls happen on the host,
    before anything touches the device."""
    import ctypes

    import numpy as np
    L = K.lib()
    out = ctypes.c_size_t(0)
    assert L.kdt_workspace_size_global(16, 2, 8, ctypes.byref(out)) == K.OK and out.value > 0
    small = out.value
    assert L.kdt_workspace_size_global(1 << 12, 4, 64, ctypes.byref(out)) == K.OK and out.value > small
    assert L.kdt_workspace_size_global(16, -1, 8, ctypes.byref(out)) == K.E_ARG
    assert L.kdt_workspace_size_global(16, 2, 0, ctypes.byref(out)) == K.E_ARG
    assert L.kdt_workspace_size_global((1 << 22) + 1, 2, 8, ctypes.byref(out)) == K.E_CAPACITY

    def init(xy, depth=1, domain=(0, 0, 64, 64), max_moves=4):
        xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
        dom = np.ascontiguousarray(domain, dtype=np.int32)
        ctx = ctypes.c_void_p()
        return L.kdt_init_global(ctypes.byref(ctx), K._ptr(xy), len(xy), depth, K._ptr(dom), max_moves,
                                 None, 0, None)

    sq = [(0, 0), (5, 0), (0, 5), (5, 5), (2, 3)]
    assert init(sq[:3]) == K.E_DEGEN                      # fewer than 4 points
    assert init([(i, i) for i in range(6)]) == K.E_DEGEN  # all collinear
    assert init(sq + [(5, 5)]) == K.E_DUP                 # a repeated cell
    assert init(sq, domain=(0, 0, 5, 64)) == K.E_RANGE    # x = 5 outside [0, 5)
    assert init(sq, domain=(3, 0, 1, 64)) == K.E_RANGE    # empty domain
    assert init(sq, depth=3) == K.E_ARG                   # fewer points than kd cells
    assert init(sq, max_moves=0) == K.E_ARG
    assert init(sq) == K.E_CAPACITY                       # no workspace given
    assert L.kdt_run_global(None, None, None, 0, None) == K.E_ARG
    assert L.kdt_rebuild_global(None) == K.E_ARG
    assert L.kdt_owner(None, None) == K.E_ARG
    assert L.kdt_global_stats(None, None) == K.E_ARG
