"""kdt_mlp_train_noalloc (no device allocation: the library's fixed scratch)
against kdt_mlp_train (scratch passed in) through the C-ABI: the same
weights after two calls in a row, the second on a smaller input, and the
batch limit refused on the host."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_noalloc_training_matches_the_scratch_entry_point():
    from paper_2308_06484_amd import kdt as K
    from paper_2308_06484_amd.selector import init_weights
    rng = np.random.default_rng(12)
    for n, batch, epochs, lr in ((5000, 4096, 3, 0.05), (700, 256, 4, 0.02)):
        print(f"no-alloc training: n {n}, batch {batch}, epochs {epochs}", flush=True)
        X = rng.normal(0, 1, (n, 16)).astype(np.float32)
        Y = rng.normal(0, 1, (n, 2)).astype(np.float32)
        xt, yt = torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV)
        a = torch.from_numpy(init_weights(n) * 0.5).to(DEV)
        b = a.clone()
        K.mlp_train(a, xt, yt, epochs, batch, lr)
        K.mlp_train_noalloc(b, xt, yt, epochs, batch, lr)
        torch.cuda.synchronize()
        # the sums are added in the same order: the same floats
        assert torch.equal(a, b), float((a - b).abs().max())
        assert not torch.equal(a, torch.from_numpy(init_weights(n) * 0.5).to(DEV))
    L = K.lib()
    w = torch.zeros(K.MLP_PARAMS, device=DEV)
    assert L.kdt_mlp_train_noalloc(ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                   ctypes.c_void_p(w.data_ptr()), 10, 1, K.MLP_NOALLOC_BATCH + 1, 0.1,
                                   None) == K.E_CAPACITY
    assert L.kdt_mlp_train_noalloc(None, None, None, 10, 1, 8, 0.1, None) == K.E_ARG
