"""The FP64 reference of the selector network against finite differences
(pins the reference before it is used to check the GPU kernels)."""
import numpy as np

from paper_2308_06484_amd.selector import fold_normalisation, init_weights
from tests import mlp_ref as R


def test_reference_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    w = rng.normal(0, 0.3, R.NPARAM)
    X = rng.normal(0, 1, (7, R.IN))
    Y = rng.normal(0, 1, (7, R.OUT))
    g = R.grad(w, X, Y)
    h = 1e-6
    for idx in list(range(0, R.NPARAM, 37)) + [R.NPARAM - 1, R.NPARAM - 2]:
        e = np.zeros(R.NPARAM)
        e[idx] = h
        fd = (R.loss(w + e, X, Y) - R.loss(w - e, X, Y)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), idx


def test_reference_closed_form_linear_case():
    # all hidden pre-activations positive: the network is affine, out = A x + c
    rng = np.random.default_rng(1)
    w = np.zeros(R.NPARAM)
    W1, b1, W2, b2, W3, b3 = R.unpack(w)
    o = 0
    W1v = np.abs(rng.normal(0, 1, (R.H, R.IN)))
    W2v = np.abs(rng.normal(0, 1, (R.H, R.H)))
    W3v = rng.normal(0, 1, (R.OUT, R.H))
    w = np.concatenate([W1v.ravel(), np.ones(R.H), W2v.ravel(), np.ones(R.H), W3v.ravel(), [0.5, -0.5]])
    X = np.abs(rng.normal(0, 1, (5, R.IN)))
    out, _ = R.forward(w, X)
    expect = (W3v @ (W2v @ (W1v @ X.T + 1).clip(0) + 1).clip(0)).T + np.array([0.5, -0.5])
    assert np.allclose(out, expect)


def test_fold_normalisation_is_exact_in_fp64():
    rng = np.random.default_rng(2)
    w = init_weights(3).astype(np.float64)
    X = rng.normal(5, 3, (9, R.IN))
    mu, sd = X.mean(0), X.std(0)
    a, _ = R.forward(w, (X - mu) / sd)
    b, _ = R.forward(fold_normalisation(w, mu, sd).astype(np.float64), X)
    assert np.allclose(a, b, rtol=1e-4, atol=1e-4)
