"""FP64 numpy reference of the selector network (test infrastructure).

16 -> 32 ReLU -> 32 ReLU -> 2, loss 0.5 * sum (out - y)^2 summed over the
samples.  Parameter layout as in include/kdt.h: W1[32][16], b1[32],
W2[32][32], b2[32], W3[2][32], b3[2].
"""
import numpy as np

IN, H, OUT = 16, 32, 2
NPARAM = H * IN + H + H * H + H + OUT * H + OUT


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    o = 0
    out = []
    for shape in ((H, IN), (H,), (H, H), (H,), (OUT, H), (OUT,)):
        n = int(np.prod(shape))
        out.append(w[o:o + n].reshape(shape))
        o += n
    return out


def forward(w, X):
    W1, b1, W2, b2, W3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0)
    return h2 @ W3.T + b3, (X, z1, h1, z2, h2)


def loss(w, X, Y):
    out, _ = forward(w, X)
    return 0.5 * float(((out - np.asarray(Y, np.float64)) ** 2).sum())


def grad(w, X, Y):
    W1, b1, W2, b2, W3, b3 = unpack(w)
    out, (X, z1, h1, z2, h2) = forward(w, X)
    d3 = out - np.asarray(Y, np.float64)
    gW3 = d3.T @ h2
    gb3 = d3.sum(0)
    d2 = (d3 @ W3) * (z2 > 0)
    gW2 = d2.T @ h1
    gb2 = d2.sum(0)
    d1 = (d2 @ W2) * (z1 > 0)
    gW1 = d1.T @ X
    gb1 = d1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
