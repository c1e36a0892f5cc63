"""FP64 reference of the root-cost MLP — TEST INFRASTRUCTURE ONLY.

Network (an addition to the paper's method, used only to order work): input
x = (log1p(f) - mean) / std for the four per-vertex features f, then
h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3.  Loss is the
mean squared error against t = log1p(tree nodes).  Adam follows Kingma & Ba
(2015) with bias correction.  Parameter layout matches the library's blob:
W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3, mean[4], std[4].
"""
from __future__ import annotations

import numpy as np

NET = 4 * 64 + 64 + 64 * 64 + 64 + 64 + 1
BLOB = NET + 8


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return dict(W1=p[0:256].reshape(64, 4), b1=p[256:320], W2=p[320:4416].reshape(64, 64), b2=p[4416:4480],
                w3=p[4480:4544], b3=p[4544], mean=p[4545:4549], std=p[4549:4553])


def pack(d) -> np.ndarray:
    return np.concatenate([d["W1"].ravel(), d["b1"], d["W2"].ravel(), d["b2"], d["w3"], [d["b3"]], d["mean"],
                           d["std"]])


def inputs(p, F):
    d = unpack(p)
    return (np.log1p(np.asarray(F, dtype=np.float64)) - d["mean"]) / d["std"]


def forward(p, F, X=None):
    d = unpack(p)
    X = inputs(p, F) if X is None else X
    Z1 = X @ d["W1"].T + d["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ d["W2"].T + d["b2"]
    H2 = np.maximum(Z2, 0.0)
    y = H2 @ d["w3"] + d["b3"]
    return y, (X, Z1, H1, Z2, H2)


def abs_output(p, F):
    """Output of the same network with every weight, bias and input replaced by
    its absolute value: the magnitude scale of the rounding error of y."""
    d = unpack(p)
    X = np.abs(inputs(p, F))
    A1 = X @ np.abs(d["W1"]).T + np.abs(d["b1"])
    A2 = A1 @ np.abs(d["W2"]).T + np.abs(d["b2"])
    return A2 @ np.abs(d["w3"]) + abs(d["b3"])


def loss_grad(p, F, T, X=None, row_weight=None):
    """Mean squared error, its gradient (NET,) and, per gradient entry, the sum
    over rows of the absolute per-row contributions, each row scaled by
    row_weight (default 1): the scale of rounding errors in the gradient."""
    d = unpack(p)
    T = np.asarray(T, dtype=np.float64)
    y, (X, Z1, H1, Z2, H2) = forward(p, F, X)
    B = y.shape[0]
    dy = 2.0 * (y - T) / B                      # [B]
    dH2 = np.outer(dy, d["w3"]) * (Z2 > 0)      # [B, 64]
    dH1 = (dH2 @ d["W2"]) * (Z1 > 0)            # [B, 64]
    g = dict(W1=dH1.T @ X, b1=dH1.sum(0), W2=dH2.T @ H1, b2=dH2.sum(0), w3=H2.T @ dy, b3=dy.sum())
    rw = np.ones(B) if row_weight is None else np.asarray(row_weight, dtype=np.float64)
    aH1, aH2, ady = np.abs(dH1) * rw[:, None], np.abs(dH2) * rw[:, None], np.abs(dy) * rw
    a = dict(W1=aH1.T @ np.abs(X), b1=aH1.sum(0), W2=aH2.T @ np.abs(H1),
             b2=aH2.sum(0), w3=np.abs(H2).T @ ady, b3=ady.sum())
    flat = lambda q: np.concatenate([q["W1"].ravel(), q["b1"], q["W2"].ravel(), q["b2"], q["w3"], [q["b3"]]])
    loss = float(np.mean((y - T) ** 2))
    return loss, flat(g), flat(a)


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    p = np.array(p, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p[:NET] -= lr * mh / (np.sqrt(vh) + eps)
    return p, m, v
