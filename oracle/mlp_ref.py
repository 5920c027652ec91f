"""Float64 reference of the per-phase selector network -- TEST INFRASTRUCTURE ONLY.

Network: 12 -> 64 (ReLU) -> 64 (ReLU) -> 6 logits. Loss: mean softmax cross-entropy over the
batch. Flat parameter layout (5382 values): W1[64][12], b1[64], W2[64][64], b2[64], W3[6][64], b3[6].
Written from the definitions (chain rule); pinned by a finite-difference test in tests/.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 12, 64, 6
SHAPES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NOUT, NH)), ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + k], np.float64).reshape(shp)
        o += k
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], np.float64).ravel() for name, _ in SHAPES])


def forward(flat, X):
    p = unpack(flat)
    X = np.asarray(X, np.float64)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["W3"].T + p["b3"]
    return z, (X, a1, h1, a2, h2)


def loss_and_grad(flat, X, y):
    """Mean softmax cross-entropy and its gradient with respect to the flat parameters."""
    p = unpack(flat)
    z, (X, a1, h1, a2, h2) = forward(flat, X)
    B = X.shape[0]
    zs = z - z.max(axis=1, keepdims=True)
    ez = np.exp(zs)
    prob = ez / ez.sum(axis=1, keepdims=True)
    y = np.asarray(y, np.int64)
    loss = float(-np.log(prob[np.arange(B), y]).mean())
    dz = prob.copy()
    dz[np.arange(B), y] -= 1.0
    dz /= B
    g = {"W3": dz.T @ h2, "b3": dz.sum(0)}
    dh2 = dz @ p["W3"]
    da2 = dh2 * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * (a1 > 0)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(0)
    return loss, pack(g)


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases, drawn from numpy's PCG64 with the given seed."""
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[1])
            parts[name] = rng.uniform(-lim, lim, size=shp)
        else:
            parts[name] = np.zeros(shp)
    return pack(parts)


def train_adam(flat, X, y, epochs=30, batch=256, lr=3e-3, seed=0):
    """Plain Adam (beta1 0.9, beta2 0.999, eps 1e-8) on shuffled minibatches, float64."""
    w = np.array(flat, np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    rng = np.random.default_rng(seed)
    t = 0
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.int64)
    for _ in range(epochs):
        order = rng.permutation(len(y))
        for s in range(0, len(y), batch):
            idx = order[s:s + batch]
            _, gr = loss_and_grad(w, X[idx], y[idx])
            t += 1
            m = 0.9 * m + 0.1 * gr
            v = 0.999 * v + 0.001 * gr * gr
            mh = m / (1 - 0.9 ** t)
            vh = v / (1 - 0.999 ** t)
            w -= lr * mh / (np.sqrt(vh) + 1e-8)
    return w
