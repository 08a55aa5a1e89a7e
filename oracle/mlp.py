"""MLP oracle (FP64 numpy) -- TEST INFRASTRUCTURE ONLY.

The config selector is a multilayer perceptron  x -> ReLU(x W1 + b1) ->
ReLU(h1 W2 + b2) -> h2 W3 + b3  that maps sparsity features (already
standardised) to one predicted log time ratio per candidate kernel
configuration.  Training minimises the masked mean squared error
    loss = sum_{m,g} M_mg (out_mg - T_mg)^2 / sum M
and updates the weights with Adam (Kingma and Ba, 2015).  Every step here is
written out plainly: forward, loss, backward by the chain rule, Adam.
Weights are stored input-major: W has shape [fan_in, fan_out].
"""
from __future__ import annotations

import numpy as np

NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def forward(params, X):
    """Returns (out, cache)."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], np.float64) for k in NAMES)
    X = np.asarray(X, np.float64)
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ W3 + b3
    return out, (X, z1, h1, z2, h2)


def loss(out, T, M) -> float:
    M = np.asarray(M, np.float64)
    cnt = M.sum()
    if cnt == 0:
        return 0.0
    d = (np.asarray(out, np.float64) - np.asarray(T, np.float64)) * M
    return float((d * d).sum() / cnt)


def backward(params, cache, out, T, M):
    """Gradients of the masked MSE with respect to every weight."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[k], np.float64) for k in NAMES)
    X, z1, h1, z2, h2 = cache
    M = np.asarray(M, np.float64)
    cnt = max(M.sum(), 1.0)
    g_out = 2.0 * (np.asarray(out, np.float64) - np.asarray(T, np.float64)) * M / cnt
    gW3 = h2.T @ g_out
    gb3 = g_out.sum(0)
    g_h2 = g_out @ W3.T
    g_z2 = g_h2 * (z2 > 0.0)
    gW2 = h1.T @ g_z2
    gb2 = g_z2.sum(0)
    g_h1 = g_z2 @ W2.T
    g_z1 = g_h1 * (z1 > 0.0)
    gW1 = X.T @ g_z1
    gb1 = g_z1.sum(0)
    return {"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "W3": gW3, "b3": gb3}


def adam_step(params, grads, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  Returns new (params, m, v)."""
    P, Mo, Vo = {}, {}, {}
    for k in NAMES:
        g = np.asarray(grads[k], np.float64)
        Mo[k] = beta1 * np.asarray(m[k], np.float64) + (1.0 - beta1) * g
        Vo[k] = beta2 * np.asarray(v[k], np.float64) + (1.0 - beta2) * g * g
        mh = Mo[k] / (1.0 - beta1 ** t)
        vh = Vo[k] / (1.0 - beta2 ** t)
        P[k] = np.asarray(params[k], np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return P, Mo, Vo
