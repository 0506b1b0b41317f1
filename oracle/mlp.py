"""FP64 reference of the warm-start network.  TEST INFRASTRUCTURE ONLY.

A 3-layer perceptron of width H with tanh activations:
    h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), y = h2 w3 + b3
trained on the mean squared error (1/B) sum_i (y_i - t_i)^2 with Adam (Kingma & Ba,
"Adam: a method for stochastic optimization", ICLR 2015: first and second moment
estimates with bias correction).  Parameters are kept in one flat vector in the order
W1 (F x H, row-major), b1 (H), W2 (H x H), b2 (H), w3 (H), b3 (1).
"""
from __future__ import annotations

import numpy as np


def sizes(F: int, H: int):
    return [("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]


def unpack(theta, F, H):
    out = {}
    o = 0
    for name, shp in sizes(F, H):
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    return out


def count(F, H):
    return sum(int(np.prod(s)) for _, s in sizes(F, H))


def forward(theta, X, H):
    F = X.shape[1]
    p = unpack(np.asarray(theta, dtype=np.float64), F, H)
    h1 = np.tanh(X @ p["W1"] + p["b1"])
    h2 = np.tanh(h1 @ p["W2"] + p["b2"])
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (h1, h2)


def loss_and_grad(theta, X, t, H):
    """MSE loss and its gradient with respect to the flat parameter vector."""
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    B, F = X.shape
    p = unpack(np.asarray(theta, dtype=np.float64), F, H)
    y, (h1, h2) = forward(theta, X, H)
    r = y - t
    loss = float(np.mean(r * r))
    gy = 2.0 * r / B                       # dL/dy
    g_w3 = h2.T @ gy
    g_b3 = np.array([gy.sum()])
    g_h2 = np.outer(gy, p["w3"]) * (1.0 - h2 * h2)
    g_W2 = h1.T @ g_h2
    g_b2 = g_h2.sum(axis=0)
    g_h1 = (g_h2 @ p["W2"].T) * (1.0 - h1 * h1)
    g_W1 = X.T @ g_h1
    g_b1 = g_h1.sum(axis=0)
    grad = np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, g_b3])
    return loss, grad


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1**step)
    vh = v / (1 - b2**step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(F, H, seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases (FP64)."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, shp in sizes(F, H):
        if name.startswith("b"):
            parts.append(np.zeros(shp).ravel())
        else:
            fan_in = shp[0]
            parts.append(g.uniform(-1, 1, shp).ravel() / np.sqrt(fan_in))
    return np.concatenate(parts)
