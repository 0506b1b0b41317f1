"""Pins for the warm-start network reference: finite differences, a hand-computed tiny
case, and Adam's first step (which moves every parameter by lr in the gradient's sign)."""
import numpy as np
import pytest

from oracle import mlp


def test_gradient_matches_finite_differences():
    F, H = 5, 7
    rng = np.random.default_rng(1)
    th = mlp.init_params(F, H, 2) + rng.normal(0, 0.1, mlp.count(F, H))
    X = rng.normal(0, 1, (13, F))
    t = rng.normal(0, 1, 13)
    L, g = mlp.loss_and_grad(th, X, t, H)
    h = 1e-6
    for i in rng.choice(th.size, 40, replace=False):
        e = np.zeros_like(th)
        e[i] = h
        fd = (mlp.loss_and_grad(th + e, X, t, H)[0] - mlp.loss_and_grad(th - e, X, t, H)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-9)


def test_tiny_network_by_hand():
    """F = 1, H = 1: y = w3 tanh(w2 tanh(w1 x + b1) + b2) + b3, written out."""
    th = np.array([0.5, 0.1, -1.2, 0.3, 2.0, -0.4])  # W1, b1, W2, b2, w3, b3
    x = np.array([[0.7]])
    y, _ = mlp.forward(th, x, 1)
    h1 = np.tanh(0.5 * 0.7 + 0.1)
    h2 = np.tanh(-1.2 * h1 + 0.3)
    assert y[0] == pytest.approx(2.0 * h2 - 0.4, rel=1e-15)


def test_adam_first_step_moves_by_lr():
    th = np.array([1.0, -2.0, 3.0])
    g = np.array([0.3, -5.0, 1e-3])
    th2, m, v = mlp.adam_step(th, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(th2, th - 0.01 * np.sign(g), rtol=0, atol=1e-7)


def test_training_fits_a_smooth_function():
    F, H = 2, 16
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, (256, F))
    t = np.sin(2 * X[:, 0]) * X[:, 1]
    th = mlp.init_params(F, H, 4)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    L0 = mlp.loss_and_grad(th, X, t, H)[0]
    for s in range(1, 801):
        L, g = mlp.loss_and_grad(th, X, t, H)
        th, m, v = mlp.adam_step(th, g, m, v, s, 1e-2)
    assert L < 0.02 * L0
