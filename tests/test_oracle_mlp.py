"""Pins of the oracle network (oracle/mlp.py) against things fixed outside it:
closed-form GELU values, finite differences of the loss, the first Adam step,
and a network reduced to a linear least-squares model."""
import numpy as np
import pytest
from scipy.stats import norm

from oracle import mlp

SHAPE = (5, 7, 2, 3)   # n_in, width, depth, n_out


def test_gelu_closed_forms():
    x = np.array([-2.0, -1.0, 0.0, 0.5, 1.0, 3.0])
    assert np.allclose(mlp.gelu(x), x * norm.cdf(x), rtol=0, atol=1e-15)
    assert mlp.gelu(0.0) == 0.0
    assert abs(mlp.gelu_prime(0.0) - 0.5) < 1e-16
    # derivative against central differences of the function
    h = 1e-6
    assert np.allclose(mlp.gelu_prime(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h), atol=1e-9)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    n = mlp.n_params(*SHAPE)
    p = rng.standard_normal(n) * 0.5
    X = rng.standard_normal((4, SHAPE[0]))
    T = rng.standard_normal((4, SHAPE[3]))
    loss, g = mlp.loss_grad(p, X, T, *SHAPE)
    h = 1e-6
    fd = np.empty(n)
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        fd[k] = (mlp.loss_grad(p + e, X, T, *SHAPE)[0] - mlp.loss_grad(p - e, X, T, *SHAPE)[0]) / (2 * h)
    assert np.abs(g - fd).max() < 1e-7 * max(1.0, np.abs(fd).max())


def test_linear_reduction_is_least_squares():
    """With the hidden weights making every hidden unit 0 (GELU(0) = 0) the
    output is the last bias; the loss gradient w.r.t. that bias is the mean
    residual, as for a constant least-squares fit."""
    rng = np.random.default_rng(1)
    n = mlp.n_params(*SHAPE)
    p = np.zeros(n)
    layers = mlp.unpack(p, *SHAPE)
    layers[-1][1][:] = [0.5, -1.0, 2.0]
    X = rng.standard_normal((6, SHAPE[0]))
    T = rng.standard_normal((6, SHAPE[3]))
    Y, _ = mlp.forward(p, X, *SHAPE)
    assert np.allclose(Y, [0.5, -1.0, 2.0])
    loss, g = mlp.loss_grad(p, X, T, *SHAPE)
    gb = mlp.unpack(g, *SHAPE)[-1][1]
    assert np.allclose(gb, 2.0 * (Y - T).sum(axis=0) / T.size)
    assert np.isclose(loss, np.mean((Y - T) ** 2))


def test_adam_first_step():
    """With zero moments the bias-corrected first step moves each parameter by
    lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
