"""Pins of the float64 cost-model network: analytic gradients against
central finite differences, the first Adam step against its closed form,
and a fit of a known function."""

import math

import numpy as np
import pytest

from oracle import mlp


@pytest.fixture(scope="module")
def small():
    rng = np.random.Generator(np.random.PCG64(1))
    X = rng.standard_normal((32, 9))
    t = rng.standard_normal(32)
    p = mlp.init(9, hidden=16, seed=2)
    return p, X, t


def test_gradients_match_finite_differences(small):
    p, X, t = small
    _, g = mlp.gradients(p, X, t)
    rng = np.random.Generator(np.random.PCG64(3))
    for name in mlp.NAMES:
        for _ in range(6):
            idx = tuple(int(rng.integers(s)) for s in p[name].shape)
            num = mlp.numeric_gradient(p, X, t, name, idx)
            ana = g[name][idx]
            assert abs(num - ana) <= 1e-6 * max(1.0, abs(num)), (name, idx, num, ana)


def test_loss_is_mean_squared_error(small):
    p, X, t = small
    y, _ = mlp.forward(p, X)
    # layer by layer with explicit loops on two rows
    for r in range(2):
        h1 = [max(0.0, sum(X[r, i] * p["W1"][i, j] for i in range(9)) + p["b1"][j]) for j in range(16)]
        h2 = [max(0.0, sum(h1[i] * p["W2"][i, j] for i in range(16)) + p["b2"][j]) for j in range(16)]
        yy = sum(h2[i] * p["W3"][i, 0] for i in range(16)) + p["b3"][0]
        assert abs(yy - y[r]) < 1e-12
    assert abs(mlp.loss(p, X, t) - np.mean((y - t) ** 2)) < 1e-15


def test_first_adam_step_closed_form(small):
    p, X, t = small
    _, g = mlp.gradients(p, X, t)
    m, v = mlp.adam_init(p)
    lr, eps = 1e-2, 1e-8
    q, m1, v1 = mlp.adam_step(p, g, m, v, 1, lr=lr, eps=eps)
    # bias-corrected first moments equal g and g^2: step = lr g / (|g| + eps)
    for k in p:
        assert np.allclose(q[k], p[k] - lr * g[k] / (np.abs(g[k]) + eps), rtol=1e-12, atol=1e-15)


def test_fits_a_smooth_function():
    rng = np.random.Generator(np.random.PCG64(4))
    X = rng.uniform(-1, 1, (256, 4))
    t = np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2]
    p = mlp.init(4, hidden=32, seed=5)
    m, v = mlp.adam_init(p)
    l0 = mlp.loss(p, X, t)
    for step in range(1, 401):
        _, g = mlp.gradients(p, X, t)
        p, m, v = mlp.adam_step(p, g, m, v, step, lr=1e-2)
    assert mlp.loss(p, X, t) < 0.05 * l0
