"""Oracle O6 (test infrastructure only): float64 reference of the step-cost
network.

A three-layer perceptron  x -> relu(x W1 + b1) -> relu(h1 W2 + b2) -> h2 W3 + b3
(widths in -> 128 -> 128 -> 1) regresses the log of a contraction step's
measured time from the step's features; it is fitted by mean squared error
with Adam (Kingma and Ba, "Adam: A Method for Stochastic Optimization",
Algorithm 1: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
theta <- theta - lr * m/(1-b1^t) / (sqrt(v/(1-b2^t)) + eps)).

Parameters are a dict of arrays W1 [in,H], b1 [H], W2 [H,H], b2 [H],
W3 [H,1], b3 [1].  Written out plainly, one matrix product per layer.
"""

from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def init(n_in: int, hidden: int = 128, seed: int = 0) -> Dict[str, np.ndarray]:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for (name, fan_in, shape) in (("W1", n_in, (n_in, hidden)), ("b1", n_in, (hidden,)),
                                  ("W2", hidden, (hidden, hidden)), ("b2", hidden, (hidden,)),
                                  ("W3", hidden, (hidden, 1)), ("b3", hidden, (1,))):
        lim = 1.0 / math.sqrt(fan_in)
        p[name] = rng.uniform(-lim, lim, size=shape)
    return p


def forward(p, X):
    """Returns (y [N], cache)."""
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ p["W3"] + p["b3"])[:, 0]
    return y, (X, z1, h1, z2, h2)


def loss(p, X, t) -> float:
    y, _ = forward(p, X)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def gradients(p, X, t) -> Tuple[float, Dict[str, np.ndarray]]:
    """Mean squared error and its gradient with respect to every parameter."""
    y, (X, z1, h1, z2, h2) = forward(p, X)
    t = np.asarray(t, np.float64)
    n = X.shape[0]
    dy = 2.0 * (y - t) / n                  # dL/dy
    g = {}
    g["W3"] = h2.T @ dy[:, None]
    g["b3"] = np.array([dy.sum()])
    dh2 = dy[:, None] @ p["W3"].T
    dz2 = dh2 * (z2 > 0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * (z1 > 0)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return float(np.mean((y - t) ** 2)), g


def adam_init(p):
    return {k: np.zeros_like(v) for k, v in p.items()}, {k: np.zeros_like(v) for k, v in p.items()}


def adam_step(p, g, m, v, step: int, lr: float = 1e-3, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    np_, nm, nv = {}, {}, {}
    for k in p:
        nm[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        nv[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k]
        mhat = nm[k] / (1.0 - beta1 ** step)
        vhat = nv[k] / (1.0 - beta2 ** step)
        np_[k] = p[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return np_, nm, nv


def numeric_gradient(p, X, t, name: str, index, h: float = 1e-6) -> float:
    """Central difference of the loss in one parameter entry."""
    q = {k: v.copy() for k, v in p.items()}
    q[name][index] += h
    lp = loss(q, X, t)
    q[name][index] -= 2 * h
    lm = loss(q, X, t)
    return (lp - lm) / (2 * h)
