"""The learned cost model's GPU kernels against the float64 oracle network,
and what the trained network adds over the FLOP+memory cost."""

import ctypes
import os
import sys

import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_18889_amd import costmodel
    return costmodel


def _to_oracle(flat, n_in, H):
    flat = flat.astype(np.float64)
    o = 0
    p = {}
    for name, shape in (("W1", (n_in, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
                        ("W3", (H, 1)), ("b3", (1,))):
        n = int(np.prod(shape))
        p[name] = flat[o:o + n].reshape(shape)
        o += n
    return p


def _flat(g):
    return np.concatenate([g[k].reshape(-1) for k in omlp.NAMES])


@pytest.mark.parametrize("batch", [1, 37, 512])
def test_forward_and_gradients_match_oracle(cm, batch):
    rng = np.random.Generator(np.random.PCG64(batch))
    X = rng.standard_normal((batch, cm.N_FEATURES)).astype(np.float32)
    T = rng.standard_normal(batch).astype(np.float32)
    flat = cm.init_params(seed=batch)
    net = cm.CostNet(flat, max_batch=512)
    dX, dT = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    y = net.forward(dX).cpu().numpy()
    g, loss = net.gradients(dX, dT)
    torch.cuda.synchronize()
    p = _to_oracle(flat, cm.N_FEATURES, cm.HIDDEN)
    y_ref, _ = omlp.forward(p, X.astype(np.float64))
    l_ref, g_ref = omlp.gradients(p, X.astype(np.float64), T.astype(np.float64))
    assert np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref) < 1e-5
    assert abs(loss.item() - l_ref) / l_ref < 1e-5
    gf = g.cpu().numpy().astype(np.float64)
    gr = _flat(g_ref)
    assert np.linalg.norm(gf - gr) / np.linalg.norm(gr) < 1e-4
    # per block as well, so a wrong small block cannot hide
    o = 0
    for k in omlp.NAMES:
        n = g_ref[k].size
        ref = g_ref[k].reshape(-1)
        if np.linalg.norm(ref) > 0:
            assert np.linalg.norm(gf[o:o + n] - ref) / np.linalg.norm(ref) < 1e-4, k
        o += n


def test_adam_matches_oracle(cm):
    rng = np.random.Generator(np.random.PCG64(9))
    X = rng.standard_normal((64, cm.N_FEATURES)).astype(np.float32)
    T = rng.standard_normal(64).astype(np.float32)
    flat = cm.init_params(seed=3)
    net = cm.CostNet(flat, max_batch=64)
    p = _to_oracle(flat, cm.N_FEATURES, cm.HIDDEN)
    m, v = omlp.adam_init(p)
    dX, dT = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    for step in range(1, 4):
        net.gradients(dX, dT)
        net.adam(lr=1e-3)
        _, g = omlp.gradients(p, X.astype(np.float64), T.astype(np.float64))
        p, m, v = omlp.adam_step(p, g, m, v, step, lr=1e-3)
    torch.cuda.synchronize()
    got = net.p.cpu().numpy().astype(np.float64)
    ref = _flat(p)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5


def test_training_reduces_loss(cm):
    rng = np.random.Generator(np.random.PCG64(5))
    X = rng.uniform(0, 20, (4096, cm.N_FEATURES)).astype(np.float32)
    t = (0.3 * X[:, 4] - 0.1 * X[:, 2] + np.sin(X[:, 3])).astype(np.float64)
    model, curve = cm.train(X, t, epochs=40, batch=256, lr=3e-3)
    assert curve[-1] < 0.3 * curve[0]
    pred = cm.predict(model, X[:512])
    assert np.mean((pred - t[:512]) ** 2) < 0.2 * np.var(t)
