"""What the trained step-cost network gains over the FLOP+memory cost.

The committed network (trained on the GPU by the library's own kernels on
measured step timings of 53-qubit, 20-cycle plans) is evaluated on committed
held-out timings that were not used in training.  The comparison is the
FLOP+memory cost with an affine map to log seconds fitted on the held-out
set itself, i.e. its best possible calibration.  The CPU check runs the
network through the float64 oracle network; the GPU check runs it through
the library's forward kernel."""

import os

import numpy as np
import pytest

from oracle import mlp as omlp

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2406_18889_amd", "data")
MODEL = os.path.join(DATA, "costmodel_mi355x.npz")
HELDOUT = os.path.join(DATA, "costmodel_heldout.npz")


def _load():
    m = np.load(MODEL, allow_pickle=False)
    h = np.load(HELDOUT, allow_pickle=False)
    return m, h


def _flopmem_log_seconds(dims):
    """Plain FLOP + bytes cost of a step, as the planner's fallback counts
    it: 8 real flops per complex multiply-add at the MFMA peak of the step's
    arithmetic, plus operand and result bytes at HBM bandwidth, plus a fixed
    launch cost."""
    nz, nm, nn, nk = (dims[:, i].astype(np.float64) for i in range(4))
    half = dims[:, 5] == 1
    macs = 2.0 ** (nz + nm + nn + nk)
    es = np.where(half, 4.0, 8.0)
    byts = es * (2.0 ** (nz + nm + nk) + 2.0 ** (nz + nn + nk) + 2.0 ** (nz + nm + nn))
    peak = np.where(half, 2.5e15, 157.3e12)
    return np.log(8 * macs / peak + byts / 8e12 + 3e-6)


def _affine_best_mse(x, y):
    A = np.stack([x, np.ones_like(x)], 1)
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    return float(np.mean((A @ coef - y) ** 2))


def _oracle_predict(m, X):
    n_in, H = int(m["x_mean"].size), 128
    flat = m["params"].astype(np.float64)
    p, o = {}, 0
    for name, shape in (("W1", (n_in, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
                        ("W3", (H, 1)), ("b3", (1,))):
        k = int(np.prod(shape))
        p[name] = flat[o:o + k].reshape(shape)
        o += k
    Xn = (X.astype(np.float64) - m["x_mean"]) / m["x_std"]
    y, _ = omlp.forward(p, Xn)
    return y.reshape(-1) * float(m["y_std"]) + float(m["y_mean"])


def test_trained_network_beats_flopmem_on_heldout_steps():
    m, h = _load()
    X, y, dims = h["X"], h["y"], h["dims"]
    assert len(y) >= 1000
    mse_net = float(np.mean((_oracle_predict(m, X) - y) ** 2))
    mse_fm = _affine_best_mse(_flopmem_log_seconds(dims), y)
    # log-seconds errors: the network must at least halve the best-calibrated
    # FLOP+memory error
    assert mse_net < 0.5 * mse_fm, (mse_net, mse_fm)
    # and it ranks steps better (Spearman correlation)
    def ranks(v):
        r = np.empty(len(v))
        r[np.argsort(v)] = np.arange(len(v))
        return r
    rho_net = np.corrcoef(ranks(_oracle_predict(m, X)), ranks(y))[0, 1]
    rho_fm = np.corrcoef(ranks(_flopmem_log_seconds(dims)), ranks(y))[0, 1]
    assert rho_net > rho_fm


@pytest.mark.gpu
def test_trained_network_gpu_forward_matches_oracle_on_heldout():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_18889_amd import costmodel
    m, h = _load()
    model = costmodel.load(MODEL)
    got = costmodel.predict(model, h["X"][:2000])
    ref = _oracle_predict(m, h["X"][:2000])
    assert np.max(np.abs(got - ref)) < 1e-3 * max(1.0, float(np.max(np.abs(ref))))


AB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                  "costmodel_ab_rqc53.json")


@pytest.mark.skipif(not os.path.exists(AB), reason="end-to-end comparison record not committed")
def test_end_to_end_record_of_the_learned_ranking():
    """The committed end-to-end comparison (measured runtime as the judge):
    seeded 53-qubit, 20-cycle circuits planned twice with the same seeds and
    restarts, the refined candidate kept by the FLOP+memory cost or by the
    trained network, each plan's slices/s measured on the GPU and its
    whole-network time = 2^S / (slices/s).  The record must cover at least
    six circuits, and its reported gains must follow from its own measured
    fields (the geometric mean of FLOP+memory network time over learned
    network time).  The value itself is the result, whichever side of 1 it
    falls on."""
    import json
    import math
    with open(AB) as f:
        rec = json.load(f)
    runs = rec["runs"]
    assert rec["circuits"] == len(runs) >= 6
    logs = []
    for r in runs:
        for side in ("flopmem", "mlp"):
            assert r[side]["slices_per_s"] > 0
            t = r[side]["n_sliced"] - math.log2(r[side]["slices_per_s"])
            assert abs(t - r[side]["log2_network_seconds"]) < 1e-9
        g = 2.0 ** (r["flopmem"]["log2_network_seconds"] - r["mlp"]["log2_network_seconds"])
        assert abs(g / r["gain_network_time"] - 1) < 1e-9
        if r["same_choice"]:
            assert r["flopmem"]["n_sliced"] == r["mlp"]["n_sliced"]
        logs.append(math.log(g))
    gm = math.exp(sum(logs) / len(logs))
    assert abs(gm / rec["geomean_gain_network_time"] - 1) < 1e-9
    assert rec["differing_choices"] == sum(not r["same_choice"] for r in runs)
