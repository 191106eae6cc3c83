"""Learned step-cost model: measured step timings -> trained network ->
planner cost.

The network (in -> 128 -> 128 -> 1, ReLU, float32) maps a contraction
step's features (lf_step_features) to the log of its measured run time.
Training runs on the GPU through the library's own kernels
(lf_mlp_gradients, lf_mlp_adam_step); the trained network is handed to the
planner with lf_costmodel_load, after which plans built with
cost_model="mlp" sum predicted step times instead of FLOP and byte counts.

  python -m paper_2406_18889_amd.costmodel collect --out data.npz [--steps 50000]
  python -m paper_2406_18889_amd.costmodel train --data data.npz --out model.npz
"""

from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import time
from typing import List, Optional, Tuple

import numpy as np

from . import _lib
from ._lib import check

N_FEATURES = _lib.LF_N_FEATURES
HIDDEN = 128
DEFAULT_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                             "costmodel_mi355x.npz")


def features(dims: np.ndarray) -> np.ndarray:
    """Feature rows for plan steps (dims rows as returned by Plan.steps())."""
    lib = _lib.load()
    out = np.zeros((len(dims), N_FEATURES), np.float32)
    buf = (ctypes.c_float * N_FEATURES)()
    for i, d in enumerate(dims):
        check(lib.lf_step_features(int(d[0]), int(d[1]), int(d[2]), int(d[3]), int(d[5]), buf),
              "lf_step_features")
        out[i] = np.frombuffer(buf, np.float32)
    return out


def init_params(n_in: int = N_FEATURES, hidden: int = HIDDEN, seed: int = 0) -> np.ndarray:
    """Uniform(+-1/sqrt(fan_in)) initial parameters in the library's layout."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_in, n in ((n_in, n_in * hidden), (n_in, hidden), (hidden, hidden * hidden),
                      (hidden, hidden), (hidden, hidden), (hidden, 1)):
        lim = 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, n))
    return np.concatenate(parts).astype(np.float32)


class CostNet:
    """The network's parameters on the GPU, with Adam state."""

    def __init__(self, params: np.ndarray, n_in: int = N_FEATURES, hidden: int = HIDDEN,
                 max_batch: int = 4096):
        import torch
        lib = _lib.load()
        npar = ctypes.c_int64()
        wsb = ctypes.c_uint64()
        check(lib.lf_mlp_sizes(n_in, hidden, max_batch, ctypes.byref(npar), ctypes.byref(wsb)),
              "lf_mlp_sizes")
        if params.size != npar.value:
            raise ValueError("parameter array has the wrong size")
        self.n_in, self.hidden, self.max_batch = n_in, hidden, max_batch
        self.p = torch.from_numpy(np.ascontiguousarray(params, np.float32)).cuda()
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.g = torch.zeros_like(self.p)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.ws = torch.empty(int(wsb.value) // 4 + 64, dtype=torch.float32, device="cuda")
        self.ws_bytes = self.ws.numel() * 4
        self.step = 0

    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def forward(self, X):
        import torch
        X = X.contiguous()
        Y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        for s in range(0, X.shape[0], self.max_batch):
            e = min(X.shape[0], s + self.max_batch)
            check(_lib.load().lf_mlp_forward(ctypes.c_void_p(self.p.data_ptr()), self.n_in, self.hidden,
                                             ctypes.c_void_p(X[s:e].data_ptr()), e - s,
                                             ctypes.c_void_p(Y[s:e].data_ptr()),
                                             ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                             self._stream()), "lf_mlp_forward")
        return Y

    def gradients(self, X, T):
        X, T = X.contiguous(), T.contiguous()
        check(_lib.load().lf_mlp_gradients(ctypes.c_void_p(self.p.data_ptr()), self.n_in, self.hidden,
                                           ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                           X.shape[0], ctypes.c_void_p(self.g.data_ptr()),
                                           ctypes.c_void_p(self.loss.data_ptr()),
                                           ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                           self._stream()), "lf_mlp_gradients")
        return self.g, self.loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        check(_lib.load().lf_mlp_adam_step(ctypes.c_void_p(self.p.data_ptr()),
                                           ctypes.c_void_p(self.m.data_ptr()),
                                           ctypes.c_void_p(self.v.data_ptr()),
                                           ctypes.c_void_p(self.g.data_ptr()), self.p.numel(),
                                           self.step, lr, beta1, beta2, eps, self._stream()),
              "lf_mlp_adam_step")


def train(X: np.ndarray, t: np.ndarray, epochs: int = 60, batch: int = 512, lr: float = 2e-3,
          seed: int = 0, log=None):
    """Fits the network on (features, log seconds) with lf_costmodel_train
    (standardisation, shuffling, batches, gradients and Adam all in the
    library); returns a model dict and the per-epoch training loss
    (standardised units)."""
    import torch
    X = np.ascontiguousarray(X, np.float32)
    t = np.ascontiguousarray(t, np.float32)
    n, n_in = X.shape
    p = torch.from_numpy(init_params(n_in, HIDDEN, seed=seed)).cuda()
    xm = np.zeros(n_in, np.float32)
    xs = np.zeros(n_in, np.float32)
    ym = ctypes.c_float()
    ys = ctypes.c_float()
    curve = np.zeros(epochs, np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    check(_lib.load().lf_costmodel_train(X.ctypes.data_as(fp), t.ctypes.data_as(fp), n, n_in, HIDDEN,
                                         epochs, batch, lr, seed, ctypes.c_void_p(p.data_ptr()),
                                         xm.ctypes.data_as(fp), xs.ctypes.data_as(fp), ctypes.byref(ym),
                                         ctypes.byref(ys), curve.ctypes.data_as(fp),
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
          "lf_costmodel_train")
    if log:
        for ep, v in enumerate(curve):
            log(f"epoch {ep} loss {v:.4f}")
    model = {"params": p.cpu().numpy(), "x_mean": xm, "x_std": xs, "y_mean": float(ym.value),
             "y_std": float(ys.value)}
    return model, [float(v) for v in curve]


def predict(model, X: np.ndarray) -> np.ndarray:
    """Predicted log seconds through the GPU forward kernel."""
    import torch
    net = CostNet(model["params"])
    Xn = torch.from_numpy(((X - model["x_mean"]) / model["x_std"]).astype(np.float32)).cuda()
    y = net.forward(Xn).cpu().numpy().astype(np.float64)
    return y * model["y_std"] + model["y_mean"]


def load_into_planner(model) -> None:
    lib = _lib.load()
    p = np.ascontiguousarray(model["params"], np.float32)
    xm = np.ascontiguousarray(model["x_mean"], np.float32)
    xs = np.ascontiguousarray(model["x_std"], np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    check(lib.lf_costmodel_load(p.ctypes.data_as(fp), N_FEATURES, HIDDEN, xm.ctypes.data_as(fp),
                                xs.ctypes.data_as(fp), float(model["y_mean"]), float(model["y_std"])),
          "lf_costmodel_load")


def clear_planner() -> None:
    check(_lib.load().lf_costmodel_clear(), "lf_costmodel_clear")


def save(model, path: str) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=model["params"], x_mean=model["x_mean"], x_std=model["x_std"],
             y_mean=model["y_mean"], y_std=model["y_std"])


def load(path: str = DEFAULT_MODEL):
    d = np.load(path, allow_pickle=False)
    return {k: d[k] for k in ("params", "x_mean", "x_std")} | {
        "y_mean": float(d["y_mean"]), "y_std": float(d["y_std"])}


def flopmem_seconds(dims: np.ndarray) -> np.ndarray:
    """The planner's fallback cost of each step (roofline sum + launch)."""
    out = np.zeros(len(dims))
    for i, d in enumerate(dims):
        nz, nm, nn, nk, dt = (int(x) for x in (d[0], d[1], d[2], d[3], d[5]))
        macs = 2.0 ** (nz + nm + nn + nk)
        es = 4.0 if dt else 8.0
        byts = es * (2.0 ** (nz + nm + nk) + 2.0 ** (nz + nn + nk) + 2.0 ** (nz + nm + nn))
        out[i] = 8 * macs / (2.5e15 if dt else 157.3e12) + byts / 8e12 + 3e-6
    return out


# ------------------------------------------------------------- collection
def collect(target_steps: int = 50_000, seed: int = 0, reps: int = 2, log=print,
            time_budget: float = 1e9, workers: int = 12,
            sa_iters: int = 200_000) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Times every step of many plans for 53-qubit, 20-cycle circuits (other
    circuit seeds, caps 2^27..2^30, both arithmetics, 1/16/256 closed
    strings) with the library's per-step HIP-event profiler.  Plans are
    searched on `workers` host threads (the planner runs outside the
    interpreter lock) while the GPU profiles the previous ones.  Returns
    (features, log seconds, dims)."""
    import concurrent.futures as cf

    import torch

    import workloads as wl
    from .api import Plan

    rng = np.random.Generator(np.random.PCG64(seed))

    def spec(k):
        cseed = int(rng.integers(1, 1 << 30))
        cap = int(rng.integers(27, 31))   # below 2^27 the search rarely fits
        nb = int(rng.choice([1, 16, 256]))
        return dict(k=k, cseed=cseed, cap=cap, dtype="chalf" if k % 2 else "c64", nb=nb,
                    rem=int(rng.integers(1, 1000)), bseed=int(rng.integers(1, 1 << 30)),
                    pseed=int(rng.integers(1, 1 << 30)))

    def make(sp):
        circ = wl.random_circuit(6, 9, 20, sp["cseed"], 1, sp["rem"])
        openq = list(range(circ.n_qubits - 10, circ.n_qubits))
        cb = wl.closed_bitstrings(circ.n_qubits, openq, sp["nb"], sp["bseed"])
        try:
            return Plan(circ, openq, cb, dtype=sp["dtype"], max_log2=sp["cap"], sa_iters=sa_iters,
                        seed=sp["pseed"], check_overflow=False)
        except Exception as e:  # infeasible at this cap
            return e

    Xs, ts, ds = [], [], []
    n = 0
    t0 = time.time()
    k = 0
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        pending = [(sp, ex.submit(make, sp)) for sp in (spec(i) for i in range(2 * workers))]
        k = len(pending)
        while pending and n < target_steps and time.time() - t0 < time_budget:
            sp, fut = pending.pop(0)
            nxt = spec(k)
            pending.append((nxt, ex.submit(make, nxt)))
            k += 1
            plan = fut.result()
            if isinstance(plan, Exception):
                log(f"plan {sp['k']}: {plan}")
                continue
            plan.bind()
            ms = plan.profile_steps(reps=reps)
            dims, _, _ = plan.steps()
            Xs.append(features(dims))
            ts.append(np.log(np.maximum(ms, 1e-6) * 1e-3))
            ds.append(dims)
            n += len(dims)
            log(f"plan {sp['k']}: cap 2^{sp['cap']} {sp['dtype']} B={sp['nb']}: {len(dims)} steps, "
                f"total {n} ({time.time() - t0:.0f} s)")
            plan.close()
            del plan
            torch.cuda.empty_cache()
        for _, fut in pending:
            fut.cancel()
    return np.concatenate(Xs), np.concatenate(ts), np.concatenate(ds)


def compare_rankings(model, n_circuits: int = 6, restarts: int = 4, sa_iters: int = 2_000_000,
                     seed: int = 99, slices: int = 6, log=print):
    """End-to-end comparison of the two ranking costs, decided by measured
    runtime: for seeded 53-qubit, 20-cycle circuits (cap 2^28, 256 closed
    strings, 10 open qubits, complex-half), plans searched with the same
    seeds and restarts, the refined candidate kept chosen by FLOP + memory
    or by the network; each plan's slices/s is measured and
    its whole-network time is n_slices / (slices/s)."""
    import concurrent.futures as cf

    import torch

    import workloads as wl
    from .api import Plan

    load_into_planner(model)
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for _ in range(n_circuits):
        circ = wl.random_circuit(6, 9, 20, int(rng.integers(1, 1 << 30)), 1, int(rng.integers(1, 1000)))
        openq = list(range(circ.n_qubits - 10, circ.n_qubits))
        cb = wl.closed_bitstrings(circ.n_qubits, openq, 256, int(rng.integers(1, 1 << 30)))
        specs.append((circ, openq, cb))

    def make(args):
        i, cost = args
        circ, openq, cb = specs[i]
        try:
            return Plan(circ, openq, cb, dtype="chalf", max_log2=28, sa_iters=sa_iters, cost_model=cost,
                        check_overflow=False, restarts=restarts, seed=1 + i)
        except Exception as e:  # infeasible
            return e

    def rate(p):
        p.bind()
        a = p.new_amplitudes()
        p.contract(0, 2, a)
        torch.cuda.synchronize()
        t = time.perf_counter()
        p.contract(2, 2 + slices, a)
        torch.cuda.synchronize()
        return slices / (time.perf_counter() - t)

    runs = []
    with cf.ThreadPoolExecutor(12) as ex:
        futs = {(i, c): ex.submit(make, (i, c)) for i in range(n_circuits) for c in ("flopmem", "mlp")}
        for i in range(n_circuits):
            pf, pm = futs[(i, "flopmem")].result(), futs[(i, "mlp")].result()
            if isinstance(pf, Exception) or isinstance(pm, Exception):
                log(f"circuit {i}: no plan ({pf if isinstance(pf, Exception) else pm})")
                continue
            fi, mi = pf.info(), pm.info()
            same = pf.sliced_wires() == pm.sliced_wires() and fi["macs_per_slice"] == mi["macs_per_slice"]
            rf = rate(pf)
            rm = rf if same else rate(pm)
            tf = fi["n_sliced_wires"] - math.log2(rf)
            tm = mi["n_sliced_wires"] - math.log2(rm)
            r = {"circuit": i, "same_choice": bool(same),
                 "flopmem": {"n_sliced": fi["n_sliced_wires"], "macs_per_slice": fi["macs_per_slice"],
                             "slices_per_s": rf, "log2_network_seconds": tf},
                 "mlp": {"n_sliced": mi["n_sliced_wires"], "macs_per_slice": mi["macs_per_slice"],
                         "slices_per_s": rm, "log2_network_seconds": tm},
                 "gain_network_time": float(2.0 ** (tf - tm))}
            log(json.dumps(r))
            runs.append(r)
            pf.close()
            pm.close()
            torch.cuda.empty_cache()
    g = [r["gain_network_time"] for r in runs]
    return {"restarts": restarts, "sa_iters": sa_iters, "circuits": len(runs),
            "differing_choices": sum(not r["same_choice"] for r in runs),
            "geomean_gain_network_time": float(np.exp(np.mean(np.log(g)))) if g else None, "runs": runs}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd")
    c = sub.add_parser("collect")
    c.add_argument("--out", required=True)
    c.add_argument("--steps", type=int, default=50_000)
    c.add_argument("--seed", type=int, default=0)
    c.add_argument("--budget", type=float, default=600.0)
    t = sub.add_parser("train")
    t.add_argument("--data", required=True)
    t.add_argument("--out", default=DEFAULT_MODEL)
    t.add_argument("--epochs", type=int, default=60)
    c2 = sub.add_parser("compare")
    c2.add_argument("--model", default=DEFAULT_MODEL)
    c2.add_argument("--circuits", type=int, default=6)
    c2.add_argument("--restarts", type=int, default=4)
    c2.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.cmd == "collect":
        X, y, d = collect(args.steps, args.seed, time_budget=args.budget)
        np.savez(args.out, X=X, y=y, dims=d)
        print(f"saved {len(y)} timings to {args.out}")
    elif args.cmd == "train":
        d = np.load(args.data, allow_pickle=False)
        X, y = d["X"], d["y"]
        rng = np.random.Generator(np.random.PCG64(7))
        perm = rng.permutation(len(y))
        n_test = max(1, len(y) // 10)
        te, tr = perm[:n_test], perm[n_test:]
        model, curve = train(X[tr], y[tr], epochs=args.epochs, log=print)
        pred = predict(model, X[te])
        mse = float(np.mean((pred - y[te]) ** 2))
        print(f"test MSE of log seconds: {mse:.4f} on {n_test} held-out steps")
        save(model, args.out)
    elif args.cmd == "compare":
        res = compare_rankings(load(args.model), args.circuits, args.restarts,
                               log=lambda m: print(m, flush=True))
        with open(args.out, "w") as f:
            json.dump(res, f)
        print(json.dumps({k: v for k, v in res.items() if k != "runs"}))
    else:
        ap.print_help()


if __name__ == "__main__":
    main()
