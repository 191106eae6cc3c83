"""The 30-qubit cross-entropy study of Methods B (Fig. 3 and Fig. 4) on the
GPU path: approximate amplitudes from a fraction f = 2^-D of the slices
(Methods A, Eq. 3), top-k post-selection over all 2^n strings, and the XEB
(Eq. 1) of the selected strings against the exact probabilities, next to
Metropolis samples drawn from the same approximate probabilities.

Everything heavy runs in the library: the contraction (all n qubits open,
one 2^n-amplitude accumulator), the selection (lf_postselect_topk over
2^n candidates), the probabilities of the selected strings
(lf_probabilities_at) and the sampler (lf_mcmc_sample).  The slices are
added in increasing order, so the accumulator passes through every prefix:
after [0, 2^(S-D)) it holds the D prefix, is selected and sampled there, and
after all 2^S slices it holds the exact amplitudes, which then give q for
every selection made on the way.  The XEB sums (float64) are taken on the
host from the gathered q.

Expected values: top-k XEB = F ln(|S~|/k) (Eq. 4, with F the fidelity of the
prefix); XEB of samples from p over the candidate set = F (Eq. 3).
"""

from __future__ import annotations

import math
import time

import numpy as np

from . import api

# planner settings for the all-open 30-qubit network (search effort; the
# tree only sets speed and memory)
PLAN_OPTS = dict(max_log2=32, sa_iters=1_000_000, restarts=4)
K_VALUES = tuple(1 << e for e in range(8, 16))


def run(d_values=(1, 2, 3, 4, 5), k_max: int = 1 << 15, mcmc_chains: int = 1 << 14,
        mcmc_per_chain: int = 64, mcmc_burn_in: int = 256, mcmc_thin: int = 16,
        mcmc_seed: int = 31, dtype: str = "c64", on_prefix=None, say=None):
    """Returns a dict of results; on_prefix(D, amps) is called with the
    accumulator holding the D prefix (amps: complex128 [1, 2^n] on the GPU)
    and on_prefix(0, amps) with the exact amplitudes."""
    import torch

    import workloads as wl

    def log(msg):
        if say:
            say(msg)

    circ, openq, cb, spec = wl.standard_workload("rqc30")
    n = circ.n_qubits
    N = 1 << n
    openq = [int(q) for q in openq]
    if openq != list(range(openq[0], openq[0] + len(openq))):
        raise ValueError("the candidate layout needs consecutive open qubits")
    t0 = time.time()
    plan = api.Plan(circ, list(range(n)), [0], dtype=dtype, sliced_wires=wl.RQC30_SLICED_WIRES,
                    check_overflow=False, **PLAN_OPTS)
    info = plan.info()
    S = info["n_sliced_wires"]
    plan.bind()
    amps = plan.new_amplitudes()
    flat = amps.view(-1)
    closed = wl.closed_bitstrings(n, openq, wl.XEB_MCMC_STRINGS, seed=wl.XEB_MCMC_SEED)
    base = torch.from_numpy(closed.astype(np.int64)).cuda()
    stride = 1 << openq[0]
    group = 1 << len(openq)
    log(f"plan ready: {info['n_slices']} slices of {info['macs_per_slice']:.3g} multiply-adds, "
        f"{time.time() - t0:.1f} s")
    sel, samples, accepted, t_contract, t_select = {}, {}, {}, 0.0, 0.0
    done = 0
    for D in sorted(d_values, reverse=True):
        end = 1 << (S - D)
        torch.cuda.synchronize()
        t1 = time.time()
        plan.contract(done, end, amps)
        torch.cuda.synchronize()
        t_contract += time.time() - t1
        done = end
        t1 = time.time()
        idx, _ = api.postselect_topk(flat, N, k_max)
        torch.cuda.synchronize()
        t_select += time.time() - t1
        sel[D] = idx[0].clone()
        samples[D], accepted[D] = api.mcmc_sample(flat, base, group, stride, mcmc_chains,
                                                  mcmc_burn_in, mcmc_thin, mcmc_per_chain,
                                                  mcmc_seed + D)
        if on_prefix:
            on_prefix(D, amps)
        log(f"D={D}: slices [0, {end}) contracted, top-{k_max} selected, "
            f"{mcmc_chains * mcmc_per_chain} samples drawn")
    torch.cuda.synchronize()
    t1 = time.time()
    plan.contract(done, 1 << S, amps)
    torch.cuda.synchronize()
    t_contract += time.time() - t1
    if on_prefix:
        on_prefix(0, amps)
    out = {"n_qubits": n, "n_slices": 1 << S, "k_values": list(K_VALUES),
           "macs_per_slice": info["macs_per_slice"], "contract_s": t_contract,
           "select_s": t_select, "mcmc_samples": mcmc_chains * mcmc_per_chain,
           "mcmc_candidates": int(closed.size) * group}
    for D in sorted(d_values):
        q = api.probabilities_at(flat, sel[D]).cpu().numpy()
        cq = np.cumsum(q)
        out[f"topk_idx_D{D}"] = sel[D].cpu().numpy()
        out[f"xeb_topk_D{D}"] = [float(N * cq[k - 1] / k - 1.0) for k in K_VALUES if k <= k_max]
        qm = api.probabilities_at(flat, samples[D]).cpu().numpy()
        out[f"xeb_mcmc_D{D}"] = float(N * qm.mean() - 1.0)
        out[f"mcmc_acceptance_D{D}"] = float(accepted[D].sum().item()) / (
            mcmc_chains * (mcmc_burn_in + mcmc_per_chain * mcmc_thin))
    out["seconds"] = time.time() - t0
    plan.workspace = None
    plan.close()
    return out


def eq4(fidelity: float, n_candidates: int, k: int) -> float:
    """Eq. 4: expected XEB of the top k of n_candidates at fidelity F."""
    return fidelity * math.log(n_candidates / k)
