"""Writes the stored expected values for the 30-qubit, 14-cycle workload.

Calls only the oracle (state vector in complex128) and the seeded input
generators; nothing here touches the library.  A 30-qubit state takes
16 GiB of host memory and one run takes minutes on 8 cores.

  python -m tests.golden.make_rqc30 exact
      rqc30_exact.npy  A[b, j] for the 256 closed strings x 64 open values
      rqc30_stats.json norm, Porter-Thomas moments, ideal top-k XEB values
  python -m tests.golden.make_rqc30 prefix
      rqc30_prefix_D{D}.npy  partial sums over the slice prefix
      [0, 2^(S-D)), i.e. the D most significant sliced wires fixed to 0
      rqc30_prefix.json      their fidelity against the exact state
  python -m tests.golden.make_rqc30 xeb
      rqc30_xeb.json      top-k XEB (Eq. 1, exact q) of each prefix state for
                          k = 2^8..2^15 over all 2^30 strings, and the exact
                          XEB expectation of sampling from each prefix's p
                          over the MCMC candidate set
      rqc30_xeb_topk.npz  the oracle's top-2^15 indices per prefix
  python -m tests.golden.make_rqc30 batch
      rqc30_batch_sample.npz  exact amplitudes of 1024 of the 2^20 closed
                              strings of the candidate set (64 open values)
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import sv, topk  # noqa: E402

# The eight sliced wires (qubit, j) of the 30-qubit workload (defined with
# the workload; any eight wires give a valid test of the slicing identity).
RQC30_SLICED_WIRES = wl.RQC30_SLICED_WIRES


def exact():
    circ, openq, cb, spec = wl.standard_workload("rqc30")
    t0 = time.time()
    psi = sv.run(circ)
    t_sv = time.time() - t0
    idx = sv.group_indices(circ.n_qubits, openq, cb)
    amps = sv.gather(psi, idx).reshape(len(cb), 1 << len(openq))
    np.save(os.path.join(HERE, "rqc30_exact.npy"), amps)
    N = psi.size
    m2, m3 = sv.moments(psi)
    nrm = sv.norm2(psi)
    # ideal global top-k over all 2^30 strings, k = 2^15 (Methods B study)
    p = sv.probs(psi)
    del psi
    k = 1 << 15
    part = np.argpartition(p, N - k)[N - k:]
    x_topk = topk.xeb(p[part], circ.n_qubits)
    del p, part
    # ideal per-group top-1 over the 256 groups of 64
    gi, _ = topk.topk(amps, 64, 1)
    q1 = topk.probabilities(amps[np.arange(len(cb)), gi[:, 0]])
    stats = dict(norm2=nrm, N_m2=N * m2, N2_m3=N * N * m3, xeb_top_2p15_of_2p30=x_topk,
                 xeb_top1_per_group64=topk.xeb(q1, circ.n_qubits),
                 sv_seconds=t_sv, threads=len(os.sched_getaffinity(0)))
    with open(os.path.join(HERE, "rqc30_stats.json"), "w") as f:
        json.dump(stats, f, indent=1)
    print(json.dumps(stats))


def prefix(d_values=(1, 2, 3, 4, 5)):
    circ, openq, cb, spec = wl.standard_workload("rqc30")
    S = len(RQC30_SLICED_WIRES)
    counts = [0] * circ.n_qubits
    for g in circ.gates:
        if len(g.qubits) == 2:
            for q in g.qubits:
                counts[q] += 1
    for (q, j) in RQC30_SLICED_WIRES:
        if not 1 <= j < counts[q]:
            raise ValueError(f"wire ({q}, {j}) is not an internal wire")
    psi = sv.run(circ)
    nrm = sv.norm2(psi)
    out = {"sliced_wires": RQC30_SLICED_WIRES}
    idx = sv.group_indices(circ.n_qubits, openq, cb)
    buf = np.empty_like(psi)
    for D in d_values:
        projs = [(q, j, 0) for (q, j) in RQC30_SLICED_WIRES[S - D:]]
        sv.run(circ, projs, out=buf)
        amps = sv.gather(buf, idx).reshape(len(cb), 1 << len(openq))
        np.save(os.path.join(HERE, f"rqc30_prefix_D{D}.npy"), amps)
        ov = abs(np.vdot(psi, buf)) ** 2 / (nrm * sv.norm2(buf))
        out[f"fidelity_D{D}"] = ov
        print(D, ov, flush=True)
    with open(os.path.join(HERE, "rqc30_prefix.json"), "w") as f:
        json.dump(out, f, indent=1)


# Methods B experiment on this circuit: S~ for the MCMC baseline is 2^20
# closed strings of the 24 closed qubits times the 64 values of the open
# qubits 24..29 (2^26 candidates); the top-k selection runs over all 2^30
# strings.  D = 1..5 prefixes as above.
XEB_MCMC_STRINGS = wl.XEB_MCMC_STRINGS
XEB_MCMC_SEED = wl.XEB_MCMC_SEED
XEB_K_MAX = 1 << 15


def xeb_candidates():
    """Basis indices of the MCMC candidate set S~ (b-major, open value j minor)."""
    circ, openq, cb, spec = wl.standard_workload("rqc30")
    closed = wl.closed_bitstrings(circ.n_qubits, openq, XEB_MCMC_STRINGS, seed=XEB_MCMC_SEED)
    return sv.group_indices(circ.n_qubits, openq, closed)


def xeb(d_values=(1, 2, 3, 4, 5)):
    """Oracle top-k XEB (Eq. 1 with exact q) of the approximate prefix states,
    for k = 2^8 .. 2^15 over all 2^30 strings, and the exact expectation of
    the XEB of samples drawn from the approximate p restricted to S~ (what an
    MCMC sampler converges to; Eq. 3 predicts it equals the fidelity)."""
    circ, openq, cb, spec = wl.standard_workload("rqc30")
    n = circ.n_qubits
    N = 1 << n
    S = len(RQC30_SLICED_WIRES)
    t0 = time.time()
    psi = sv.run(circ)
    q = sv.probs(psi)
    del psi
    cand = xeb_candidates().astype(np.int64)
    q_c = q[cand]
    out = {"k_values": [1 << e for e in range(8, 16)], "n_candidates_topk": N,
           "mcmc_candidates": int(cand.size), "mcmc_strings": XEB_MCMC_STRINGS,
           "mcmc_seed": XEB_MCMC_SEED}
    buf = np.empty(N, np.complex128)
    kk = XEB_K_MAX + 4096
    top_idx = {}
    for D in d_values:
        projs = [(qq, j, 0) for (qq, j) in RQC30_SLICED_WIRES[S - D:]]
        sv.run(circ, projs, out=buf)
        p = sv.probs(buf)
        # top k by (p descending, index ascending): a partition to a margin,
        # then an exact lexsort of the margin
        part = np.argpartition(p, N - kk)[N - kk:]
        order = part[np.lexsort((part, -p[part]))][:XEB_K_MAX]
        top_idx[D] = order.astype(np.int32)
        cq = np.cumsum(q[order])
        out[f"xeb_topk_D{D}"] = [float(N * cq[k - 1] / k - 1.0) for k in out["k_values"]]
        # sampling from p over S~: E[N q] under p / sum p, and its spread
        w = p[cand]
        z = w.sum()
        m1 = float((w * q_c).sum() / z) * N
        m2 = float((w * q_c * q_c).sum() / z) * N * N
        out[f"mcmc_xeb_expect_D{D}"] = m1 - 1.0
        out[f"mcmc_nq_std_D{D}"] = float(np.sqrt(max(0.0, m2 - m1 * m1)))
        print(D, out[f"xeb_topk_D{D}"][-1], out[f"mcmc_xeb_expect_D{D}"], flush=True)
        del p, w
    out["seconds"] = time.time() - t0
    out["threads"] = len(os.sched_getaffinity(0))
    np.savez_compressed(os.path.join(HERE, "rqc30_xeb_topk.npz"),
                        **{f"D{D}": v for D, v in top_idx.items()})
    with open(os.path.join(HERE, "rqc30_xeb.json"), "w") as f:
        json.dump(out, f, indent=1)


BATCH_SAMPLE_ROWS = 1024
BATCH_SAMPLE_SEED = 77


def batch_sample_rows():
    """Rows (closed strings) of the 2^20-string candidate set that the
    stored large-batch values cover: 1024 drawn without replacement."""
    rng = np.random.Generator(np.random.PCG64(BATCH_SAMPLE_SEED))
    return np.sort(rng.choice(XEB_MCMC_STRINGS, BATCH_SAMPLE_ROWS, replace=False)).astype(np.int64)


def batch():
    """Exact amplitudes of 1024 of the 2^20 closed strings of the candidate
    set (all 64 open values each), for the large-batch sparse output."""
    circ, openq, cb, spec = wl.standard_workload("rqc30")
    closed = wl.closed_bitstrings(circ.n_qubits, openq, XEB_MCMC_STRINGS, seed=XEB_MCMC_SEED)
    rows = batch_sample_rows()
    psi = sv.run(circ)
    idx = sv.group_indices(circ.n_qubits, openq, closed[rows])
    amps = sv.gather(psi, idx).reshape(rows.size, 1 << len(openq))
    np.savez_compressed(os.path.join(HERE, "rqc30_batch_sample.npz"), rows=rows, amps=amps)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "exact"
    if what == "exact":
        exact()
    elif what == "prefix":
        prefix()
    elif what == "xeb":
        xeb()
    elif what == "batch":
        batch()
    else:
        raise SystemExit("usage: make_rqc30 exact|prefix|xeb|batch")
