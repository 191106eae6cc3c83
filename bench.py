"""Benchmark: sliced-subtask contractions per second on one MI355X.

A step contracts one chunk of slices of the workload into a float64
amplitude accumulator and runs the top-k post-selection on it (the whole hot
path).  Inputs (plan, leaves, workspace) are resident in HBM before timing.
Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rqc30|rqc53|mix512|xeb30|paper53]
                  [--dtype chalf|c64] [--slices-per-step S]
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MI355X = {"hbm_gbs": 8000.0, "fp16_tflops": 2500.0, "fp32_tflops": 157.3}
# kernel ids of the contraction steps; the large tiles are instances of
# gett_mfma_big<TO, WM, WN, MINB, ST, BK, FULL, ORDER>, named here by
# WM,WN,MINB,ST,BK,ORDER (a profiler lists FULL true and false separately)
KERNEL_NAMES = {0: "gett_thin", 1: "gett_mfma", 2: "gett_mfma_big<4,2,2,1,32,0>", 3: "gett_narrow",
                4: "gett_mfma_big<4,4,1,1,32,0>", 5: "gett_mfma_big<4,4,1,2,32,0>",
                6: "gett_mfma_big<4,4,1,1,64,0>", 7: "gett_skinny",
                8: "gett_mfma_big<4,2,2,1,32,1>", 9: "gett_mfma_big<4,4,1,2,32,1>",
                10: "gett_mfma_big<4,4,1,1,32,1>", 11: "gett_mfma_dma<0,8>", 12: "gett_mfma_dma<1,8>",
                13: "gett_mfma_dma<0,4>", 14: "gett_mfma_dma<1,4>",
                15: "gett_longk", 16: "gett_mfma_dma<0,4,128,2>", 17: "gett_mfma_dma<1,4,128,2>"}
# planner settings per workload (search effort, not inputs)
PLAN_OPTS = {"rqc53": {"sa_iters": 4_000_000, "restarts": 8, "chalf_exec_min_log2": 22}}
# the kernel choices (step shape and operand types -> kernel variant) the
# benchmark loads, so that every machine runs the same kernels; written by
# an autotuning run (--retune --save-autotune)
TUNE_FILE = os.path.join(ROOT, "paper_2406_18889_amd", "data", "autotune_mi355x.txt")


def source_hash():
    """Hash of the contraction kernels' sources and of the committed kernel
    choices: counter summaries taken with other kernels are not used."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip",):
        with open(os.path.join(ROOT, "paper_2406_18889_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if os.path.exists(TUNE_FILE):
        with open(TUNE_FILE, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def shape_key(name, d):
    return f"{name}|{int(d[0])},{int(d[1])},{int(d[2])},{int(d[3])}"


def traffic_for(workload, dtype, keys_launches):
    """Measured HBM bytes per launch, averaged over the given launches
    ({(kernel, shape) key: launches}), from the committed counter summary of
    the same sources; None if it is missing, stale, or lacks a key."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{dtype}.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    if d.get("source_hash") != source_hash():
        return None
    per = d.get("per_step", {})
    tot, n = 0.0, 0
    for key, cnt in keys_launches.items():
        if key not in per:
            return None
        tot += cnt * (per[key]["fetch_bytes"] + per[key]["write_bytes"])
        n += cnt
    return tot / n if n else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rqc53")
    ap.add_argument("--dtype", default="chalf")
    ap.add_argument("--compare", default="c64", help="second dtype timed on the same slices")
    ap.add_argument("--slices-per-step", type=int, default=16)
    ap.add_argument("--launch", default="stream")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=45.0)
    ap.add_argument("--keep-batch-order", action="store_true",
                    help="contract the closed strings in the given order (no sort by gathered bits)")
    ap.add_argument("--dump-steps", default="", help="write per-step shapes and times (json)")
    ap.add_argument("--autotune-cache", default=None,
                    help="kernel choices to load (default: the committed MI355X choices)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="paper53: use the shape rule instead of timing kernel variants")
    ap.add_argument("--retune", action="store_true",
                    help="load no kernel choices: time every variant on this machine")
    ap.add_argument("--save-autotune", default="", help="write the kernel choices here")
    ap.add_argument("--trace", action="store_true",
                    help="timed steps only (for an external profiler): no per-step timing, "
                         "no second arithmetic, no CPU baseline")
    ap.add_argument("--dump-launches", default="",
                    help="with --trace: write the contraction launches of one slice (json)")
    ap.add_argument("--summarize-pmc", nargs="+", default=None, metavar="CSV",
                    help="summarize rocprofv3 counter CSVs of a --trace run per (kernel, step "
                         "shape) using --launches; no GPU work")
    ap.add_argument("--launches", default="", help="launch list written by --dump-launches")
    ap.add_argument("--copy-pmc", nargs="*", default=[],
                    help="counter CSVs of a plain 1 GiB device copy (FETCH_SIZE/WRITE_SIZE scale)")
    ap.add_argument("--summary-out", default="", help="--summarize-pmc: write json here")
    ap.add_argument("--summarize-trace", default="", metavar="CSV",
                    help="rocprofv3 kernel trace: time per kernel over the last whole slice (between the last "
                         "two accumulate launches) and the share of the traced time with 1, 2, ... kernels "
                         "in flight")
    return ap.parse_args()


def cpu_baseline(plan, circ, openq, cb, seconds):
    """The oracle's complex128 contraction of slice 0 for one closed string,
    along the plan's tree (the oracle handles one string at a time at this
    size; each string is a sub-network of the same cost).  It runs the whole
    sub-network when the first steps' rate says it fits in `seconds`, else
    stops there and extrapolates by multiply-adds (then marked an estimate).
    One slice of the workload is that work for every closed string."""
    import numpy as np
    from oracle import tn

    leaf_canon, steps, base = plan.tree()
    wires = plan.sliced_wires()
    leaves = tn.canonical_network(circ, openq, cb[:1])
    if wires:
        leaves = tn.fix_wires(leaves, wires, tn.slice_values(0, len(wires)))
    keep = tn._keep_labels(openq)
    # dry run over shapes: the oracle's own multiply-adds per step
    shapes = {k: dict(zip(l, d.shape)) for k, (l, d) in leaves.items()}
    work = []
    for i, (a, b) in enumerate(steps):
        da, db = shapes.pop(a), shapes.pop(b)
        u = dict(da)
        u.update(db)
        work.append(float(np.prod(list(u.values()), dtype=np.float64)))
        shapes[base + i] = {x: v for x, v in u.items() if not (x in da and x in db) or x in keep}
    total = sum(work)
    nodes = dict(leaves)
    done, n_done = 0.0, 0
    t_start = time.time()
    for i, (a, b) in enumerate(steps):
        el = time.time() - t_start
        if n_done > 0 and el > 0.5:
            rate = done / el
            if el + (total - done) / rate > seconds and el + work[i] / rate > seconds / 2:
                break
        la, A = nodes.pop(a)
        lb, B = nodes.pop(b)
        nodes[base + i] = tn.contract_pair(la, A, lb, B, keep)
        done += work[i]
        n_done += 1
    el = time.time() - t_start
    whole = n_done == len(steps)
    est_slice = el * total / done
    if whole:
        sample = (f"complex128 numpy contraction of the whole slice-0 sub-network of 1 of {len(cb)} "
                  f"closed strings along the plan's tree ({len(steps)} steps) in {el:.1f} s, "
                  f"times {len(cb)} strings")
    else:
        sample = (f"estimate: complex128 numpy contraction of slice 0 for 1 of {len(cb)} closed "
                  f"strings along the plan's tree stopped after {n_done}/{len(steps)} steps = "
                  f"{done / total:.3g} of its multiply-adds in {el:.1f} s; slice time extrapolated "
                  f"by multiply-adds and multiplied by {len(cb)} strings")
    return {"value": 1.0 / (est_slice * len(cb)), "unit": "slices/s",
            "cores": len(os.sched_getaffinity(0)), "kind": "oracle", "sample": sample,
            "measured_whole_subnetwork": whole}


def run_mix(args):
    """The batched uneven workload: 512 sliced subtasks (one slice each) of
    8 seeded circuits (30..53 qubits, 12..20 cycles, caps 2^24..2^27), all
    contracted per step by one recorded graph per lane (4 lanes of plan
    chains on parallel streams), then the per-circuit top-1 post-selection.
    Also times the same items launched one slice after another on one
    stream (no graph) and the other arithmetic."""
    import numpy as np
    import torch

    import paper_2406_18889_amd as lf
    import workloads as wl

    circuits, subtasks = wl.mixed_workload()
    t_start = time.time()

    def say(msg):
        print(f"[mix512 {time.time() - t_start:6.1f}s] {msg}", file=sys.stderr, flush=True)

    def plans_for(dtype):
        ps = [lf.Plan(c["circuit"], c["open_qubits"], c["closed_bits"], max_log2=c["max_log2"],
                      dtype=dtype, search_dtype="chalf", check_overflow=False).bind()
              for c in circuits]
        say(f"{dtype}: {len(ps)} plans bound")
        # calibration and kernel tuning of each plan, on scratch accumulators
        for k, p in enumerate(ps):
            p.contract(0, 1, p.new_amplitudes())
            torch.cuda.synchronize()
            say(f"{dtype}: plan {k} ready ({p.info()['n_steps']} steps)")
        outs = [p.new_amplitudes() for p in ps]
        items = []
        for (k, draw) in subtasks:
            s0 = draw % ps[k].info()["n_slices"]
            items.append((ps[k], s0, s0 + 1, outs[k]))
        return ps, outs, items

    def timed(items, outs, mode, steps, warmup, lanes=0):
        def one():
            lf.contract_batch(items, mode, lanes=lanes)
            for o, c in zip(outs, circuits):
                lf.postselect_topk(o, 1 << len(c["open_qubits"]), 1)
        for i in range(warmup):
            one()
            torch.cuda.synchronize()
            say(f"{mode}: warm-up step {i} done")
        t0 = time.perf_counter()
        for _ in range(steps):
            one()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        say(f"{mode}: {steps} timed steps, {dt * 1e3:.1f} ms per step")
        return dt

    ps, outs, items = plans_for(args.dtype)
    macs = sum(ps[k].info()["macs_per_slice"] for (k, _) in subtasks)
    dt = timed(items, outs, "graph", args.steps, max(1, args.warmup))
    dt_seq = timed(items, outs, "sequential", max(1, min(args.steps, 3)), 1)
    value = len(items) / dt
    out = {
        "metric": "sliced-subtask contractions/s",
        "value": value, "unit": "subtasks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": max(1, args.warmup), "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "chalf" if args.dtype == "chalf" else "c64", "data": "synthetic",
        "config": {"workload": "mix512", "subtasks": len(items), "circuits": len(circuits),
                   "grids": [list(c["grid"]) for c in circuits],
                   "cycles": [c["cycles"] for c in circuits],
                   "caps_log2": [c["max_log2"] for c in circuits]},
        "algorithmic_tflops": 8.0 * macs / dt / 1e12,
        "mfma_frac_algorithmic": 8.0 * macs / dt / 1e12 /
                                  (MI355X["fp16_tflops"] if args.dtype == "chalf" else MI355X["fp32_tflops"]),
        "lanes": min(4, len(circuits)),
        "sequential": {"value": len(items) / dt_seq, "unit": "subtasks/s",
                       "graph_speedup": dt_seq / dt},
    }
    if args.compare and args.compare not in ("none", args.dtype):
        for o in outs:
            o.zero_()
        lf.contract_batch(items, "graph")
        torch.cuda.synchronize()
        a = [o.cpu().numpy() for o in outs]
        del ps, outs, items
        torch.cuda.empty_cache()
        ps2, outs2, items2 = plans_for(args.compare)
        dt2 = timed(items2, outs2, "graph", 1, 1)
        for o in outs2:
            o.zero_()
        lf.contract_batch(items2, "graph")
        torch.cuda.synchronize()
        say("agreement pass done")
        x = np.concatenate([v.reshape(-1) for v in a])
        y = np.concatenate([o.cpu().numpy().reshape(-1) for o in outs2])
        rel = float(np.linalg.norm(x - y) / np.linalg.norm(y))
        fid = float(abs(np.vdot(y, x)) ** 2 / (np.vdot(x, x).real * np.vdot(y, y).real))
        out["compare"] = {"dtype": args.compare, "value": len(items2) / dt2, "unit": "subtasks/s",
                          "speedup": dt2 / dt, "rel_err_vs_compare": rel, "fidelity_vs_compare": fid}
    print(json.dumps(out))


def run_xeb(args):
    """The 30-qubit cross-entropy study (Methods B, Fig. 3 and Fig. 4): all
    30 qubits open, prefixes D = 1..5 of the 2^8 slices, top-2^15 over 2^30
    strings and Metropolis samples at each prefix, then the exact amplitudes;
    XEB of the selections and samples with the exact q, next to Eq. 4 and
    the oracle's fidelities of the prefixes."""
    import torch
    from paper_2406_18889_amd import xeb

    torch.cuda.set_device(0)
    t_start = time.time()

    def say(msg):
        print(f"[xeb30 {time.time() - t_start:6.1f}s] {msg}", file=sys.stderr, flush=True)

    res = xeb.run(say=say, dtype=args.dtype if args.dtype in ("c64", "chalf") else "c64")
    fid = {}
    try:
        with open(os.path.join(ROOT, "tests", "golden", "rqc30_prefix.json")) as f:
            fj = json.load(f)
        fid = {D: fj[f"fidelity_D{D}"] for D in range(1, 6)}
    except (OSError, KeyError):
        pass
    N = 1 << res["n_qubits"]
    out = {"workload": "xeb30", "dtype": args.dtype, "data": "synthetic",
           "contract_s": res["contract_s"], "select_s": res["select_s"], "seconds": res["seconds"],
           "slices": res["n_slices"], "macs_per_slice": res["macs_per_slice"],
           "k_values": res["k_values"], "mcmc_samples": res["mcmc_samples"],
           "mcmc_candidates": res["mcmc_candidates"], "per_D": {}}
    for D in range(1, 6):
        r = {"xeb_topk": res[f"xeb_topk_D{D}"], "xeb_mcmc": res[f"xeb_mcmc_D{D}"],
             "mcmc_acceptance": res[f"mcmc_acceptance_D{D}"]}
        if D in fid:
            r["fidelity_oracle"] = fid[D]
            r["eq4"] = [xeb.eq4(fid[D], N, k) for k in res["k_values"]]
            r["topk_amplification"] = res[f"xeb_topk_D{D}"][-1] / fid[D]
        out["per_D"][D] = r
    print(json.dumps(out))


PAPER_STRINGS = 3_000_000
PAPER_PLAN = dict(max_log2=32, sa_iters=4_000_000, restarts=8, search_dtype="chalf")


def run_paper(args):
    """One GPU at the output scale of the paper's run (Methods D): the
    53-qubit, 20-cycle circuit with l = 10 open qubits and 3 million sampled
    closed strings, so every slice yields |S~| = 3e6 x 2^10 amplitudes into
    one float64 accumulator (3.07e9 complex128, 49 GB); then the global top
    3e6 over all of S~ (Methods A) and the top-1 of every group.  The cap is
    2^32 elements per tensor (16 GiB in complex-half).  A step is one slice;
    the selections are timed separately (they run once per job, not per
    slice)."""
    import numpy as np
    import torch

    import paper_2406_18889_amd as lf
    import workloads as wl

    torch.cuda.set_device(0)
    t_start = time.time()

    def say(msg):
        print(f"[paper53 {time.time() - t_start:6.1f}s] {msg}", file=sys.stderr, flush=True)

    tune = None if args.retune else (args.autotune_cache or TUNE_FILE)
    if tune and os.path.exists(tune):
        lf.autotune_load(tune)
    circ, openq, cb, spec = wl.standard_workload("rqc53")
    closed = wl.closed_bitstrings(circ.n_qubits, openq, PAPER_STRINGS, seed=wl.BITSTRING_SEED)
    say(f"{closed.size} closed strings drawn")
    plan = lf.Plan(circ, openq, closed, dtype=args.dtype, launch=args.launch, check_overflow=False,
                   autotune=not args.no_autotune, keep_batch_order=args.keep_batch_order, **PAPER_PLAN)
    info = plan.info()
    say(f"plan: 2^{info['n_sliced_wires']} slices of {info['macs_per_slice']:.3e} multiply-adds, "
        f"workspace {info['workspace_bytes'] / 2**30:.1f} GiB, batch padded to 2^{info['n_batch_log2']}")
    plan.bind()
    amps = plan.new_amplitudes()
    say(f"workspace bound, accumulator {amps.numel() * 16 / 1e9:.1f} GB")
    t0 = time.time()
    plan.contract(0, 1, amps)
    torch.cuda.synchronize()
    t_first = time.time() - t0
    say(f"slice 0 (calibration, kernel choice) {t_first:.1f} s")
    for i in range(args.warmup):
        plan.contract(1 + i, 2 + i, amps)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i].record()
        s0 = 1 + args.warmup + i
        plan.contract(s0, s0 + 1, amps)
    evs[-1].record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    step_ms = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    say(f"{args.steps} timed slices, {dt / args.steps * 1e3:.1f} ms each")
    ov = plan.overflow()
    n_amp = amps.numel()
    k = PAPER_STRINGS
    t1 = time.perf_counter()
    idx, prob = lf.postselect_topk(amps, n_amp, k)
    torch.cuda.synchronize()
    t_top = time.perf_counter() - t1
    t1 = time.perf_counter()
    g1, p1 = lf.postselect_topk(amps, 1 << len(openq), 1)
    torch.cuda.synchronize()
    t_top1 = time.perf_counter() - t1
    say(f"global top-{k} of {n_amp} in {t_top * 1e3:.1f} ms, per-group top-1 in {t_top1 * 1e3:.1f} ms")
    if args.save_autotune:
        lf.autotune_save(args.save_autotune)
    value = args.steps / dt
    flops = 8.0 * info["macs_per_slice"]
    out = {"metric": "sliced-subtask contractions/s", "value": value, "unit": "slices/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "chalf" if args.dtype == "chalf" else "c64", "data": "synthetic",
           "config": {"workload": "paper53", "qubits": circ.n_qubits, "cycles": spec["cycles"],
                      "open_qubits": len(openq), "closed_strings": PAPER_STRINGS,
                      "amplitudes_per_slice": n_amp, "max_log2_intermediate": info["max_log2_intermediate"],
                      "slices_total_log2": info["n_sliced_wires"],
                      "batch_order": "given" if args.keep_batch_order else "sorted by gathered bits"},
           "macs_per_slice": info["macs_per_slice"],
           "algorithmic_tflops": value * flops / 1e12,
           "mfma_frac_algorithmic": value * flops / 1e12 /
                                     (MI355X["fp16_tflops"] if args.dtype == "chalf" else MI355X["fp32_tflops"]),
           "step_ms": {"median": float(np.median(step_ms)), "p10": float(np.percentile(step_ms, 10)),
                       "p90": float(np.percentile(step_ms, 90))},
           "first_slice_s": t_first,
           "accumulator_gb": n_amp * 16 / 1e9, "workspace_gib": info["workspace_bytes"] / 2 ** 30,
           "topk_global": {"k": k, "candidates": n_amp, "ms": t_top * 1e3},
           "top1_per_group": {"groups": PAPER_STRINGS, "ms": t_top1 * 1e3},
           "saturation": {"saturated_values": ov["saturated"], "first_bad_slice": ov["first_bad_slice"]},
           "device": device_record()}
    print(json.dumps(out))


def device_record():
    """Device name, architecture, clocks and software versions."""
    import ctypes
    import torch
    prop = torch.cuda.get_device_properties(0)
    rec = {"device": torch.cuda.get_device_name(0), "arch": getattr(prop, "gcnArchName", ""),
           "compute_units": prop.multi_processor_count,
           "hbm_gib": round(prop.total_memory / 2 ** 30, 1),
           "hip_torch": torch.version.hip, "torch": torch.__version__}
    try:
        hip = ctypes.CDLL("libamdhip64.so")
        v = ctypes.c_int()
        if hip.hipRuntimeGetVersion(ctypes.byref(v)) == 0:
            rec["hip_runtime"] = v.value
        # hipDeviceAttributeClockRate (peak shader clock, kHz)
        if hip.hipDeviceGetAttribute(ctypes.byref(v), 5, 0) == 0 and v.value > 0:
            rec["peak_sclk_mhz"] = v.value / 1000.0
    except OSError:
        pass
    try:
        with open("/opt/rocm/.info/version") as f:
            rec["rocm"] = f.read().strip()
    except OSError:
        pass
    return rec


def plan_roofline(dims, macs, byts, sel_steps, slice_ms):
    """Sum over the slice-dependent steps of max(flop / MFMA peak of the
    step's arithmetic, bytes / HBM bandwidth), against the measured time of a
    slice; and the share of flops in steps above the ridge point."""
    import numpy as np
    half = dims[:, 5] == 1
    peak = np.where(half, MI355X["fp16_tflops"], MI355X["fp32_tflops"]) * 1e12
    t_mfma = 8.0 * macs / peak
    t_hbm = byts / (MI355X["hbm_gbs"] * 1e9)
    t_roof = np.maximum(t_mfma, t_hbm)
    m = sel_steps
    mfma_bound = m & (t_mfma >= t_hbm)
    return {"t_roof_ms_per_slice": float(t_roof[m].sum() * 1e3),
            "t_ms_per_slice": slice_ms,
            "frac": float(t_roof[m].sum() * 1e3 / slice_ms),
            "mfma_bound_steps": int(mfma_bound.sum()), "hbm_bound_steps": int((m & ~mfma_bound).sum()),
            "t_roof_ms_mfma_bound": float(t_roof[mfma_bound].sum() * 1e3),
            "t_roof_ms_hbm_bound": float(t_roof[m & ~mfma_bound].sum() * 1e3),
            "mfma_bound_flop_share": float(macs[mfma_bound].sum() / max(1.0, macs[m].sum()))}


def summarize_pmc(args):
    """Per (kernel, step shape) averages of rocprofv3 counters over the timed
    launches of a --trace run: the last steps * slices-per-step slices each
    launch the slice-dependent steps once, in the order of --launches."""
    import csv
    from collections import defaultdict

    with open(args.launches) as f:
        lj = json.load(f)
    seq = lj["launches"]                     # one slice: [{step, kernel, name, dims}]
    n_timed = lj["timed_slices"]

    def load(paths):
        disp = defaultdict(dict)
        for path in paths:
            with open(path) as f:
                for row in csv.DictReader(f):
                    d = disp[int(row["Dispatch_Id"])]
                    d["name"] = row["Kernel_Name"]
                    if "Counter_Name" in row:
                        c = row["Counter_Name"]
                        d[c] = d.get(c, 0.0) + float(row["Counter_Value"])
                    for k in ("Start_Timestamp", "End_Timestamp"):
                        if k in row and row[k]:
                            d[k] = int(row[k])
        return [disp[k] for k in sorted(disp)]

    def scale(paths):
        # a plain device copy of 1 GiB reads and writes 1 GiB
        if not paths:
            return {}
        ds = load(paths)
        big = [d for d in ds if d.get("FETCH_SIZE", 0) > 1e5 or d.get("WRITE_SIZE", 0) > 1e5]
        f = {}
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            v = [d[c] for d in big if c in d]
            if v:
                f[c] = (1 << 30) / (1024.0 * (sum(v) / len(v)))
        return f

    fac = scale(args.copy_pmc)
    ds = [d for d in load(args.summarize_pmc) if "gett_" in d["name"]]

    def same_kernel(base, name):
        at = name.find(base)
        return at >= 0 and not name[at + len(base):at + len(base) + 1] == "_"

    need = n_timed * len(seq)
    if len(ds) < need:
        raise SystemExit(f"{len(ds)} contraction dispatches, expected at least {need}")
    ds = ds[len(ds) - need:]
    acc = defaultdict(lambda: defaultdict(float))
    for i, d in enumerate(ds):
        l = seq[i % len(seq)]
        if not same_kernel(l["name"].split("<")[0], d["name"]):
            raise SystemExit(f"dispatch {i}: {d['name'][:60]} does not match step {l['step']} ({l['name']})")
        key = shape_key(l["name"], l["dims"])
        a = acc[key]
        a["dispatches"] += 1
        for c, v in d.items():
            if isinstance(v, float):
                a[c] += v
        if "Start_Timestamp" in d and "End_Timestamp" in d:
            a["ns"] += d["End_Timestamp"] - d["Start_Timestamp"]
    per = {}
    for key, a in acc.items():
        n = a["dispatches"]
        e = {"dispatches": int(n)}
        for c, v in a.items():
            if c == "dispatches":
                continue
            e[c] = v / n
        if "FETCH_SIZE" in e:
            e["fetch_bytes"] = e["FETCH_SIZE"] * 1024.0 * fac.get("FETCH_SIZE", 1.0)
        if "WRITE_SIZE" in e:
            e["write_bytes"] = e["WRITE_SIZE"] * 1024.0 * fac.get("WRITE_SIZE", 1.0)
        per[key] = e
    out = {"workload": lj["workload"], "dtype": lj["dtype"], "source_hash": lj["source_hash"],
           "copy_factors": fac, "timed_slices": n_timed, "per_step": per}
    if args.summary_out:
        with open(args.summary_out, "w") as f:
            json.dump(out, f, indent=1)
    print(json.dumps(out))


def summarize_trace(args):
    """Per-kernel time of the last whole slice of a rocprofv3 kernel trace
    (the dispatches after the second-to-last accumulate launch, up to and
    including the last), its longest dispatches, and how much of the traced
    span had 1, 2, ... kernels executing at once (concurrent lanes)."""
    import csv
    from collections import defaultdict
    with open(args.summarize_trace) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Start_Timestamp"]))
    dur = lambda r: (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
    short = lambda r: r["Kernel_Name"].split("(")[0][:90]
    out = {"dispatches": len(rows)}
    acc = [i for i, r in enumerate(rows) if "accumulate_kernel" in r["Kernel_Name"]]
    if len(acc) >= 2:
        seg = rows[acc[-2] + 1:acc[-1] + 1]
        per = defaultdict(lambda: [0, 0.0])
        for r in seg:
            per[short(r)][0] += 1
            per[short(r)][1] += dur(r)
        out["slice"] = {"kernels": len(seg), "kernel_ms": sum(dur(r) for r in seg),
                        "span_ms": (int(seg[-1]["End_Timestamp"]) - int(rows[acc[-2]]["End_Timestamp"])) / 1e6,
                        "by_kernel": sorted(([k, v[0], v[1]] for k, v in per.items()), key=lambda x: -x[2]),
                        "longest": [[short(r), dur(r), int(r["Grid_Size_X"])]
                                    for r in sorted(seg, key=lambda r: -dur(r))[:8]]}
    ev = []
    for r in rows:
        ev.append((int(r["Start_Timestamp"]), 1))
        ev.append((int(r["End_Timestamp"]), -1))
    ev.sort()
    busy = defaultdict(float)
    cur, last = 0, ev[0][0] if ev else 0
    for t, d in ev:
        if cur > 0:
            busy[cur] += (t - last) / 1e6
        cur += d
        last = t
    out["ms_with_k_kernels_in_flight"] = {str(k): v for k, v in sorted(busy.items())}
    print(json.dumps(out))


def main():
    args = parse()
    if args.summarize_pmc:
        return summarize_pmc(args)
    if args.summarize_trace:
        return summarize_trace(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "mix512":
        return run_mix(args)
    if args.workload == "xeb30":
        return run_xeb(args)
    if args.workload == "paper53":
        return run_paper(args)
    import numpy as np
    import torch

    import paper_2406_18889_amd as lf
    import workloads as wl

    torch.cuda.set_device(0)
    tune = None if args.retune else (args.autotune_cache or TUNE_FILE)
    if tune and os.path.exists(tune):
        lf.autotune_load(tune)
    circ, openq, cb, spec = wl.standard_workload(args.workload)
    kw = dict(PLAN_OPTS.get(args.workload, {}))
    if args.workload == "rqc30":
        kw["sliced_wires"] = wl.RQC30_SLICED_WIRES
    # both arithmetics search with the complex-half step costs, so they share
    # one tree and one slicing (slice s is the same sub-network in both)
    kw["search_dtype"] = "chalf"
    kw["keep_batch_order"] = args.keep_batch_order
    # a traced run maps dispatches to steps by launch order: one launch per step
    kw["group_small_steps"] = not args.trace
    plan = lf.Plan(circ, openq, cb, dtype=args.dtype, max_log2=spec["max_log2"],
                   launch=args.launch, check_overflow=False, **kw)
    info = plan.info()
    plan.bind()
    n_slices = info["n_slices"]
    S = min(args.slices_per_step, n_slices)
    amps = plan.new_amplitudes()

    # calibrate / invariant part outside the timed region
    plan.contract(0, 1, amps)
    torch.cuda.synchronize()

    def step(i):
        s0 = (i * S) % n_slices
        s1 = min(s0 + S, n_slices)
        plan.contract(s0, s1, amps)
        lf.postselect_topk(amps, 1 << len(openq), 1)
        return s1 - s0

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    dims, macs, byts = plan.steps()
    var = dims[:, 4] == 1
    if not args.trace:
        # isolated per-step timing (outside the timed region) picks the
        # dominant kernel: the variant with the largest total time per slice
        ms = plan.profile_steps(reps=3)
        kinds = sorted(set(int(k) for k in dims[var, 7]))
        tot = {k: float(ms[var & (dims[:, 7] == k)].sum()) for k in kinds}
        dom_k = max(tot, key=tot.get)
        sel = var & (dims[:, 7] == dom_k)
        # its launches in the timed region are bracketed by HIP events on the
        # plan's launch stream
        plan.time_kernel(dom_k, reserve=int(sel.sum()) * S * args.steps)
        plan.kernel_times()
    # every timed step bracketed by events on the launch stream as well
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    done = 0
    for i in range(args.steps):
        evs[i].record()
        done += step(args.warmup + i)
    evs[-1].record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = done / dt
    step_ms = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    ov = plan.overflow()
    launches = [{"step": int(s), "kernel": int(dims[s, 7]), "name": KERNEL_NAMES.get(int(dims[s, 7]), "?"),
                 "dims": [int(x) for x in dims[s, :4]]} for s in np.nonzero(var)[0]]
    if args.trace:
        if args.save_autotune:
            lf.autotune_save(args.save_autotune)
        if args.dump_launches:
            with open(args.dump_launches, "w") as f:
                json.dump({"workload": args.workload, "dtype": args.dtype, "source_hash": source_hash(),
                           "timed_slices": done, "launches": launches}, f)
        print(json.dumps({"trace": True, "value": value, "unit": "slices/s", "steps": args.steps,
                          "slices_per_step": S, "workload": args.workload, "dtype": args.dtype,
                          "saturated": ov["saturated"], "source_hash": source_hash()}))
        return

    # the dominant kernel over its launches in the timed region: algorithmic
    # flops (8 per complex multiply-add) and bytes of the launched steps over
    # their summed event-timed durations
    tot_ms, n_launch, per_ms, per_n = plan.kernel_times()
    plan.time_kernel(-1)
    timing = "HIP events around its launches in the timed steps"
    if n_launch == 0:
        # graph launches are not bracketed by events: use the isolated
        # per-step timing of the same launches (one slice's worth)
        per_n = sel.astype(np.int64)
        per_ms = np.where(sel, ms, 0.0)
        tot_ms, n_launch = float(per_ms.sum()), int(sel.sum())
        timing = "isolated per-step HIP-event timing (graph launches carry no events)"
    t = tot_ms * 1e-3
    flops = 8.0 * float((macs * per_n).sum())
    bytes_ = float((byts * per_n).sum())
    half = bool((dims[sel, 5] == 1).all())
    peak_tf = MI355X["fp16_tflops"] if half else MI355X["fp32_tflops"]
    ridge = peak_tf * 1e12 / (MI355X["hbm_gbs"] * 1e9)
    if flops / bytes_ >= ridge:
        roof = {"bound": "mfma", "achieved": flops / t / 1e12, "peak": peak_tf, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": bytes_ / t / 1e9, "peak": MI355X["hbm_gbs"], "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    dom_name = KERNEL_NAMES.get(dom_k, "?")
    keys = {}
    for s_ in np.nonzero(per_n)[0]:
        k_ = shape_key(dom_name, dims[s_])
        keys[k_] = keys.get(k_, 0) + int(per_n[s_])
    roof["traffic"] = traffic_for(args.workload, args.dtype, keys)
    roof["kernel"] = {"name": dom_name, "timing": timing,
                      "launches_per_slice": int(sel.sum()),
                      "timed_launches": int(n_launch),
                      "avg_launch_ms": tot_ms / max(1, n_launch),
                      "algorithmic_flop_per_launch": flops / max(1, n_launch),
                      "algorithmic_bytes_per_launch": bytes_ / max(1, n_launch),
                      "share_of_slice_time": tot_ms / max(1, n_launch) * int(sel.sum()) /
                                             (dt / done * 1e3),
                      "launches_by_shape": keys}
    # isolated per-step timings (3 repetitions each), summed per kernel
    roof["isolated_ms_per_slice_by_kernel"] = {KERNEL_NAMES.get(k, "?"): v for k, v in tot.items()}
    if args.dump_steps:
        with open(args.dump_steps, "w") as f:
            json.dump({"dims": dims.tolist(), "macs": macs.tolist(), "bytes": byts.tolist(),
                       "ms": [float(x) for x in ms]}, f)
    per_slice_flops = 8.0 * info["macs_per_slice"]
    choice = {}
    for l in launches:
        choice[l["name"]] = choice.get(l["name"], 0) + 1
    import hashlib
    out = {
        "metric": "sliced-subtask contractions/s",
        "value": value,
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "chalf" if args.dtype == "chalf" else "c64",
        "data": "synthetic",
        "config": {"workload": args.workload, "qubits": circ.n_qubits, "cycles": spec["cycles"],
                   "open_qubits": len(openq), "closed_strings": len(cb),
                   "slices_total": n_slices, "slices_per_step": S,
                   "max_log2_intermediate": info["max_log2_intermediate"],
                   "batch_order": "given" if args.keep_batch_order else "sorted by gathered bits"},
        "algorithmic_tflops": value * per_slice_flops / 1e12,
        "mfma_frac_algorithmic": value * per_slice_flops / 1e12 /
                                  (MI355X["fp16_tflops"] if args.dtype == "chalf" else MI355X["fp32_tflops"]),
        "macs_per_slice": info["macs_per_slice"],
        "step_ms": {"median": float(np.median(step_ms)), "p10": float(np.percentile(step_ms, 10)),
                    "p90": float(np.percentile(step_ms, 90)),
                    "timing": "HIP events on the launch stream around each timed step"},
        "roofline": roof,
        "plan_roofline": plan_roofline(dims, macs, byts, var, dt / done * 1e3),
        "kernel_choice": {"file": os.path.relpath(tune, ROOT) if tune and os.path.exists(tune) else None,
                          "hash": hashlib.sha256(json.dumps(launches).encode()).hexdigest()[:16],
                          "launches_per_slice": choice},
        "saturation": {"saturated_values": ov["saturated"], "first_bad_slice": ov["first_bad_slice"],
                       "checked": "after the timed region, over every slice since calibration"},
        "device": device_record(),
    }
    if args.compare and args.compare not in ("none", args.dtype):
        # the other arithmetic on the same slices: throughput and agreement
        other = lf.Plan(circ, openq, cb, dtype=args.compare, max_log2=spec["max_log2"],
                        launch=args.launch, check_overflow=False, **kw)
        if other.sliced_wires() != plan.sliced_wires():
            raise RuntimeError("the two arithmetics planned different slicings")
        other.bind()
        ref = other.new_amplitudes()
        other.contract(0, 1, ref)
        torch.cuda.synchronize()
        n_cmp = max(1, min(args.steps, 4))
        t1 = time.perf_counter()
        done_o = 0
        for i in range(n_cmp):
            s0 = ((args.warmup + i) * S) % n_slices
            s1 = min(s0 + S, n_slices)
            other.contract(s0, s1, ref)
            done_o += s1 - s0
        torch.cuda.synchronize()
        v_other = done_o / (time.perf_counter() - t1)
        # agreement over slices [0, S): both dtypes, fresh accumulators
        a1 = plan.new_amplitudes()
        plan.contract(0, S, a1)
        a2 = other.new_amplitudes()
        other.contract(0, S, a2)
        torch.cuda.synchronize()
        x, y = a1.cpu().numpy().reshape(-1), a2.cpu().numpy().reshape(-1)
        rel = float(np.linalg.norm(x - y) / np.linalg.norm(y))
        fid = float(abs(np.vdot(y, x)) ** 2 / (np.vdot(x, x).real * np.vdot(y, y).real))
        out["compare"] = {"dtype": args.compare, "value": v_other, "unit": "slices/s",
                          "speedup": value / v_other,
                          "agreement_slices": [0, S], "rel_err_vs_compare": rel,
                          "fidelity_vs_compare": fid}
        del other
    if args.workload == "rqc30":
        # time to the exact amplitudes (all slices) against the oracle's state
        # vector run that wrote the stored exact values
        try:
            with open(os.path.join(ROOT, "tests", "golden", "rqc30_stats.json")) as f:
                st = json.load(f)
            out["time_to_exact"] = {"gpu_s": n_slices / value, "oracle_state_vector_s": st["sv_seconds"],
                                    "oracle_threads": st["threads"],
                                    "note": "oracle time from the run that wrote the stored values"}
        except (OSError, KeyError):
            pass
    if args.save_autotune:
        lf.autotune_save(args.save_autotune)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(plan, circ, openq, cb, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
