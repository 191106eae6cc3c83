"""Benchmark: sliced-subtask contractions per second on one MI355X.

A step contracts one chunk of slices of the workload into a float64
amplitude accumulator and runs the top-k post-selection on it (the whole hot
path).  Inputs (plan, leaves, workspace) are resident in HBM before timing.
Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rqc30|rqc53|mix512]
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
                13: "gett_mfma_dma<0,4>", 14: "gett_mfma_dma<1,4>"}
# planner settings per workload (search effort, not inputs)
PLAN_OPTS = {"rqc53": {"sa_iters": 4_000_000, "restarts": 8}}


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "runtime.hip"):
        with open(os.path.join(ROOT, "paper_2406_18889_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(workload, dtype, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken with the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{dtype}.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None
    if d.get("source_hash") != source_hash():
        return None
    return d.get("bytes_per_launch", {}).get(kernel)


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
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--dump-steps", default="", help="write per-step shapes and times (json)")
    ap.add_argument("--autotune-cache", default="", help="load/save the kernel choices here")
    ap.add_argument("--trace", action="store_true",
                    help="timed steps only (for an external profiler): no per-step timing, "
                         "no second arithmetic, no CPU baseline")
    return ap.parse_args()


def cpu_baseline(plan, circ, openq, cb, seconds):
    """The oracle's complex128 contraction of slice 0 for one closed string,
    along the plan's tree, run for about `seconds` of host time.  Its
    multiply-add rate extrapolates to the whole slice; one slice of the
    workload is that work for every closed string (the oracle handles one
    string at a time at this size)."""
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
            if el + work[i] / rate > seconds:
                break
        la, A = nodes.pop(a)
        lb, B = nodes.pop(b)
        nodes[base + i] = tn.contract_pair(la, A, lb, B, keep)
        done += work[i]
        n_done += 1
    el = time.time() - t_start
    est_slice = el * total / done
    return {"value": 1.0 / (est_slice * len(cb)), "unit": "slices/s",
            "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
            "sample": f"complex128 numpy contraction of slice 0 for 1 of {len(cb)} closed strings "
                      f"along the plan's tree: {n_done}/{len(steps)} steps = {done / total:.3g} "
                      f"of its multiply-adds in {el:.1f} s; slice time extrapolated by "
                      f"multiply-adds and multiplied by {len(cb)} strings"}


def run_mix(args):
    """The batched uneven workload: 512 sliced subtasks (one slice each) of
    8 seeded circuits (30..53 qubits, 12..20 cycles, caps 2^24..2^27), all
    contracted by one recorded graph launch per step, then the per-circuit
    top-1 post-selection.  Also times the same items launched one slice
    after another (no graph) and the other arithmetic."""
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
        # one stream for the slower arithmetic (no lane tuning: a tuning pass
        # replays the whole batch six times)
        dt2 = timed(items2, outs2, "graph", 1, 1, lanes=1)
        for o in outs2:
            o.zero_()
        lf.contract_batch(items2, "graph", lanes=1)
        torch.cuda.synchronize()
        say("agreement pass done")
        x = np.concatenate([v.reshape(-1) for v in a])
        y = np.concatenate([o.cpu().numpy().reshape(-1) for o in outs2])
        rel = float(np.linalg.norm(x - y) / np.linalg.norm(y))
        fid = float(abs(np.vdot(y, x)) ** 2 / (np.vdot(x, x).real * np.vdot(y, y).real))
        out["compare"] = {"dtype": args.compare, "value": len(items2) / dt2, "unit": "subtasks/s",
                          "speedup": dt2 / dt, "rel_err_vs_compare": rel, "fidelity_vs_compare": fid}
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "mix512":
        return run_mix(args)
    import numpy as np
    import torch

    import paper_2406_18889_amd as lf
    import workloads as wl

    torch.cuda.set_device(0)
    if args.autotune_cache and os.path.exists(args.autotune_cache):
        lf.autotune_load(args.autotune_cache)
    circ, openq, cb, spec = wl.standard_workload(args.workload)
    kw = dict(PLAN_OPTS.get(args.workload, {}))
    if args.workload == "rqc30":
        from tests.golden.make_rqc30 import RQC30_SLICED_WIRES
        kw["sliced_wires"] = RQC30_SLICED_WIRES
    # both arithmetics search with the complex-half step costs, so they share
    # one tree and one slicing (slice s is the same sub-network in both)
    kw["search_dtype"] = "chalf"
    plan = lf.Plan(circ, openq, cb, dtype=args.dtype, max_log2=spec["max_log2"],
                   launch=args.launch, check_overflow=False, **kw)
    info = plan.info()
    plan.bind()
    n_slices = info["n_slices"]
    S = min(args.slices_per_step, n_slices)
    amps = plan.new_amplitudes()
    stream = torch.cuda.current_stream()

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
    if not args.trace:
        # isolated per-step timing (outside the timed region) picks the
        # dominant kernel: the variant with the largest total time per slice
        ms = plan.profile_steps(reps=3)
        dims, macs, byts = plan.steps()
        var = dims[:, 4] == 1
        kinds = sorted(set(int(k) for k in dims[var, 7]))
        tot = {k: float(ms[var & (dims[:, 7] == k)].sum()) for k in kinds}
        dom_k = max(tot, key=tot.get)
        sel = var & (dims[:, 7] == dom_k)
        # its launches in the timed region are bracketed by HIP events on the
        # plan's launch stream
        plan.time_kernel(dom_k, reserve=int(sel.sum()) * S * args.steps)
        plan.kernel_times()
    t0 = time.perf_counter()
    done = 0
    for i in range(args.steps):
        done += step(args.warmup + i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = done / dt
    if args.autotune_cache:
        lf.autotune_save(args.autotune_cache)
    if args.trace:
        print(json.dumps({"trace": True, "value": value, "unit": "slices/s", "steps": args.steps,
                          "slices_per_step": S, "workload": args.workload, "dtype": args.dtype,
                          "source_hash": source_hash()}))
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
    roof["traffic"] = traffic_for(args.workload, args.dtype, KERNEL_NAMES.get(dom_k, "?"))
    roof["kernel"] = {"name": KERNEL_NAMES.get(dom_k, "?"), "timing": timing,
                      "launches_per_slice": int(sel.sum()),
                      "timed_launches": int(n_launch),
                      "avg_launch_ms": tot_ms / max(1, n_launch),
                      "algorithmic_flop_per_launch": flops / max(1, n_launch),
                      "algorithmic_bytes_per_launch": bytes_ / max(1, n_launch),
                      "share_of_slice_time": tot_ms / max(1, n_launch) * int(sel.sum()) /
                                             (dt / done * 1e3)}
    # isolated per-step timings (3 repetitions each), summed per kernel
    roof["isolated_ms_per_slice_by_kernel"] = {KERNEL_NAMES.get(k, "?"): v for k, v in tot.items()}
    if args.dump_steps:
        with open(args.dump_steps, "w") as f:
            json.dump({"dims": dims.tolist(), "macs": macs.tolist(), "bytes": byts.tolist(),
                       "ms": [float(x) for x in ms]}, f)
    per_slice_flops = 8.0 * info["macs_per_slice"]
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
                   "max_log2_intermediate": info["max_log2_intermediate"]},
        "algorithmic_tflops": value * per_slice_flops / 1e12,
        "mfma_frac_algorithmic": value * per_slice_flops / 1e12 /
                                  (MI355X["fp16_tflops"] if args.dtype == "chalf" else MI355X["fp32_tflops"]),
        "macs_per_slice": info["macs_per_slice"],
        "roofline": roof,
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
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(plan, circ, openq, cb, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
