"""Stored expected values for single slices of the 53-qubit, 20-cycle
workload (6x9 grid minus one site, 10 open qubits, 256 closed strings,
2^28-element cap), on the plan the benchmark times.

No state vector exists at 53 qubits, so the oracle here is the complex128
contraction of one sliced sub-network (slicing identity, Methods C) for one
closed string at a time.  A slice is defined by its sliced wires and their
values; the contraction order only sets memory and time (the value of a
network does not depend on it), so the oracle follows the plan's tree to stay
within host memory.

  python -m tests.golden.make_rqc53 plan
      rqc53_plan.json: the sliced wires (bit order) and the contraction tree
      of the benchmark's plan, as exported by the library's planner (host
      code, no device).  This is the definition of "slice sigma", not an
      expected value.
  python -m tests.golden.make_rqc53 values
      rqc53_slices.npy: complex128 [n_cases][1024], case (sigma, b) of
      rqc53_plan.json's "cases", computed by the oracle only (oracle.tn),
      from the circuit, the closed strings and rqc53_plan.json.
"""

import hashlib
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

PLAN_JSON = os.path.join(HERE, "rqc53_plan.json")
VALUES_NPY = os.path.join(HERE, "rqc53_slices.npy")

# closed strings checked: first, last, and two in between
STRINGS = (0, 37, 128, 255)
# slices checked: the first four, and one far slice drawn once (seeded)
FIRST_SLICES = (0, 1, 2, 3)
FAR_SEED = 53


def tree_hash(wires, leaf_canon, steps, base):
    h = hashlib.sha256()
    h.update(json.dumps([list(map(int, w)) for w in wires]).encode())
    h.update(json.dumps([int(x) for x in leaf_canon]).encode())
    h.update(json.dumps([[int(a), int(b)] for a, b in steps]).encode())
    h.update(str(int(base)).encode())
    return h.hexdigest()[:16]


def cases_for(n_sliced):
    far = int(np.random.Generator(np.random.PCG64(FAR_SEED)).integers(0, 1 << n_sliced))
    out = [(s, b) for s in FIRST_SLICES for b in STRINGS]
    out.append((far, 200))
    return out


def plan():
    """Export the benchmark plan's slicing and tree (library planner, host)."""
    import bench
    import paper_2406_18889_amd as lf

    circ, openq, cb, spec = wl.standard_workload("rqc53")
    kw = dict(bench.PLAN_OPTS["rqc53"])
    t0 = time.time()
    p = lf.Plan(circ, openq, cb, dtype="chalf", max_log2=spec["max_log2"], search_dtype="chalf",
                **kw)
    wires = p.sliced_wires()
    leaf_canon, steps, base = p.tree()
    info = p.info()
    out = {"workload": "rqc53", "plan_opts": kw, "search_dtype": "chalf",
           "max_log2": spec["max_log2"], "n_sliced": len(wires),
           "sliced_wires": [list(w) for w in wires], "leaf_canon": list(leaf_canon),
           "steps": [list(s) for s in steps], "id_base": base,
           "macs_per_slice": info["macs_per_slice"],
           "tree_hash": tree_hash(wires, leaf_canon, steps, base),
           "cases": cases_for(len(wires)), "planning_seconds": time.time() - t0}
    with open(PLAN_JSON, "w") as f:
        json.dump(out, f)
    print(f"{len(wires)} sliced wires, {len(steps)} steps, hash {out['tree_hash']}")


def values():
    """Oracle contraction of every stored case along the stored tree."""
    from oracle import tn

    with open(PLAN_JSON) as f:
        pj = json.load(f)
    circ, openq, cb, spec = wl.standard_workload("rqc53")
    wires = [tuple(w) for w in pj["sliced_wires"]]
    steps = [tuple(s) for s in pj["steps"]]
    keep = tn._keep_labels(openq)
    res = np.zeros((len(pj["cases"]), 1 << len(openq)), np.complex128)
    for i, (sigma, b) in enumerate(pj["cases"]):
        t0 = time.time()
        leaves = tn.canonical_network(circ, openq, cb[b:b + 1])
        leaves = tn.fix_wires(leaves, wires, tn.slice_values(sigma, len(wires)))
        labels, data = tn.contract_tree(leaves, steps, pj["id_base"], keep)
        order = ([labels.index("b")] if "b" in labels else []) + \
            [labels.index(("o", int(q))) for q in reversed(list(openq))]
        res[i] = np.transpose(data, order).reshape(-1)
        del data, leaves
        print(f"case {i}: slice {sigma}, string {b}: |a|^2 sum {np.vdot(res[i], res[i]).real:.4e}"
              f" ({time.time() - t0:.1f} s)", flush=True)
        np.save(VALUES_NPY, res)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "values"
    if what == "plan":
        plan()
    elif what == "values":
        values()
    else:
        raise SystemExit("usage: make_rqc53 plan|values")
