"""Host-side checks of the C ABI (no GPU): the library loads and exports
every declared symbol, argument errors come back as status codes, and the
plan's exported tree and slicing are checked by the oracle's own contractor
(the value of a network does not depend on the contraction order, so the
oracle following the plan's tree must reproduce the state vector)."""

import ctypes
import os
import re

import numpy as np
import pytest

import workloads as wl
from oracle import sv, tn

pytestmark = pytest.mark.usefixtures("oracle_built")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2406_18889_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2406_18889_amd import build
        build.build()
    return _lib.load()


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:lf_status|void|const char\*)\s+(lf_\w+)\s*\(", txt, re.M))
    return names


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_python_binding_covers_header(lib):
    from paper_2406_18889_amd import _lib
    assert declared_symbols() <= set(_lib.SIGNATURES)


def test_argument_errors(lib):
    from paper_2406_18889_amd import _lib
    h = ctypes.c_void_p()
    opts = _lib.lf_plan_opts()
    lib.lf_plan_opts_default(ctypes.byref(opts))
    c = wl.random_circuit(2, 2, 2, seed=1)
    from paper_2406_18889_amd.api import _circuit_struct
    cs, keep = _circuit_struct(c)
    openq = (ctypes.c_int32 * 1)(7)  # out of range
    cb = np.zeros(1, np.uint64)
    st = lib.lf_build_network(ctypes.byref(cs), openq, 1,
                              cb.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), 1,
                              ctypes.byref(opts), ctypes.byref(h))
    assert st == _lib.LF_INVALID_ARGUMENT
    assert b"open qubit" in lib.lf_last_error()
    # contracting an unbound plan
    p = __import__("paper_2406_18889_amd").Plan(c, [0, 1, 2, 3], [0], max_log2=10)
    st = lib.lf_contract_slices(p._handle, 0, 1, ctypes.c_void_p(16), None)
    assert st == _lib.LF_NOT_BOUND
    # top-k argument range
    st = lib.lf_postselect_topk(ctypes.c_void_p(16), 1, 64, 65, ctypes.c_void_p(16),
                                ctypes.c_void_p(16), None)
    assert st == _lib.LF_INVALID_ARGUMENT
    # infeasible cap with a forced slicing set that cannot reach it
    with pytest.raises(Exception):
        __import__("paper_2406_18889_amd").Plan(c, [0, 1, 2, 3], [0], max_log2=10,
                                                sliced_wires=[(0, 9)])


def _oracle_with_plan_tree(plan, c, o, cb, sigma):
    leaf_canon, steps, base = plan.tree()
    wires = plan.sliced_wires()
    leaves = tn.canonical_network(c, o, cb)
    assert sorted(leaf_canon) == sorted(leaves)
    if wires:
        leaves = tn.fix_wires(leaves, wires, tn.slice_values(sigma, len(wires)))
    keep = tn._keep_labels(o)
    labels, data = tn.contract_tree(leaves, steps, base, keep)
    order = ([labels.index("b")] if "b" in labels else []) + \
        [labels.index(("o", int(q))) for q in reversed(list(o))]
    res = np.transpose(data, order).reshape(-1, 1 << len(o))
    if res.shape[0] == 1 and len(cb) > 1:
        res = np.repeat(res, len(cb), 0)
    return res


@pytest.mark.parametrize("grid,cycles,n_open,nb,cap", [((3, 4), 8, 12, 1, 20),
                                                       ((4, 4), 10, 4, 16, 14),
                                                       ((3, 5), 12, 3, 8, 14)])
def test_plan_tree_reproduces_state_vector(lib, grid, cycles, n_open, nb, cap):
    import paper_2406_18889_amd as lf
    c = wl.random_circuit(grid[0], grid[1], cycles, seed=5)
    n = c.n_qubits
    o = list(range(n - n_open, n))
    cb = wl.closed_bitstrings(n, o, nb, seed=6)
    plan = lf.Plan(c, o, cb, max_log2=cap, greedy_trials=4)
    inf = plan.info()
    assert inf["max_log2_intermediate"] <= cap
    exact = sv.group_amplitudes(c, o, cb)
    total = np.zeros_like(exact)
    for s in range(inf["n_slices"]):
        total += _oracle_with_plan_tree(plan, c, o, cb, s)
    assert np.abs(total - exact).max() < 1e-12


def test_plan_step_counts_recount(lib):
    """Per-step work recounted from the exported tree with the oracle's own
    network: a subtree's closed output legs stay separate legs while fewer
    than nb = log2(batch) of them are gathered, and become the batch index
    of 2^nb strings from there on."""
    import paper_2406_18889_amd as lf
    c = wl.random_circuit(4, 4, 10, seed=8)
    o = [12, 13, 14, 15]
    B = 16
    nb = 4
    cb = wl.closed_bitstrings(16, o, B, seed=9)
    plan = lf.Plan(c, o, cb, max_log2=12)
    leaf_canon, steps, base = plan.tree()
    wires = plan.sliced_wires()
    leaves = tn.fix_wires(tn.canonical_network(c, o, cb), wires, [0] * len(wires))
    # closed legs per leaf: the leaf holding the last two-qubit gate of q
    last = {}
    k = 0
    for g in c.gates:
        if len(g.qubits) == 2:
            for q in g.qubits:
                last[q] = k
            k += 1
    nclosed = {lid: 0 for lid in leaves}
    for q in range(16):
        if q not in o:
            nclosed[last[q]] += 1
    legs = {lid: {x: d for x, d in zip(l, t.shape) if x != "b"} for lid, (l, t) in leaves.items()}
    keep = tn._keep_labels(o)
    dims, macs, _ = plan.steps()
    biggest = 0
    for i, (a, b) in enumerate(steps):
        da, db = legs.pop(a), legs.pop(b)
        qa, qb = nclosed.pop(a), nclosed.pop(b)
        union = dict(da)
        union.update(db)
        plain = float(np.prod(list(union.values()), dtype=np.float64))
        batched = qa + qb >= nb
        expect = plain * (2.0 ** nb if batched else 2.0 ** (qa + qb))
        assert macs[i] == expect, (i, macs[i], expect)
        out = {x: v for x, v in union.items() if not (x in da and x in db) or x in keep}
        size = int(np.prod(list(out.values()), dtype=np.int64)) * (2 ** nb if batched else 2 ** (qa + qb))
        biggest = max(biggest, size)
        legs[base + i] = out
        nclosed[base + i] = qa + qb
        nz, nm, nn, nk = dims[i, :4]
        assert 2.0 ** (nz + nm + nn + nk) == macs[i]
        assert nz == (nb if batched else 0)
    assert biggest <= 2 ** plan.info()["max_log2_intermediate"]


def test_forced_slices_are_reported_in_order(lib):
    import paper_2406_18889_amd as lf
    c = wl.random_circuit(4, 4, 10, seed=77)
    o = [12, 13, 14, 15]
    cb = wl.closed_bitstrings(16, o, 4, seed=5)
    wires = tn.wire_list(tn.canonical_network(c, o, cb))
    pick = [wires[10], wires[3], wires[20]]
    plan = lf.Plan(c, o, cb, max_log2=24, sliced_wires=pick)
    assert plan.sliced_wires() == pick
    assert plan.info()["n_slices"] == 8


def test_bench_plan_matches_stored_slice_definition(lib):
    """The 53-qubit plan the benchmark times is what the stored oracle
    values of its slices were computed for: same sliced wires and tree
    (planning is deterministic: seeded search, restarts ranked by cost with
    ties to the lower rank, independent of thread timing)."""
    import json
    import bench
    import paper_2406_18889_amd as lf
    from tests.golden.make_rqc53 import PLAN_JSON, cases_for, tree_hash

    with open(PLAN_JSON) as f:
        pj = json.load(f)
    circ, openq, cb, spec = wl.standard_workload("rqc53")
    p = lf.Plan(circ, openq, cb, dtype="c64", max_log2=spec["max_log2"], search_dtype="chalf",
                **bench.PLAN_OPTS["rqc53"])
    wires = p.sliced_wires()
    leaf_canon, steps, base = p.tree()
    assert [list(w) for w in wires] == pj["sliced_wires"]
    assert tree_hash(wires, leaf_canon, steps, base) == pj["tree_hash"]
    assert [list(c) for c in cases_for(len(wires))] == pj["cases"]
    assert p.info()["max_log2_intermediate"] <= 28
    # the oracle contracts the same network along the stored tree: it must be
    # a full binary tree over the oracle's own leaves (checked by contract_tree
    # on the shapes only, via a dry run of the labels)
    leaves = tn.canonical_network(circ, openq, cb[:1])
    leaves = tn.fix_wires(leaves, [tuple(w) for w in pj["sliced_wires"]],
                          tn.slice_values(0, len(wires)))
    assert sorted(leaves) == sorted(pj["leaf_canon"])
    used = set()
    for a, b in pj["steps"]:
        assert a not in used and b not in used and a != b
        used.update((a, b))
    assert len(pj["steps"]) == len(leaves) - 1


def test_plan_options_mult_and_autotune_cache(lib, tmp_path):
    """lf_plan_opts.mult: 4M (or AUTO) builds, 3M is rejected with a message
    (the library computes every complex product as four real products);
    autotune_cache: a missing file is not an error, an existing one is
    merged into the process's kernel choices when the plan is built."""
    import paper_2406_18889_amd as lf
    from paper_2406_18889_amd import _lib
    c = wl.random_circuit(3, 3, 4, seed=2)
    o = [6, 7, 8]
    cb = wl.closed_bitstrings(9, o, 4, seed=1)
    for m in ("auto", "4m"):
        lf.Plan(c, o, cb, mult=m).close()
    with pytest.raises(_lib.LeapfrogError) as ex:
        lf.Plan(c, o, cb, mult="3m")
    assert "3M" in str(ex.value)
    missing = str(tmp_path / "none.txt")
    lf.Plan(c, o, cb, autotune_cache=missing).close()
    path = tmp_path / "tune.txt"
    path.write_text("3 9 4 5 1 1 1 11\n")
    lf.Plan(c, o, cb, autotune_cache=str(path)).close()
    out = tmp_path / "saved.txt"
    lf.autotune_save(str(out))
    assert "3 9 4 5 1 1 1 11" in out.read_text()


def test_batched_step_gathers_cover_closed_qubits(lib):
    """Every closed output leg is absorbed exactly once: over the batched
    steps, the closed qubits of the gathered (plain) operands are disjoint
    and together are all the closed qubits; the step where the batch index
    appears gathers both operands, later ones read the running batched
    tensor as one of them.  The batch order option changes no step."""
    import paper_2406_18889_amd as lf
    c = wl.random_circuit(4, 5, 10, seed=3)
    o = [16, 17, 18, 19]
    cb = wl.closed_bitstrings(20, o, 1000, seed=4)
    for keep in (False, True):
        p = lf.Plan(c, o, cb, max_log2=20, keep_batch_order=keep)
        dims, _, _ = p.steps()
        seen = []
        first = None
        for s in range(len(dims)):
            g = p.step_gather(s)
            if g[0][0] < 0:
                assert g[1][0] < 0
                continue
            if first is None:
                first = s
                assert g[0][0] == 0 and g[1][0] == 0
            else:
                assert g[0][0] + g[1][0] >= 1
            for stored, qs, strides in g:
                if stored == 0:
                    seen += qs
                    assert all(st > 0 for st in strides)
        closed = sorted(set(range(20)) - set(o))
        assert first is not None
        assert sorted(seen) == closed
        if keep:
            assert np.array_equal(dims, dims_sorted)
        dims_sorted = dims
        p.close()


def test_plan_info_groups_before_contraction(lib):
    """Grouped launches are set up by the first contraction (after tuning
    and calibration): a fresh plan reports none, with or without grouping."""
    import paper_2406_18889_amd as lf
    c = wl.random_circuit(3, 3, 4, seed=2)
    o = [6, 7, 8]
    cb = wl.closed_bitstrings(9, o, 4, seed=1)
    for g in (True, False):
        p = lf.Plan(c, o, cb, group_small_steps=g)
        info = p.info()
        assert info["n_step_groups"] == 0 and info["n_grouped_steps"] == 0
        p.close()
