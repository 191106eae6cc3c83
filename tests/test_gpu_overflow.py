"""Complex-half scaling edge cases and the saturation protocol, through the
C ABI (per-tensor power-of-two exponents are an extension: the paper
computes in complex64).

* Values far outside the half range (gates scaled by 2^+-20, amplitudes by
  2^+-60) are carried by the exponents: no saturation, same tolerance.
* A leaf multiplied by 2^12 after calibration (fault injection, exponent
  unchanged) saturates the slices that use it: LF_OVERFLOW under the report
  policy with the accumulator holding exactly the slices before the first
  saturated one; the rest contracted afterwards gives the uninterrupted
  result bit for bit; the recalibration policy recovers on its own.
* Batches report saturation, and a recorded batch graph follows a rebind.
Oracle: the state vector with projectors on the sliced wires (one slice) or
without (full sums), complex128.
"""

import dataclasses
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import sv, tn

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_built")]

torch = pytest.importorskip("torch")

C64_TOL = 1e-5
CHALF_TOL = 5e-3


def _say(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_18889_amd as lf
    from paper_2406_18889_amd import _lib
    _lib.load()
    return lf


def rel_err(a, ref):
    a = np.asarray(a).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def fidelity(a, ref):
    a = np.asarray(a).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    return float(abs(np.vdot(ref, a)) ** 2 / (np.vdot(a, a).real * np.vdot(ref, ref).real))


def _net(seed=77):
    c = wl.random_circuit(4, 4, 10, seed=seed)
    o = [12, 13, 14, 15]
    cb = wl.closed_bitstrings(16, o, 16, seed=5)
    wires = tn.wire_list(tn.canonical_network(c, o, cb))
    mid = [w for w in wires if w[1] == 3][:4]
    return c, o, cb, mid


def _plan(lf, c, o, cb, mid, dtype="chalf", **kw):
    return lf.Plan(c, o, cb, dtype=dtype, max_log2=20, sliced_wires=mid, chalf_min_log2=6,
                   **kw).bind()


def _slice_ref(c, o, cb, mid, sigma):
    v = tn.slice_values(sigma, len(mid))
    return sv.group_amplitudes(c, o, cb, [(q, j, x) for (q, j), x in zip(mid, v)])


@pytest.mark.parametrize("log2_gate", [-20, 20])
@pytest.mark.parametrize("dtype", ["chalf", "c64"])
def test_values_far_outside_half_range(lf, log2_gate, dtype):
    """Three two-qubit gates scaled by 2^log2_gate (amplitudes by 2^(3x)):
    far below the half subnormals or far above the half maximum; the
    exponents absorb the factor and nothing saturates."""
    c, o, cb, mid = _net()
    gates = list(c.gates)
    two = [i for i, g in enumerate(gates) if len(g.qubits) == 2]
    for i in (two[3], two[len(two) // 2], two[-2]):
        gates[i] = dataclasses.replace(gates[i], matrix=gates[i].matrix * 2.0 ** log2_gate)
    c2 = dataclasses.replace(c, gates=gates)
    exact = sv.group_amplitudes(c2, o, cb)
    assert abs(np.log2(np.linalg.norm(exact)) - 3 * log2_gate) < 8
    plan = _plan(lf, c2, o, cb, mid, dtype=dtype)
    got = plan.contract(0, 16).cpu().numpy()
    e, f = rel_err(got, exact), fidelity(got, exact)
    _say(f"gates x2^{log2_gate} {dtype}: rel_err={e:.2e} fidelity={f:.6f}")
    assert e < (CHALF_TOL if dtype == "chalf" else C64_TOL)
    assert f >= 0.999
    st = plan.overflow()
    assert st["saturated"] == 0 and st["first_bad_slice"] == -1 and st["recalibrations"] == 0


def test_injected_saturation_report_keeps_committed_prefix(lf):
    c, o, cb, mid = _net()
    plan = _plan(lf, c, o, cb, mid, overflow_policy="report")
    ref = _plan(lf, c, o, cb, mid, overflow_policy="report")
    assert plan.info()["n_half_steps"] > 0
    plan.contract(0, 1)               # calibration on slice 0, no saturation
    ref.contract(0, 1)
    torch.cuda.synchronize()
    # slices with bit 2 set (4..7, 12..15) now carry values 2^12 above the
    # calibration: 2^(12 + 12) exceeds the half range
    plan.debug_scale_slice_leaf(2, 1, 12)
    out = plan.new_amplitudes()
    with pytest.raises(lf.LeapfrogError) as ei:
        plan.contract(0, 16, out)
    assert ei.value.status == 5     # LF_OVERFLOW
    st = plan.overflow()
    _say(f"report policy: {st}")
    assert st["saturated"] > 0 and st["first_bad_slice"] == 4 and st["recalibrations"] == 0
    want = ref.contract(0, 4)
    torch.cuda.synchronize()
    assert torch.equal(out, want)
    # the committed prefix plus the rest equals the uninterrupted run, bit for bit
    plan.debug_scale_slice_leaf(2, 1, 0)
    plan.overflow(clear=True)
    plan.contract(4, 16, out)
    full = ref.contract(0, 16)
    torch.cuda.synchronize()
    assert torch.equal(out, full)
    exact = sv.group_amplitudes(c, o, cb)
    assert rel_err(full.cpu().numpy(), exact) < CHALF_TOL
    # without the check the call is asynchronous; the state says what was left out
    quiet = _plan(lf, c, o, cb, mid, check_overflow=False)
    quiet.contract(0, 1)
    quiet.debug_scale_slice_leaf(2, 1, 12)
    q_out = quiet.new_amplitudes()
    quiet.contract(0, 16, q_out)
    st = quiet.overflow(clear=True)
    assert st["saturated"] > 0 and st["first_bad_slice"] == 4
    torch.cuda.synchronize()
    assert torch.equal(q_out, want)


def test_injected_saturation_recalibrates(lf):
    c, o, cb, mid = _net()
    plan = _plan(lf, c, o, cb, mid)          # default policy: recalibrate
    plan.contract(0, 1)
    plan.debug_scale_slice_leaf(2, 1, 12)
    out = plan.contract(0, 16)
    st = plan.overflow()
    _say(f"recalibrate policy: {st}")
    assert st["recalibrations"] >= 1 and st["saturated"] == 0 and st["first_bad_slice"] == -1
    assert st["headroom_bits"] > 4
    w = [2.0 ** 12 if (s >> 2) & 1 else 1.0 for s in range(16)]
    want = sum(w[s] * _slice_ref(c, o, cb, mid, s) for s in range(16))
    got = out.cpu().numpy()
    e, f = rel_err(got, want), fidelity(got, want)
    _say(f"recalibrated sum: rel_err={e:.2e} fidelity={f:.6f}")
    assert e < CHALF_TOL and f >= 0.999
    # the unscaled slices keep their accuracy under the shifts fitted to the
    # 2^12 larger ones
    low = plan.contract(0, 4).cpu().numpy()
    want_low = sum(_slice_ref(c, o, cb, mid, s) for s in range(4))
    assert rel_err(low, want_low) < CHALF_TOL


def test_recalibrate_entry_point(lf):
    """lf_plan_recalibrate on another slice with more headroom gives the same
    amplitudes to the complex-half tolerance."""
    c, o, cb, mid = _net()
    plan = _plan(lf, c, o, cb, mid)
    a = plan.contract(0, 16).cpu().numpy()
    plan.recalibrate(9, headroom_bits=7)
    assert plan.overflow()["headroom_bits"] == 7
    b = plan.contract(0, 16).cpu().numpy()
    exact = sv.group_amplitudes(c, o, cb)
    assert rel_err(a, exact) < CHALF_TOL and rel_err(b, exact) < CHALF_TOL


def test_batch_reports_saturation(lf):
    c, o, cb, mid = _net()
    c2, o2, cb2, mid2 = _net(seed=78)
    bad = _plan(lf, c, o, cb, mid, overflow_policy="report")
    good = _plan(lf, c2, o2, cb2, mid2)
    bad.contract(0, 1)
    good.contract(0, 1)
    bad.debug_scale_slice_leaf(2, 1, 12)
    ob, og = bad.new_amplitudes(), good.new_amplitudes()
    items = [(bad, 0, 8, ob), (good, 0, 16, og), (bad, 8, 16, ob)]
    for mode in ("sequential", "graph"):
        ob.zero_()
        og.zero_()
        with pytest.raises(lf.LeapfrogError) as ei:
            lf.contract_batch(items, mode, lanes=2)
        assert ei.value.status == 5
        st = bad.overflow(clear=True)
        assert st["first_bad_slice"] == 4
        torch.cuda.synchronize()
        assert rel_err(og.cpu().numpy(), sv.group_amplitudes(c2, o2, cb2)) < CHALF_TOL
        want = sum(_slice_ref(c, o, cb, mid, s) for s in range(4))
        assert rel_err(ob.cpu().numpy(), want) < CHALF_TOL


def test_batch_graph_follows_rebind(lf):
    """A recorded batch graph is not replayed on a plan's old workspace: after
    a rebind (new workspace, new calibration) the batch equals sequential
    launches."""
    c, o, cb, mid = _net()
    c2, o2, cb2, mid2 = _net(seed=78)
    p1 = _plan(lf, c, o, cb, mid, dtype="c64")
    p2 = _plan(lf, c2, o2, cb2, mid2, dtype="c64")
    o1, o2_ = p1.new_amplitudes(), p2.new_amplitudes()
    items = [(p1, 0, 16, o1), (p2, 0, 16, o2_)]
    lf.contract_batch(items, "graph", lanes=2)
    torch.cuda.synchronize()
    first = (o1.clone(), o2_.clone())
    old_ws = p1.workspace
    p1.bind()                               # new workspace
    del old_ws
    torch.cuda.empty_cache()
    # likely to reuse the freed block: a stale replay would read 7.0s
    junk = torch.full((p1.info()["workspace_bytes"] // 4 + 64,), 7.0, device="cuda")
    o1.zero_()
    o2_.zero_()
    lf.contract_batch(items, "graph", lanes=2)
    torch.cuda.synchronize()
    del junk
    assert torch.equal(o1, first[0]) and torch.equal(o2_, first[1])
    s1, s2 = p1.new_amplitudes(), p2.new_amplitudes()
    lf.contract_batch([(p1, 0, 16, s1), (p2, 0, 16, s2)], "sequential")
    torch.cuda.synchronize()
    assert torch.equal(o1, s1) and torch.equal(o2_, s2)
