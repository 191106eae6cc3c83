"""Parity of the HIP path against the oracle, through the C ABI.

Tolerances (norm-wise relative error over the whole output, ||a - ref|| /
||ref||): complex64 1e-5; complex-half 5e-3 with fidelity overlap >= 0.999.
Top-k: bit-exact against the oracle's selection on the same amplitudes.
"""

import math
import os
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import sv, tn, topk

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
    _lib.load()  # fails loudly if the library is missing
    return lf


def rel_err(a, ref):
    a = np.asarray(a).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def fidelity(a, ref):
    a = np.asarray(a).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    return float(abs(np.vdot(ref, a)) ** 2 / (np.vdot(a, a).real * np.vdot(ref, ref).real))


# ------------------------------------------------------------- kernel pairs
def _ref_pair(A, B, nz, nm, nn, nk):
    Z, M, N, K = 1 << nz, 1 << nm, 1 << nn, 1 << nk
    a = A.reshape(Z, M, K).astype(np.complex128)
    b = B.reshape(Z, N, K).astype(np.complex128)
    return np.matmul(a, np.transpose(b, (0, 2, 1)))  # [Z, M, N]


def _rand_strides(nz, nm, nn, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(nz + nm + nn)
    return (1 << perm).astype(np.int64)  # bit b of the concatenated (z, m, n) -> stride


def _scatter(ref, nz, nm, nn, strides):
    Z, M, N = 1 << nz, 1 << nm, 1 << nn
    out = np.zeros(Z * M * N, np.complex128)
    z = np.arange(Z)[:, None, None]
    m = np.arange(M)[None, :, None]
    n = np.arange(N)[None, None, :]
    off = np.zeros((Z, M, N), np.int64)
    for b in range(nz):
        off += ((z >> b) & 1) * strides[b]
    for b in range(nm):
        off += ((m >> b) & 1) * strides[nz + b]
    for b in range(nn):
        off += ((n >> b) & 1) * strides[nz + nm + b]
    out[off.reshape(-1)] = ref.reshape(-1)
    return out


SHAPES = [
    # nz, nm, nn, nk: thin, tails below a tile, multi-tile, batch, K = 1
    (0, 10, 2, 2), (0, 3, 1, 0), (2, 6, 5, 3), (0, 8, 7, 6), (3, 7, 6, 5),
    (0, 9, 6, 9), (1, 4, 4, 1), (0, 5, 4, 4), (0, 12, 8, 4), (0, 8, 6, 1), (2, 7, 5, 0),
    (0, 9, 7, 2), (1, 9, 3, 3), (0, 8, 0, 6), (2, 8, 4, 0), (0, 13, 2, 2), (0, 10, 4, 4),
    (1, 8, 8, 0), (1, 10, 9, 3), (0, 9, 8, 3), (2, 7, 4, 5), (0, 6, 3, 6),
    # whole tiles of the large kernels (bounds-free loop, ordered write-out)
    (1, 9, 8, 5), (0, 10, 7, 6), (2, 8, 7, 7),
    # whole tiles, long K: the three-stage LDS ring wraps several times
    (0, 8, 7, 8), (0, 9, 7, 10),
    # more tiles than resident blocks: the persistent 4 x 2 tile loops
    (1, 14, 9, 5), (1, 14, 9, 3),
    # long K with a small result per batch entry (M, N <= 32): K split over waves
    (8, 5, 5, 9), (3, 4, 3, 10), (0, 5, 5, 7), (2, 2, 5, 8),
    # the 128 x 128 two-stage tile: one m tile, one and two k tiles
    (1, 7, 7, 5), (2, 7, 8, 6),
    # batched products with 32 or 64 rows per entry and N up to 32 complex
    # (the last stem steps): one wave per 32 rows, one or two B' fragments
    (3, 5, 5, 5), (2, 6, 5, 3), (1, 5, 5, 6), (2, 5, 3, 4), (4, 5, 5, 2), (1, 6, 4, 6),
    # batched steps of at least 2^8 entries: 16 entries per wave; B staged in
    # LDS per chunk when four slabs share it
    (8, 5, 5, 5), (8, 8, 2, 6), (8, 9, 3, 3), (9, 6, 4, 4), (8, 7, 1, 2),
]


def _applicable(kernel, dt, shape):
    nz, nm, nn, nk = shape
    if kernel == 1:
        return nm >= 5 and nn >= 4
    if kernel in (2, 8):
        return dt == "chalf" and nm >= 7 and nn >= 5
    if kernel == 3:
        return nm >= 8 and nk <= 6 and nn <= 8 and nn + nk <= 8
    if kernel in (4, 5, 6, 9, 10):
        return dt == "chalf" and nm >= 7 and nn >= 6
    if kernel == 7:
        return dt == "chalf" and nn <= 5 and 2 <= nk <= 6 and nm >= 5
    if kernel in (11, 12, 13, 14):
        return dt == "chalf" and nm >= 8 and nn >= 7 and 5 <= nk <= 21
    if kernel == 15:
        return dt == "chalf" and nm <= 5 and nn <= 5 and nk >= 7
    if kernel in (16, 17):
        return dt == "chalf" and nm >= 7 and nn >= 7 and 5 <= nk <= 21
    return True


@pytest.mark.parametrize("kernel", [0, 1, 3])
@pytest.mark.parametrize("shape", SHAPES)
def test_pair_c64(lf, kernel, shape):
    nz, nm, nn, nk = shape
    if not _applicable(kernel, "c64", shape):
        pytest.skip("kernel variant not applicable to this shape")
    _say(f"pair c64 kernel={kernel} shape={shape}")
    A = wl.random_complex((1 << (nz + nm + nk),), seed=1 + sum(shape)).astype(np.complex64)
    B = wl.random_complex((1 << (nz + nn + nk),), seed=2 + sum(shape)).astype(np.complex64)
    st = _rand_strides(nz, nm, nn, seed=3 + sum(shape))
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    dC = torch.zeros(1 << (nz + nm + nn), dtype=torch.complex64, device="cuda")
    lf.contract_pair(dA, dB, dC, nz, nm, nn, nk, st, 1.0, kernel)
    torch.cuda.synchronize()
    ref = _scatter(_ref_pair(A, B, nz, nm, nn, nk), nz, nm, nn, st)
    assert rel_err(dC.cpu().numpy(), ref) < C64_TOL


def _to_half_pairs(x, e):
    v = np.stack([x.real, x.imag], -1) * 2.0 ** (-e)
    return torch.from_numpy(v.astype(np.float16)).cuda()


@pytest.mark.parametrize("kernel", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17])
@pytest.mark.parametrize("shape", SHAPES)
def test_pair_chalf(lf, kernel, shape):
    nz, nm, nn, nk = shape
    if not _applicable(kernel, "chalf", shape):
        pytest.skip("kernel variant not applicable to this shape")
    _say(f"pair chalf kernel={kernel} shape={shape}")
    A = wl.random_complex((1 << (nz + nm + nk),), seed=11 + sum(shape))
    B = wl.random_complex((1 << (nz + nn + nk),), seed=12 + sum(shape))
    st = _rand_strides(nz, nm, nn, seed=13 + sum(shape))
    dA = _to_half_pairs(A, -8)
    dB = _to_half_pairs(B, -8)
    # stored A, B are value * 2^8; result scaled back by 2^-16 into half range
    dC = torch.zeros((1 << (nz + nm + nn), 2), dtype=torch.float16, device="cuda")
    lf.contract_pair(dA, dB, dC, nz, nm, nn, nk, st, 2.0 ** -16 * 64, kernel)
    torch.cuda.synchronize()
    Ah = (dA.cpu().numpy().astype(np.float64) @ np.array([1, 1j])) * 2.0 ** -8
    Bh = (dB.cpu().numpy().astype(np.float64) @ np.array([1, 1j])) * 2.0 ** -8
    ref = _scatter(_ref_pair(Ah, Bh, nz, nm, nn, nk), nz, nm, nn, st) * 64
    got = dC.cpu().numpy().astype(np.float64) @ np.array([1, 1j])
    # inputs exact in both; the only roundings are fp32 accumulation and the
    # final fp16 store
    assert rel_err(got, ref) < 2e-3


# Output layouts of the large complex-half tiles' write-out: n fastest (the
# two smallest strides are tile bits 1 and 2 apart: 16-byte stores), m
# fastest, z fastest (strides 1 and 2 outside the tile: 4-byte stores), and
# n fastest with a z bit between the two lowest n bits.
def _layout_strides(kind, nz, nm, nn):
    if kind == "n_fastest":
        bits = list(range(nz + nm, nz + nm + nn)) + list(range(nz, nz + nm)) + list(range(nz))
    elif kind == "m_fastest":
        bits = list(range(nz, nz + nm)) + list(range(nz + nm, nz + nm + nn)) + list(range(nz))
    elif kind == "z_fastest":
        bits = list(range(nz)) + list(range(nz + nm, nz + nm + nn)) + list(range(nz, nz + nm))
    else:  # "split_pair": n0, z0, n1, ...
        n = list(range(nz + nm, nz + nm + nn))
        bits = [n[0], 0] + n[1:] + list(range(nz, nz + nm)) + list(range(1, nz))
    st = np.zeros(nz + nm + nn, np.int64)
    for p, b in enumerate(bits):
        st[b] = 1 << p
    return st


@pytest.mark.parametrize("kernel", [2, 5, 8, 11, 12, 13, 14, 16, 17])
@pytest.mark.parametrize("layout", ["n_fastest", "m_fastest", "z_fastest", "split_pair"])
def test_pair_chalf_layouts(lf, kernel, layout):
    nz, nm, nn, nk = 1, 9, 8, 6
    if not _applicable(kernel, "chalf", (nz, nm, nn, nk)):
        pytest.skip("kernel variant not applicable to this shape")
    _say(f"pair chalf layout={layout} kernel={kernel}")
    A = wl.random_complex((1 << (nz + nm + nk),), seed=41)
    B = wl.random_complex((1 << (nz + nn + nk),), seed=42)
    st = _layout_strides(layout, nz, nm, nn)
    assert sorted(st.tolist()) == [1 << i for i in range(nz + nm + nn)]
    dA = _to_half_pairs(A, -8)
    dB = _to_half_pairs(B, -8)
    dC = torch.zeros((1 << (nz + nm + nn), 2), dtype=torch.float16, device="cuda")
    lf.contract_pair(dA, dB, dC, nz, nm, nn, nk, st, 2.0 ** -16 * 64, kernel)
    torch.cuda.synchronize()
    Ah = (dA.cpu().numpy().astype(np.float64) @ np.array([1, 1j])) * 2.0 ** -8
    Bh = (dB.cpu().numpy().astype(np.float64) @ np.array([1, 1j])) * 2.0 ** -8
    ref = _scatter(_ref_pair(Ah, Bh, nz, nm, nn, nk), nz, nm, nn, st) * 64
    got = dC.cpu().numpy().astype(np.float64) @ np.array([1, 1j])
    assert rel_err(got, ref) < 2e-3


# The streaming kernels over the same layouts.
@pytest.mark.parametrize("kernel", [0, 3, 7])
@pytest.mark.parametrize("layout", ["n_fastest", "m_fastest", "z_fastest", "split_pair"])
@pytest.mark.parametrize("shape", [(1, 9, 4, 2), (2, 8, 2, 4), (1, 10, 3, 3),
                                   # 32 x 32 blocks per entry: staged write-out when
                                   # each entry's block is contiguous (n or m fastest)
                                   (8, 5, 5, 5), (3, 5, 5, 3), (9, 5, 5, 6)])
def test_pair_chalf_streaming_layouts(lf, kernel, layout, shape):
    nz, nm, nn, nk = shape
    if not _applicable(kernel, "chalf", shape):
        pytest.skip("kernel variant not applicable to this shape")
    _say(f"pair chalf streaming layout={layout} kernel={kernel} shape={shape}")
    A = wl.random_complex((1 << (nz + nm + nk),), seed=51 + sum(shape))
    B = wl.random_complex((1 << (nz + nn + nk),), seed=52 + sum(shape))
    st = _layout_strides(layout, nz, nm, nn)
    assert sorted(st.tolist()) == [1 << i for i in range(nz + nm + nn)]
    dA = _to_half_pairs(A, -8)
    dB = _to_half_pairs(B, -8)
    dC = torch.zeros((1 << (nz + nm + nn), 2), dtype=torch.float16, device="cuda")
    lf.contract_pair(dA, dB, dC, nz, nm, nn, nk, st, 2.0 ** -16 * 64, kernel)
    torch.cuda.synchronize()
    Ah = (dA.cpu().numpy().astype(np.float64) @ np.array([1, 1j])) * 2.0 ** -8
    Bh = (dB.cpu().numpy().astype(np.float64) @ np.array([1, 1j])) * 2.0 ** -8
    ref = _scatter(_ref_pair(Ah, Bh, nz, nm, nn, nk), nz, nm, nn, st) * 64
    got = dC.cpu().numpy().astype(np.float64) @ np.array([1, 1j])
    assert rel_err(got, ref) < 2e-3


@pytest.mark.parametrize("kernel", [0, 3, 7])
@pytest.mark.parametrize("shape", [(0, 10, 2, 2), (1, 9, 3, 3), (0, 10, 4, 4), (2, 7, 4, 5),
                                   (0, 6, 3, 6), (0, 8, 0, 6), (0, 13, 2, 2), (3, 5, 3, 4),
                                   (1, 5, 4, 6), (2, 6, 2, 3)])
def test_pair_mixed_half_a_c64_b(lf, kernel, shape):
    """Complex-half A with a complex64 B (the planner keeps small B
    operands in complex64), complex64 result: B enters the streaming kernels
    exactly and the MFMA kernel as a high + low half pair."""
    nz, nm, nn, nk = shape
    if not _applicable(kernel, "chalf", shape):
        pytest.skip("kernel variant not applicable to this shape")
    _say(f"pair mixed kernel={kernel} shape={shape}")
    A = wl.random_complex((1 << (nz + nm + nk),), seed=31 + sum(shape))
    B = wl.random_complex((1 << (nz + nn + nk),), seed=32 + sum(shape)).astype(np.complex64)
    st = _rand_strides(nz, nm, nn, seed=33 + sum(shape))
    dA = _to_half_pairs(A, 0)
    dB = torch.from_numpy(B).cuda()
    dC = torch.zeros(1 << (nz + nm + nn), dtype=torch.complex64, device="cuda")
    lf.contract_pair(dA, dB, dC, nz, nm, nn, nk, st, 1.0, kernel)
    torch.cuda.synchronize()
    Ah = dA.cpu().numpy().astype(np.float64) @ np.array([1, 1j])
    ref = _scatter(_ref_pair(Ah, B.astype(np.complex128), nz, nm, nn, nk), nz, nm, nn, st)
    assert rel_err(dC.cpu().numpy(), ref) < C64_TOL


@pytest.mark.parametrize("kernel,shape", [(1, (0, 7, 5, 6)), (11, (0, 8, 7, 6)), (12, (1, 8, 7, 5)),
                                          (13, (0, 9, 7, 8)), (14, (1, 8, 8, 5)), (15, (6, 5, 5, 9)),
                                          (16, (1, 7, 7, 6)), (17, (0, 8, 7, 9))])
def test_pair_half_in_c64_out(lf, kernel, shape):
    nz, nm, nn, nk = shape
    _say(f"pair half in, c64 out kernel={kernel} shape={shape}")
    A = wl.random_complex((1 << (nz + nm + nk),), seed=21)
    B = wl.random_complex((1 << (nz + nn + nk),), seed=22)
    st = _rand_strides(nz, nm, nn, seed=23)
    dA, dB = _to_half_pairs(A, 0), _to_half_pairs(B, 0)
    dC = torch.zeros(1 << (nz + nm + nn), dtype=torch.complex64, device="cuda")
    lf.contract_pair(dA, dB, dC, nz, nm, nn, nk, st, 1.0, kernel)
    torch.cuda.synchronize()
    Ah = dA.cpu().numpy().astype(np.float64) @ np.array([1, 1j])
    Bh = dB.cpu().numpy().astype(np.float64) @ np.array([1, 1j])
    ref = _scatter(_ref_pair(Ah, Bh, nz, nm, nn, nk), nz, nm, nn, st)
    assert rel_err(dC.cpu().numpy(), ref) < 1e-5


# ---------------------------------------------------------- whole circuits
def test_rqc12_full_amplitudes_c64(lf):
    """Configuration 1: 12 qubits, 8 cycles, all open, no slicing."""
    _say("rqc12 c64")
    c, o, cb, spec = wl.standard_workload("rqc12")
    ref = sv.group_amplitudes(c, o, cb)
    plan = lf.Plan(c, o, cb, max_log2=spec["max_log2"]).bind()
    out = plan.contract(0, plan.info()["n_slices"])
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert got.shape == (1, 4096)
    assert rel_err(got, ref) < C64_TOL


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_rqc12_other_seeds(lf, seed):
    c = wl.random_circuit(3, 4, 8, seed)
    o = np.arange(12)
    cb = np.zeros(1, np.uint64)
    ref = sv.group_amplitudes(c, o, cb)
    plan = lf.Plan(c, o, cb, max_log2=20).bind()
    got = plan.contract(0, plan.info()["n_slices"]).cpu().numpy()
    assert rel_err(got, ref) < C64_TOL


def _small_sliced(lf, dtype="c64", launch="stream", n_batch=16, chalf_min=16):
    c = wl.random_circuit(4, 4, 10, seed=77)
    o = [12, 13, 14, 15]
    cb = wl.closed_bitstrings(16, o, n_batch, seed=5)
    wires = tn.wire_list(tn.canonical_network(c, o, cb))
    mid = [w for w in wires if w[1] == 3][:4]
    plan = lf.Plan(c, o, cb, dtype=dtype, max_log2=20, sliced_wires=mid, launch=launch,
                   slices_per_graph=4, chalf_min_log2=chalf_min).bind()
    return c, o, cb, mid, plan


def test_slices_match_projector_state_vector(lf):
    """Each slice equals the state vector with projectors on the sliced wires;
    the full range equals the exact amplitudes (slicing identity)."""
    c, o, cb, mid, plan = _small_sliced(lf)
    assert plan.sliced_wires() == mid
    total = np.zeros((len(cb), 1 << len(o)), np.complex128)
    for s in range(16):
        _say(f"slice {s}")
        got = plan.contract(s, s + 1).cpu().numpy()
        v = tn.slice_values(s, 4)
        ref = sv.group_amplitudes(c, o, cb, [(q, j, x) for (q, j), x in zip(mid, v)])
        assert rel_err(got, ref) < C64_TOL
        total += got
    exact = sv.group_amplitudes(c, o, cb)
    assert rel_err(total, exact) < C64_TOL
    full = plan.contract(0, 16).cpu().numpy()
    assert rel_err(full, exact) < C64_TOL


def test_slice_additivity_and_determinism(lf):
    _, _, _, _, plan = _small_sliced(lf)
    a = plan.contract(0, 16)
    b = plan.new_amplitudes()
    plan.contract(0, 5, b)
    plan.contract(5, 11, b)
    plan.contract(11, 16, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    c2 = plan.contract(0, 16)
    assert torch.equal(a, c2)
    empty = plan.contract(3, 3)
    assert torch.count_nonzero(empty).item() == 0


def test_graph_launch_matches_stream(lf):
    _, _, _, _, p1 = _small_sliced(lf, launch="stream")
    _, _, _, _, p2 = _small_sliced(lf, launch="graph")
    a = p1.contract(0, 16)
    b = p2.contract(0, 16)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # replay again (graph reuse) with eager work between replays
    b2 = p2.new_amplitudes()
    p2.contract(0, 9, b2)
    torch.cuda.synchronize()
    p2.contract(9, 16, b2)
    torch.cuda.synchronize()
    assert torch.equal(a, b2)


def test_live_kernel_timing_counts_launches(lf):
    """lf_plan_time_kernel brackets exactly the launches of the chosen
    kernel inside ordinary contractions (what bench.py's roofline divides
    by), and leaves the results unchanged."""
    _, _, _, _, plan = _small_sliced(lf)
    ref = plan.contract(0, 16)
    torch.cuda.synchronize()
    dims, _, _ = plan.steps()
    var = dims[:, 4] == 1
    kernel = int(np.bincount(dims[var, 7]).argmax())
    per_slice = int((var & (dims[:, 7] == kernel)).sum())
    plan.time_kernel(kernel, reserve=per_slice * 16)
    got = plan.contract(0, 16)
    total_ms, n, per_ms, per_n = plan.kernel_times()
    plan.time_kernel(-1)
    assert n == per_slice * 16
    assert int(per_n.sum()) == n and bool(((per_n > 0) == (var & (dims[:, 7] == kernel))).all())
    assert total_ms > 0 and abs(float(per_ms.sum()) - total_ms) < 1e-6 * max(1.0, total_ms)
    assert torch.equal(got, ref)
    # the counters restart after a read; timing off records nothing
    plan.contract(0, 4, got)
    assert plan.kernel_times()[1] == 0


def test_complex_half_small(lf):
    c, o, cb, mid, plan = _small_sliced(lf, dtype="chalf", chalf_min=6)
    assert plan.info()["n_half_steps"] > 0
    got = plan.contract(0, 16).cpu().numpy()
    exact = sv.group_amplitudes(c, o, cb)
    e = rel_err(got, exact)
    f = fidelity(got, exact)
    _say(f"chalf small rel_err={e:.2e} fidelity={f:.6f}")
    assert e < CHALF_TOL
    assert f >= 0.999


def test_rqc12_complex_half(lf):
    c, o, cb, spec = wl.standard_workload("rqc12")
    ref = sv.group_amplitudes(c, o, cb)
    plan = lf.Plan(c, o, cb, dtype="chalf", max_log2=spec["max_log2"], chalf_min_log2=4).bind()
    got = plan.contract(0, 1).cpu().numpy()
    e, f = rel_err(got, ref), fidelity(got, ref)
    _say(f"rqc12 chalf rel_err={e:.2e} fidelity={f:.6f}")
    assert e < CHALF_TOL and f >= 0.999


# -------------------------------------------------------------------- top-k
@pytest.mark.parametrize("gs,k", [(64, 1), (64, 7), (1024, 1), (1024, 33), (256 * 64, 100)])
def test_topk_bit_exact(lf, gs, k):
    rng = np.random.Generator(np.random.PCG64(gs + k))
    n = 256 * 64 if gs <= 256 * 64 else gs
    n = max(n, gs)
    a = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / 64
    # planted ties: duplicated values inside groups
    a[5::97] = a[3]
    d = torch.from_numpy(a).cuda()
    idx, prob = lf.postselect_topk(d, gs, k)
    i_ref, p_ref = topk.topk(a, gs, k)
    assert np.array_equal(idx.cpu().numpy(), i_ref)
    assert np.array_equal(prob.cpu().numpy(), p_ref)


def test_topk_on_contracted_amplitudes(lf):
    c, o, cb, mid, plan = _small_sliced(lf)
    amps = plan.contract(0, 16)
    idx, prob = lf.postselect_topk(amps, 16, 1)
    i_ref, p_ref = topk.topk(amps.cpu().numpy(), 16, 1)
    assert np.array_equal(idx.cpu().numpy(), i_ref)
    assert np.array_equal(prob.cpu().numpy(), p_ref)


# ------------------------------------------------------------- 30 qubits
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rqc30_plan(lf, dtype="c64", **kw):
    from tests.golden.make_rqc30 import RQC30_SLICED_WIRES
    c, o, cb, spec = wl.standard_workload("rqc30")
    plan = lf.Plan(c, o, cb, dtype=dtype, max_log2=spec["max_log2"],
                   sliced_wires=RQC30_SLICED_WIRES, **kw).bind()
    return plan


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLD, "rqc30_exact.npy")),
                    reason="30-qubit oracle values not generated")
def test_rqc30_full_sum_c64(lf):
    """Configuration 2: 30 qubits, 14 cycles, 6 open, 256 closed strings,
    2^8 slices; the sum of all slices equals the state vector."""
    _say("rqc30 c64 full")
    ref = np.load(os.path.join(GOLD, "rqc30_exact.npy"))
    plan = _rqc30_plan(lf)
    assert plan.info()["n_slices"] == 256
    got = plan.contract(0, 256).cpu().numpy()
    assert rel_err(got, ref) < C64_TOL
    idx, _ = lf.postselect_topk(plan.contract(0, 256), 64, 1)
    i_ref, _ = topk.topk(ref, 64, 1)
    # selection from c64 amplitudes agrees with the exact one except where
    # the two largest probabilities are within the error bound
    p = topk.probabilities(ref)
    agree = idx.cpu().numpy()[:, 0] == i_ref[:, 0]
    for g in np.nonzero(~agree)[0]:
        top2 = np.sort(p[g])[-2:]
        assert top2[1] - top2[0] <= 4 * C64_TOL * top2[1]


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLD, "rqc30_prefix_D1.npy")),
                    reason="30-qubit prefix oracle values not generated")
@pytest.mark.parametrize("D", [1, 2, 3, 4, 5])
def test_rqc30_prefix_partial_sums(lf, D):
    """A slice prefix [0, 2^(8-D)) equals the state vector with the D
    most significant sliced wires projected on 0 (fraction f = 2^-D)."""
    ref = np.load(os.path.join(GOLD, f"rqc30_prefix_D{D}.npy"))
    plan = _rqc30_plan(lf)
    got = plan.contract(0, 1 << (8 - D)).cpu().numpy()
    assert rel_err(got, ref) < C64_TOL


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLD, "rqc30_exact.npy")),
                    reason="30-qubit oracle values not generated")
def test_rqc30_full_sum_complex_half(lf):
    ref = np.load(os.path.join(GOLD, "rqc30_exact.npy"))
    plan = _rqc30_plan(lf, dtype="chalf")
    got = plan.contract(0, 256).cpu().numpy()
    e, f = rel_err(got, ref), fidelity(got, ref)
    _say(f"rqc30 chalf rel_err={e:.2e} fidelity={f:.6f} half_steps={plan.info()['n_half_steps']}")
    assert e < CHALF_TOL and f >= 0.999


# ------------------------------------------------- batched uneven subtasks
@pytest.mark.parametrize("dtype", ["c64", "chalf"])
def test_batch_order_does_not_change_amplitudes(lf, dtype):
    """1000 closed strings (padded to 2^10) of a 20-qubit circuit: the
    library's own contraction order (sorted by the gathered closed bits) and
    the caller's order give the same out_amps bit for bit (each string's
    values go through the same arithmetic), in the caller's row order, and
    both match the state vector."""
    _say(f"batch order {dtype}")
    c = wl.random_circuit(4, 5, 10, seed=3)
    o = [16, 17, 18, 19]
    cb = wl.closed_bitstrings(20, o, 1000, seed=4)
    ref = sv.group_amplitudes(c, o, cb)
    outs = []
    for keep in (False, True):
        plan = lf.Plan(c, o, cb, dtype=dtype, max_log2=20, keep_batch_order=keep,
                       chalf_min_log2=8).bind()
        out = plan.contract(0, plan.info()["n_slices"])
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
        plan.workspace = None
        plan.close()
    assert outs[0].shape == (1000, 16)
    assert np.array_equal(outs[0], outs[1])
    assert rel_err(outs[0], ref) < (C64_TOL if dtype == "c64" else CHALF_TOL)


def test_batched_skinny_steps_with_gathers(lf, tmp_path):
    """The skinny kernel on the batched steps of a plan (entry chunks that
    reuse a gathered block while it does not change, in the library's sorted
    order and in the caller's order): kernel 7 is forced on every batched
    step it applies to, and the amplitudes match the state vector."""
    _say("batched skinny steps")
    c = wl.random_circuit(4, 5, 10, seed=3)
    o = [16, 17, 18, 19]
    cb = wl.closed_bitstrings(20, o, 1000, seed=4)
    ref = sv.group_amplitudes(c, o, cb)
    probe = lf.Plan(c, o, cb, dtype="chalf", max_log2=20, chalf_min_log2=8)
    dims, _, _ = probe.steps()
    lines = []
    for s in range(len(dims)):
        nz, nm, nn, nk = (int(x) for x in dims[s, :4])
        if nz > 0 and dims[s, 5] == 1 and nn <= 5 and 2 <= nk <= 6 and nm >= 5:
            lines.append(f"{nz} {nm} {nn} {nk} 1 1 {int(dims[s, 6])} 7\n")
    probe.close()
    assert lines, "no batched step of this plan fits the skinny kernel"
    path = tmp_path / "tune.txt"
    path.write_text("".join(lines))
    lf.autotune_load(str(path))
    outs = []
    for keep in (False, True):
        plan = lf.Plan(c, o, cb, dtype="chalf", max_log2=20, chalf_min_log2=8, keep_batch_order=keep).bind()
        dims, _, _ = plan.steps()
        out = plan.contract(0, plan.info()["n_slices"])
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
        plan.workspace = None
        plan.close()
    assert np.array_equal(outs[0], outs[1])
    e = rel_err(outs[0], ref)
    _say(f"rel_err {e:.2e}")
    assert e < CHALF_TOL


@pytest.mark.parametrize("dtype", ["c64", "chalf"])
@pytest.mark.parametrize("launch", ["stream", "graph"])
def test_grouped_small_steps_identical(lf, dtype, launch):
    """Small independent streaming steps grouped into one launch give the
    same amplitudes bit for bit as one launch per step, on the 30-qubit
    workload (many small steps per slice), and match the oracle."""
    if not os.path.exists(os.path.join(GOLD, "rqc30_exact.npy")):
        pytest.skip("stored 30-qubit amplitudes not generated")
    _say(f"grouped small steps {dtype} {launch}")
    c, o, cb, spec = wl.standard_workload("rqc30")
    outs = []
    for grouped in (True, False):
        plan = lf.Plan(c, o, cb, dtype=dtype, max_log2=spec["max_log2"], sliced_wires=wl.RQC30_SLICED_WIRES,
                       launch=launch, slices_per_graph=8, group_small_steps=grouped).bind()
        out = plan.contract(0, 32)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
        info = plan.info()
        _say(f"grouped={grouped}: {info['n_step_groups']} groups of {info['n_grouped_steps']} steps")
        if grouped:
            assert info["n_step_groups"] > 0 and info["n_grouped_steps"] >= 2 * info["n_step_groups"]
        else:
            assert info["n_step_groups"] == 0
        plan.workspace = None
        plan.close()
    assert np.array_equal(outs[0], outs[1])


def test_batch_graph_matches_sequential(lf):
    """Many subtasks of uneven shape from several circuits: one recorded
    graph with parallel lanes gives bit-identical accumulators to per-item
    launches, and both equal per-plan contract calls in item order; each
    accumulator equals the oracle's projector state vector for its slices."""
    circuits, subtasks = wl.mixed_workload(4, 48, seed=11, small=True)
    plans = [lf.Plan(c["circuit"], c["open_qubits"], c["closed_bits"], max_log2=c["max_log2"],
                     dtype="c64").bind() for c in circuits]
    items_s, items_g = [], []
    outs_s = [p.new_amplitudes() for p in plans]
    outs_g = [p.new_amplitudes() for p in plans]
    outs_r = [p.new_amplitudes() for p in plans]
    for (k, draw) in subtasks:
        ns = plans[k].info()["n_slices"]
        s0 = draw % ns
        items_s.append((plans[k], s0, s0 + 1, outs_s[k]))
        items_g.append((plans[k], s0, s0 + 1, outs_g[k]))
        plans[k].contract(s0, s0 + 1, outs_r[k])
    lf.contract_batch(items_s, "sequential")
    lf.contract_batch(items_g, "graph", lanes=2)
    torch.cuda.synchronize()
    for k in range(len(plans)):
        assert torch.equal(outs_s[k], outs_g[k])
        assert torch.equal(outs_s[k], outs_r[k])
    # replay the same recorded graph (eager work in between) and tune lanes
    for o in outs_g:
        o.zero_()
    torch.cuda.synchronize()
    lf.contract_batch(items_g, "graph", lanes=2)
    torch.cuda.synchronize()
    for k in range(len(plans)):
        assert torch.equal(outs_s[k], outs_g[k])
    for o in outs_g:
        o.zero_()
    lf.contract_batch(items_g, "graph", lanes=0)
    torch.cuda.synchronize()
    for k in range(len(plans)):
        assert torch.equal(outs_s[k], outs_g[k])
    # oracle: each accumulator is a sum of slices (with multiplicity)
    for k, c in enumerate(circuits[:2]):
        wires = plans[k].sliced_wires()
        ref = np.zeros((len(c["closed_bits"]), 1 << len(c["open_qubits"])), np.complex128)
        for (kk, draw) in subtasks:
            if kk != k:
                continue
            s0 = draw % plans[k].info()["n_slices"]
            v = tn.slice_values(s0, len(wires))
            ref += sv.group_amplitudes(c["circuit"], c["open_qubits"], c["closed_bits"],
                                       [(q, j, x) for (q, j), x in zip(wires, v)])
        if np.linalg.norm(ref) > 0:
            assert rel_err(outs_s[k].cpu().numpy(), ref) < C64_TOL


# ------------------------------------------- 53 qubits, the benchmark's plan
def _rqc53_stored():
    import json
    with open(os.path.join(GOLD, "rqc53_plan.json")) as f:
        return json.load(f), np.load(os.path.join(GOLD, "rqc53_slices.npy"))


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLD, "rqc53_slices.npy")),
                    reason="stored 53-qubit slice values not generated")
@pytest.mark.parametrize("dtype", ["c64", "chalf"])
def test_rqc53_bench_plan_slices_vs_oracle(lf, dtype):
    """Configuration 3 at full size, on the plan the benchmark times (its
    search options: 8 restarts, 4M annealing moves; 2^39 slices): slices
    0..3 for closed strings 0, 37, 128, 255 and one far slice for string
    200, all 1024 open values each, against the oracle's complex128
    contraction of the same sliced sub-networks (stored values).  The
    complex-half plan calibrates its shifts on slice 0 and reuses them on the
    others, as the benchmark does; saturation fails the test.  Complex64 to
    1e-5, complex-half to 5e-3 with fidelity >= 0.999, per case."""
    import bench
    from tests.golden.make_rqc53 import tree_hash

    pj, ref = _rqc53_stored()
    c, o, cb, spec = wl.standard_workload("rqc53")
    plan = lf.Plan(c, o, cb, dtype=dtype, max_log2=spec["max_log2"], search_dtype="chalf",
                   check_overflow=True, overflow_policy="report", **bench.PLAN_OPTS["rqc53"])
    wires = plan.sliced_wires()
    leaf_canon, steps, base = plan.tree()
    assert tree_hash(wires, leaf_canon, steps, base) == pj["tree_hash"], \
        "the benchmark's plan changed: regenerate tests/golden/rqc53_*"
    assert plan.info()["max_log2_intermediate"] <= 28
    plan.bind()
    tol = C64_TOL if dtype == "c64" else CHALF_TOL
    sigmas = []
    for (s, _) in pj["cases"]:
        if s not in sigmas:
            sigmas.append(s)
    assert sigmas[0] == 0
    got = {}
    for s in sigmas:
        got[s] = plan.contract(s, s + 1).cpu().numpy()
    ov = plan.overflow()
    assert ov["saturated"] == 0 and ov["first_bad_slice"] == -1
    worst = 0.0
    for i, (s, b) in enumerate(pj["cases"]):
        e, f = rel_err(got[s][b], ref[i]), fidelity(got[s][b], ref[i])
        _say(f"rqc53 {dtype} slice {s} string {b}: rel_err={e:.2e} fidelity={f:.6f}")
        worst = max(worst, e)
        assert e < tol
        if dtype == "chalf":
            assert f >= 0.999
    _say(f"rqc53 {dtype}: worst rel_err {worst:.2e} over {len(pj['cases'])} cases")
    plan.workspace = None
    plan.close()
    torch.cuda.empty_cache()
