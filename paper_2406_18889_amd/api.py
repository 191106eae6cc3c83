"""Python face of the C-ABI library: the same calls as include/leapfrog.h.

PyTorch supplies device memory (workspace, amplitude and top-k buffers) and
streams; every computation runs in the library.
"""

from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import _lib
from ._lib import check

DTYPES = {"c64": _lib.LF_C64, "complex64": _lib.LF_C64, "chalf": _lib.LF_CHALF,
          "complex-half": _lib.LF_CHALF}
COST = {"flopmem": _lib.LF_COST_FLOPMEM, "mlp": _lib.LF_COST_MLP}
LAUNCH = {"stream": _lib.LF_LAUNCH_STREAM, "graph": _lib.LF_LAUNCH_GRAPH}
OVERFLOW_POLICY = {"recalibrate": _lib.LF_OVERFLOW_RECALIBRATE, "report": _lib.LF_OVERFLOW_REPORT}


def _circuit_struct(circuit):
    n = len(circuit.gates)
    arr = (_lib.lf_gate * max(n, 1))()
    for i, g in enumerate(circuit.gates):
        arr[i].n_q = len(g.qubits)
        arr[i].q[0] = g.qubits[0]
        arr[i].q[1] = g.qubits[1] if len(g.qubits) > 1 else -1
        arr[i].layer = g.cycle
        flat = np.asarray(g.matrix, np.complex128).reshape(-1)
        for e, v in enumerate(flat):
            arr[i].mat[2 * e] = v.real
            arr[i].mat[2 * e + 1] = v.imag
    c = _lib.lf_circuit(circuit.n_qubits, n, ctypes.cast(arr, ctypes.POINTER(_lib.lf_gate)))
    return c, arr


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """Opaque plan handle (lf_plan); destroyed with close() or on collection."""

    def __init__(self, circuit, open_qubits: Sequence[int], closed_bits: Sequence[int],
                 dtype: str = "c64", max_log2: int = 28, n_sliced: int = -1,
                 sliced_wires: Optional[Sequence[Tuple[int, int]]] = None,
                 cost_model: str = "flopmem", greedy_trials: int = 8,
                partition_trials: int = 64, sa_iters: int = 0,
                 seed: int = 1, chalf_min_log2: int = 16, launch: str = "stream",
                 check_overflow: bool = True, slices_per_graph: int = 8,
                 search_dtype: Optional[str] = None, autotune: bool = True,
                 restarts: int = 1, chalf_headroom_bits: int = 4,
                 overflow_policy: str = "recalibrate", chalf_exec_min_log2: int = -1,
                 mult: str = "auto", autotune_cache: Optional[str] = None,
                 keep_batch_order: bool = False, group_small_steps: bool = True):
        lib = _lib.load()
        self._lib = lib
        self._handle = ctypes.c_void_p()
        self.n_qubits = circuit.n_qubits
        self.open_qubits = [int(q) for q in open_qubits]
        self.closed_bits = np.asarray(closed_bits, np.uint64)
        opts = _lib.lf_plan_opts()
        lib.lf_plan_opts_default(ctypes.byref(opts))
        opts.dtype = DTYPES[dtype]
        opts.max_log2_intermediate = max_log2
        opts.n_sliced_wires = n_sliced
        keep = None
        if sliced_wires:
            flat = np.asarray(sliced_wires, np.int32).reshape(-1)
            keep = (ctypes.c_int32 * flat.size)(*flat.tolist())
            opts.sliced_wires = ctypes.cast(keep, ctypes.POINTER(ctypes.c_int32))
            opts.n_forced = len(sliced_wires)
        opts.cost_model = COST[cost_model]
        opts.greedy_trials = greedy_trials
        opts.partition_trials = partition_trials
        opts.sa_iters = sa_iters
        opts.seed = seed
        opts.chalf_min_log2 = chalf_min_log2
        opts.launch_mode = LAUNCH[launch]
        opts.check_overflow = 1 if check_overflow else 0
        opts.slices_per_graph = slices_per_graph
        opts.search_dtype = -1 if search_dtype is None else DTYPES[search_dtype]
        opts.autotune = 1 if autotune else 0
        opts.restarts = int(restarts)
        opts.chalf_headroom_bits = int(chalf_headroom_bits)
        opts.overflow_policy = OVERFLOW_POLICY[overflow_policy]
        opts.chalf_exec_min_log2 = int(chalf_exec_min_log2)
        opts.mult = {"auto": _lib.LF_MULT_AUTO, "4m": _lib.LF_MULT_4M, "3m": _lib.LF_MULT_3M}[mult.lower()]
        cache = autotune_cache.encode() if autotune_cache else None
        opts.autotune_cache = cache
        opts.keep_batch_order = int(bool(keep_batch_order))
        opts.group_small_steps = int(bool(group_small_steps))
        c, arr = _circuit_struct(circuit)
        openq = (ctypes.c_int32 * max(1, len(self.open_qubits)))(*self.open_qubits)
        cb = np.ascontiguousarray(self.closed_bits)
        st = lib.lf_build_network(ctypes.byref(c), openq, len(self.open_qubits),
                                  cb.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), cb.size,
                                  ctypes.byref(opts), ctypes.byref(self._handle))
        del arr, keep, cache
        check(st, "lf_build_network")
        self.workspace = None
        self.dtype = dtype

    # ---------------------------------------------------------------- info
    def info(self) -> dict:
        inf = _lib.lf_plan_info()
        check(self._lib.lf_plan_get_info(self._handle, ctypes.byref(inf)), "lf_plan_get_info")
        return {name: getattr(inf, name) for name, _ in inf._fields_}

    def sliced_wires(self) -> List[Tuple[int, int]]:
        n = self.info()["n_sliced_wires"]
        buf = (ctypes.c_int32 * max(1, 2 * n))()
        check(self._lib.lf_plan_sliced_wires(self._handle, buf), "lf_plan_sliced_wires")
        return [(buf[2 * t], buf[2 * t + 1]) for t in range(n)]

    def tree(self):
        """(leaf canonical ids, [(left, right)] per step, id_base)."""
        inf = self.info()
        L, S = inf["n_leaves"], inf["n_steps"]
        lc = (ctypes.c_int32 * max(1, L))()
        le = (ctypes.c_int32 * max(1, S))()
        ri = (ctypes.c_int32 * max(1, S))()
        check(self._lib.lf_plan_tree(self._handle, lc, le, ri), "lf_plan_tree")
        return [lc[i] for i in range(L)], [(le[s], ri[s]) for s in range(S)], inf["leaf_id_base"]

    def steps(self):
        """int32 [n_steps, 8] (nz, nm, nn, nk, variant, dtype, out_dtype, kernel), macs, bytes."""
        S = self.info()["n_steps"]
        dims = np.zeros((max(1, S), 8), np.int32)
        macs = np.zeros(max(1, S))
        byts = np.zeros(max(1, S))
        check(self._lib.lf_plan_steps(self._handle,
                                      dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      macs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      byts.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
              "lf_plan_steps")
        return dims[:S], macs[:S], byts[:S]

    def step_strides(self, step: int) -> np.ndarray:
        dims, _, _ = self.steps()
        n = int(dims[step, 0] + dims[step, 1] + dims[step, 2])
        out = np.zeros(max(1, n), np.int64)
        check(self._lib.lf_plan_step_strides(self._handle, step,
                                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
              "lf_plan_step_strides")
        return out[:n]

    def step_gather(self, step: int):
        """Operands of a batched step: [(stored_batched, qubits, strides)] for
        A and B (stored_batched -1 when the step is not batched)."""
        info = np.zeros(6, np.int32)
        q = [np.zeros(64, np.int32), np.zeros(64, np.int32)]
        s = [np.zeros(64, np.int64), np.zeros(64, np.int64)]
        i32 = ctypes.POINTER(ctypes.c_int32)
        i64 = ctypes.POINTER(ctypes.c_int64)
        check(self._lib.lf_plan_step_gather(self._handle, step, info.ctypes.data_as(i32),
                                            q[0].ctypes.data_as(i32), s[0].ctypes.data_as(i64),
                                            q[1].ctypes.data_as(i32), s[1].ctypes.data_as(i64)),
              "lf_plan_step_gather")
        return [(int(info[3 * w]), q[w][:info[3 * w + 1]].tolist(), s[w][:info[3 * w + 1]].tolist())
                for w in range(2)]

    # ------------------------------------------------------------- device
    def bind(self, workspace=None, stream=None):
        """Binds (allocating with torch if not given) the device workspace."""
        import torch
        need = int(self.info()["workspace_bytes"])
        if workspace is None:
            workspace = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
        base = workspace.data_ptr()
        pad = (-base) % 256
        check(self._lib.lf_plan_bind_workspace(self._handle, ctypes.c_void_p(base + pad),
                                               workspace.numel() - pad, _stream_ptr(stream)),
              "lf_plan_bind_workspace")
        self.workspace = workspace
        return self

    def new_amplitudes(self):
        import torch
        return torch.zeros((self.closed_bits.size, 1 << len(self.open_qubits)),
                           dtype=torch.complex128, device="cuda")

    def contract(self, begin: int, end: int, out=None, stream=None):
        """Adds slices [begin, end) into out (complex128 [n_batch, 2^l]); returns out."""
        if out is None:
            out = self.new_amplitudes()
        if out.dtype.__str__() != "torch.complex128" or not out.is_contiguous():
            raise ValueError("out must be a contiguous complex128 tensor")
        if out.numel() != self.closed_bits.size << len(self.open_qubits):
            raise ValueError("out has the wrong number of amplitudes")
        check(self._lib.lf_contract_slices(self._handle, int(begin), int(end),
                                           ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
              "lf_contract_slices")
        return out

    def overflow(self, clear: bool = False, stream=None) -> dict:
        """lf_plan_overflow: saturation state (synchronizes the stream)."""
        inf = _lib.lf_overflow_info()
        check(self._lib.lf_plan_overflow(self._handle, _stream_ptr(stream), ctypes.byref(inf),
                                         1 if clear else 0), "lf_plan_overflow")
        return {name: getattr(inf, name) for name, _ in inf._fields_ if name != "reserved"}

    def recalibrate(self, sigma: int, headroom_bits: int = 4, stream=None):
        check(self._lib.lf_plan_recalibrate(self._handle, int(sigma), int(headroom_bits),
                                            _stream_ptr(stream)), "lf_plan_recalibrate")

    def debug_scale_slice_leaf(self, wire_bit: int, value: int, log2_factor: int, stream=None):
        """Fault injection for saturation tests (lf_debug_scale_slice_leaf)."""
        check(self._lib.lf_debug_scale_slice_leaf(self._handle, int(wire_bit), int(value),
                                                  int(log2_factor), _stream_ptr(stream)),
              "lf_debug_scale_slice_leaf")

    def profile_steps(self, reps: int = 3, stream=None) -> np.ndarray:
        S = self.info()["n_steps"]
        out = np.zeros(max(1, S))
        check(self._lib.lf_profile_steps(self._handle, reps,
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         _stream_ptr(stream)), "lf_profile_steps")
        return out[:S]

    def time_kernel(self, kernel: int, reserve: int = 0):
        """Bracket every launch of contraction kernel `kernel` with HIP events
        in later stream-mode contractions (-1: off)."""
        check(self._lib.lf_plan_time_kernel(self._handle, int(kernel), int(reserve)),
              "lf_plan_time_kernel")

    def kernel_times(self):
        """(total_ms, launches, per_step_ms, per_step_launches) of the launches
        timed since the previous call."""
        S = self.info()["n_steps"]
        per_ms = np.zeros(max(1, S))
        per_n = np.zeros(max(1, S), np.int64)
        tot = ctypes.c_double()
        n = ctypes.c_int64()
        check(self._lib.lf_plan_kernel_times(self._handle, ctypes.byref(tot), ctypes.byref(n),
                                             per_ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                             per_n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
              "lf_plan_kernel_times")
        return tot.value, n.value, per_ms[:S], per_n[:S]

    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            self._lib.lf_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_network(circuit, open_qubits, closed_bits, **opts) -> Plan:
    return Plan(circuit, open_qubits, closed_bits, **opts)


def contract_slices(plan: Plan, begin: int, end: int, out_amps=None, stream=None):
    return plan.contract(begin, end, out_amps, stream)


def contract_batch(items, mode: str = "graph", lanes: int = 0, stream=None):
    """items: sequence of (plan, slice_begin, slice_end, out_amps tensor)."""
    arr = (_lib.lf_batch_item * max(1, len(items)))()
    for i, (plan, s0, s1, out) in enumerate(items):
        arr[i].plan = plan._handle.value
        arr[i].slice_begin = int(s0)
        arr[i].slice_end = int(s1)
        arr[i].out_amps = out.data_ptr()
    m = {"sequential": _lib.LF_BATCH_SEQUENTIAL, "graph": _lib.LF_BATCH_GRAPH}[mode]
    check(_lib.load().lf_contract_batch(arr, len(items), m, lanes, _stream_ptr(stream)),
          "lf_contract_batch")


def postselect_topk(amps, group_size: int, k: int, stream=None):
    """Top-k per group of `group_size` consecutive amplitudes (device tensors)."""
    import torch
    if amps.dtype != torch.complex128 or not amps.is_contiguous() or not amps.is_cuda:
        raise ValueError("amps must be a contiguous complex128 CUDA tensor")
    n = amps.numel()
    if group_size <= 0 or n % group_size:
        raise ValueError("amplitude count must be a multiple of group_size")
    g = n // group_size
    idx = torch.empty((g, k), dtype=torch.int64, device=amps.device)
    prob = torch.empty((g, k), dtype=torch.float64, device=amps.device)
    check(_lib.load().lf_postselect_topk(ctypes.c_void_p(amps.data_ptr()), g, group_size, k,
                                         ctypes.c_void_p(idx.data_ptr()),
                                         ctypes.c_void_p(prob.data_ptr()), _stream_ptr(stream)),
          "lf_postselect_topk")
    return idx, prob


def postselect_topk_noalloc(amps, group_size: int, k: int, out_idx, out_prob, stream=None):
    """lf_postselect_topk_noalloc: the same selection into caller-provided
    int64 / float64 device tensors of [n_groups, k], with no device
    allocation (fixed library scratch; overlapping calls on one GPU race)."""
    import torch
    if amps.dtype != torch.complex128 or not amps.is_contiguous() or not amps.is_cuda:
        raise ValueError("amps must be a contiguous complex128 CUDA tensor")
    n = amps.numel()
    if group_size <= 0 or n % group_size:
        raise ValueError("amplitude count must be a multiple of group_size")
    g = n // group_size
    for t, dt in ((out_idx, torch.int64), (out_prob, torch.float64)):
        if t.dtype != dt or not t.is_contiguous() or not t.is_cuda or t.numel() != g * k:
            raise ValueError("outputs must be contiguous CUDA tensors of n_groups * k elements")
    check(_lib.load().lf_postselect_topk_noalloc(ctypes.c_void_p(amps.data_ptr()), g, group_size, k,
                                                 ctypes.c_void_p(out_idx.data_ptr()),
                                                 ctypes.c_void_p(out_prob.data_ptr()),
                                                 _stream_ptr(stream)),
          "lf_postselect_topk_noalloc")
    return out_idx, out_prob


def probabilities_at(amps, idx, stream=None):
    """p (float64, each product and the sum rounded separately) of the
    amplitudes at positions idx (int64 device tensor) of the flat complex128
    device tensor amps; NaN for a position outside it."""
    import torch
    if amps.dtype != torch.complex128 or not amps.is_contiguous() or not amps.is_cuda:
        raise ValueError("amps must be a contiguous complex128 CUDA tensor")
    if idx.dtype != torch.int64 or not idx.is_contiguous() or not idx.is_cuda:
        raise ValueError("idx must be a contiguous int64 CUDA tensor")
    out = torch.empty(idx.numel(), dtype=torch.float64, device=amps.device)
    check(_lib.load().lf_probabilities_at(ctypes.c_void_p(amps.data_ptr()), amps.numel(),
                                          ctypes.c_void_p(idx.data_ptr()), idx.numel(),
                                          ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
          "lf_probabilities_at")
    return out


def mcmc_sample(amps, group_base, group_size: int, stride: int, n_chains: int, burn_in: int,
                thin: int, per_chain: int, seed: int, stream=None):
    """lf_mcmc_sample: Metropolis samples from p over the candidate set
    {group_base[g] + j * stride : j < group_size} of the flat complex128
    device tensor amps.  Returns (positions int64 [n_chains * per_chain],
    accepted moves int64 [n_chains])."""
    import torch
    if amps.dtype != torch.complex128 or not amps.is_contiguous() or not amps.is_cuda:
        raise ValueError("amps must be a contiguous complex128 CUDA tensor")
    if group_base.dtype != torch.int64 or not group_base.is_contiguous() or not group_base.is_cuda:
        raise ValueError("group_base must be a contiguous int64 CUDA tensor")
    out = torch.empty(n_chains * per_chain, dtype=torch.int64, device=amps.device)
    acc = torch.empty(n_chains, dtype=torch.int64, device=amps.device)
    check(_lib.load().lf_mcmc_sample(ctypes.c_void_p(amps.data_ptr()), amps.numel(),
                                     ctypes.c_void_p(group_base.data_ptr()), group_base.numel(),
                                     group_size, stride, n_chains, burn_in, thin, per_chain, seed,
                                     ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(acc.data_ptr()),
                                     _stream_ptr(stream)), "lf_mcmc_sample")
    return out, acc


def contract_pair(A, B, C, nz: int, nm: int, nn: int, nk: int, c_strides, scale: float = 1.0,
                  kernel: int = -1, stream=None):
    """lf_contract_pair on device tensors.  A, B, C are torch tensors holding
    (re, im) pairs: complex64 (float32 pairs) or complex-half (float16 pairs
    with a trailing dimension of 2); A and B share a dtype, or A is
    complex-half and B complex64."""
    import torch

    def dt(t):
        if t.dtype == torch.complex64:
            return _lib.LF_C64
        if t.dtype == torch.float16:
            return _lib.LF_CHALF
        raise ValueError("tensors must be complex64 or float16 pairs")

    if dt(A) != dt(B) and not (dt(A) == _lib.LF_CHALF and dt(B) == _lib.LF_C64):
        raise ValueError("A and B must share a dtype, or be complex-half A and complex64 B")
    st = np.ascontiguousarray(np.asarray(c_strides, np.int64))
    if st.size != nz + nm + nn:
        raise ValueError("need nz + nm + nn strides")
    check(_lib.load().lf_contract_pair(dt(A), dt(B), dt(C), kernel, ctypes.c_void_p(A.data_ptr()),
                                       ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(C.data_ptr()),
                                       nz, nm, nn, nk,
                                       st.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       float(scale), _stream_ptr(stream)), "lf_contract_pair")
    return C


def autotune_save(path: str) -> None:
    check(_lib.load().lf_autotune_save(path.encode()), "lf_autotune_save")


def autotune_load(path: str) -> None:
    check(_lib.load().lf_autotune_load(path.encode()), "lf_autotune_load")
