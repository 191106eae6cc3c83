"""Oracle O1/O2 (test infrastructure only): complex128 state vector.

phi(s) = <s|U|0^n> for the circuit U of Fig. 1 (Methods A), computed gate
by gate by oracle/sv.c.  With projectors on wires it gives the value of a
sliced sub-network (Methods C, slicing identity) or of a prefix of slices
that fixes D wires (the fraction f = 2^-D of Methods A and Eq. 3).
"""

from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence, Tuple

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.sv_run_circuit.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, P,
                                       ctypes.c_int, P, P, P, ctypes.c_int]
        lib.sv_run_circuit.restype = ctypes.c_int
        lib.sv_apply_1q.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
        lib.sv_apply_2q.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        lib.sv_zero_state.argtypes = [P, ctypes.c_int]
        lib.sv_project.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.sv_gather.argtypes = [P, ctypes.c_int64, P, P]
        lib.sv_norm2.argtypes = [P, ctypes.c_int]
        lib.sv_norm2.restype = ctypes.c_double
        lib.sv_moments.argtypes = [P, ctypes.c_int, P, P]
        lib.sv_sample_sorted.argtypes = [P, ctypes.c_int, ctypes.c_int64, P, P]
        lib.sv_probs.argtypes = [P, ctypes.c_int, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def apply_1q(psi: np.ndarray, q: int, g: np.ndarray) -> None:
    n = int(np.log2(psi.size))
    g = np.ascontiguousarray(g, np.complex128)
    _load().sv_apply_1q(_ptr(psi), n, q, _ptr(g))


def apply_2q(psi: np.ndarray, q0: int, q1: int, g: np.ndarray) -> None:
    n = int(np.log2(psi.size))
    g = np.ascontiguousarray(g, np.complex128)
    _load().sv_apply_2q(_ptr(psi), n, q0, q1, _ptr(g))


def run(circuit, projectors: Sequence[Tuple[int, int, int]] = (),
        stop_after_gate: int = -1, out: Optional[np.ndarray] = None) -> np.ndarray:
    """State after the circuit (or its first `stop_after_gate` gates).

    projectors: (qubit, j, v) inserts |v><v| on wire (qubit, j), the point
    immediately before the j-th two-qubit gate on that qubit.
    """
    n = circuit.n_qubits
    nq, qs, mats, _ = circuit.to_arrays()
    nq = np.ascontiguousarray(nq)
    qs = np.ascontiguousarray(qs.reshape(-1))
    mats = np.ascontiguousarray(mats.reshape(-1))
    pq = np.array([p[0] for p in projectors], np.int32)
    pj = np.array([p[1] for p in projectors], np.int32)
    pv = np.array([p[2] for p in projectors], np.int32)
    if out is None:
        out = np.empty(1 << n, np.complex128)
    rc = _load().sv_run_circuit(_ptr(out), n, len(circuit.gates), _ptr(nq), _ptr(qs),
                                _ptr(mats), len(projectors), _ptr(pq), _ptr(pj),
                                _ptr(pv), stop_after_gate)
    if rc != 0:
        raise RuntimeError(f"sv_run_circuit failed: {rc}")
    return out


def group_indices(n_qubits: int, open_qubits: Sequence[int],
                  closed_bits: Sequence[int]) -> np.ndarray:
    """Basis indices s(b, j): closed string c_b with bit open_qubits[i] = bit i of j."""
    l = len(open_qubits)
    j = np.arange(1 << l, dtype=np.uint64)
    spread = np.zeros(1 << l, dtype=np.uint64)
    for i, q in enumerate(open_qubits):
        spread |= ((j >> np.uint64(i)) & np.uint64(1)) << np.uint64(q)
    cb = np.asarray(closed_bits, dtype=np.uint64)
    return (cb[:, None] | spread[None, :]).reshape(-1)


def gather(psi: np.ndarray, idx: np.ndarray) -> np.ndarray:
    idx = np.ascontiguousarray(idx, np.uint64)
    out = np.empty(idx.size, np.complex128)
    _load().sv_gather(_ptr(psi), idx.size, _ptr(idx), _ptr(out))
    return out


def group_amplitudes(circuit, open_qubits, closed_bits,
                     projectors: Sequence[Tuple[int, int, int]] = ()) -> np.ndarray:
    """A[b, j] = phi(s(b, j)) (Methods A), optionally with wire projectors."""
    psi = run(circuit, projectors)
    idx = group_indices(circuit.n_qubits, open_qubits, closed_bits)
    a = gather(psi, idx).reshape(len(closed_bits), 1 << len(open_qubits))
    del psi
    return a


def norm2(psi: np.ndarray) -> float:
    n = int(np.log2(psi.size))
    return float(_load().sv_norm2(_ptr(psi), n))


def moments(psi: np.ndarray) -> Tuple[float, float]:
    n = int(np.log2(psi.size))
    m2 = np.zeros(1)
    m3 = np.zeros(1)
    _load().sv_moments(_ptr(psi), n, _ptr(m2), _ptr(m3))
    return float(m2[0]), float(m3[0])


def probs(psi: np.ndarray) -> np.ndarray:
    n = int(np.log2(psi.size))
    p = np.empty(psi.size, np.float64)
    _load().sv_probs(_ptr(psi), n, _ptr(p))
    return p


def sample_exact(psi: np.ndarray, m: int, seed: int) -> np.ndarray:
    """m samples from |psi|^2 by inversion of sorted uniforms."""
    n = int(np.log2(psi.size))
    total = norm2(psi)
    rng = np.random.Generator(np.random.PCG64(seed))
    u = np.sort(rng.random(m) * total)
    out = np.empty(m, np.uint64)
    _load().sv_sample_sorted(_ptr(psi), n, m, _ptr(u), _ptr(out))
    return out
