"""Random quantum circuits and closed bitstrings (inputs only).

Circuit family (Fig. 1 caption): every cycle applies a random single-qubit
gate from {sqrt X, sqrt Y, sqrt W} on every qubit, then a layer of two-qubit
gates on nearest-neighbour pairs.  The paper names neither the matrices nor
the two-qubit gate nor the coupling patterns; the readings used here are:

* sqrt P = exp(-i pi/4 P) for P in {X, Y, W}, W = (X + Y)/sqrt 2;
* the two-qubit gate is fSim(pi/2, pi/6);
* on an R x C grid (qubits numbered row-major over surviving sites) pattern
  A pairs (r,c)-(r,c+1) with c even, B with c odd, C pairs (r,c)-(r+1,c) with
  r even, D with r odd; cycle t uses pattern "ABCD"[t mod 4];
* cycle 0 draws each qubit's gate uniformly from the three, later cycles
  uniformly from the two that differ from that qubit's previous gate, qubits
  in ascending order, one PCG64 stream per circuit seed;
* the closed bitstrings of Methods A are uniform over the non-open qubits
  (duplicates rejected), from their own PCG64 stream.

A two-qubit matrix is indexed by 2*bit(q[0]) + bit(q[1]) on both sides.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

_S = 1.0 / math.sqrt(2.0)
_EIPI4 = complex(math.cos(math.pi / 4), math.sin(math.pi / 4))  # sqrt(i)

SQRT_X = np.array([[_S, -1j * _S], [-1j * _S, _S]], dtype=np.complex128)
SQRT_Y = np.array([[_S, -_S], [_S, _S]], dtype=np.complex128)
# W = (X + Y)/sqrt2 has off-diagonals e^{-i pi/4} (row 0) and e^{+i pi/4}
# (row 1); exp(-i pi/4 W) = (I - i W)/sqrt 2.
SQRT_W = np.array(
    [[_S, -1j * _S * _EIPI4.conjugate()], [-1j * _S * _EIPI4, _S]],
    dtype=np.complex128,
)
ONE_QUBIT_GATES = (SQRT_X, SQRT_Y, SQRT_W)
ONE_QUBIT_NAMES = ("sqrtX", "sqrtY", "sqrtW")


def fsim(theta: float, phi: float) -> np.ndarray:
    """fSim(theta, phi) in the basis |00>, |01>, |10>, |11>."""
    c, s = math.cos(theta), math.sin(theta)
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = 1.0
    m[1, 1] = c
    m[1, 2] = -1j * s
    m[2, 1] = -1j * s
    m[2, 2] = c
    m[3, 3] = complex(math.cos(phi), -math.sin(phi))
    return m


FSIM_DEFAULT = fsim(math.pi / 2, math.pi / 6)


@dataclasses.dataclass(frozen=True)
class Gate:
    qubits: Tuple[int, ...]      # (q,) or (q0, q1)
    matrix: np.ndarray           # 2x2 or 4x4 complex128, row = output
    cycle: int
    name: str = ""


@dataclasses.dataclass
class Circuit:
    n_qubits: int
    gates: List[Gate]
    rows: int = 0
    cols: int = 0
    removed_sites: Tuple[int, ...] = ()
    seed: int = 0

    @property
    def n_two_qubit(self) -> int:
        return sum(1 for g in self.gates if len(g.qubits) == 2)

    def to_arrays(self):
        """Flat arrays: nq[G], q[G,2], mat[G,16] complex128, cycle[G]."""
        g = len(self.gates)
        nq = np.zeros(g, np.int32)
        qs = np.full((g, 2), -1, np.int32)
        mats = np.zeros((g, 16), np.complex128)
        cyc = np.zeros(g, np.int32)
        for i, gate in enumerate(self.gates):
            nq[i] = len(gate.qubits)
            qs[i, : len(gate.qubits)] = gate.qubits
            flat = gate.matrix.reshape(-1)
            mats[i, : flat.size] = flat
            cyc[i] = gate.cycle
        return nq, qs, mats, cyc

    def save(self, path: str) -> None:
        nq, qs, mats, cyc = self.to_arrays()
        np.savez(path, n_qubits=self.n_qubits, nq=nq, q=qs, mat=mats, cycle=cyc,
                 rows=self.rows, cols=self.cols,
                 removed=np.array(self.removed_sites, np.int64), seed=self.seed)

    @staticmethod
    def load(path: str) -> "Circuit":
        d = np.load(path, allow_pickle=False)
        gates = []
        for i in range(d["nq"].shape[0]):
            k = int(d["nq"][i])
            dim = 2 ** k
            gates.append(Gate(tuple(int(x) for x in d["q"][i, :k]),
                              d["mat"][i, : dim * dim].reshape(dim, dim).copy(),
                              int(d["cycle"][i])))
        return Circuit(int(d["n_qubits"]), gates, int(d["rows"]), int(d["cols"]),
                       tuple(int(x) for x in d["removed"]), int(d["seed"]))


def grid_sites(rows: int, cols: int, removed: Sequence[int] = ()):
    """Map grid site r*cols+c -> qubit index (row-major over surviving sites)."""
    rem = set(int(x) for x in removed)
    site_to_q = {}
    q = 0
    for s in range(rows * cols):
        if s in rem:
            continue
        site_to_q[s] = q
        q += 1
    return site_to_q


def abcd_patterns(rows: int, cols: int, removed: Sequence[int] = ()):
    """Four couplings patterns A, B, C, D as lists of qubit pairs."""
    s2q = grid_sites(rows, cols, removed)
    pats = []
    for horiz, parity in ((True, 0), (True, 1), (False, 0), (False, 1)):
        pairs = []
        for r in range(rows):
            for c in range(cols):
                if horiz:
                    if c % 2 != parity or c + 1 >= cols:
                        continue
                    a, b = r * cols + c, r * cols + c + 1
                else:
                    if r % 2 != parity or r + 1 >= rows:
                        continue
                    a, b = r * cols + c, (r + 1) * cols + c
                if a in s2q and b in s2q:
                    pairs.append((s2q[a], s2q[b]))
        pats.append(pairs)
    return pats


def random_circuit(rows: int, cols: int, cycles: int, seed: int,
                   n_removed: int = 0, removal_seed: int = 0,
                   two_qubit: np.ndarray = FSIM_DEFAULT) -> Circuit:
    """Seeded random circuit on an R x C grid with `n_removed` sites dropped."""
    removed: Tuple[int, ...] = ()
    if n_removed:
        rr = np.random.Generator(np.random.PCG64(removal_seed))
        removed = tuple(sorted(int(x) for x in
                               rr.choice(rows * cols, size=n_removed, replace=False)))
    n = rows * cols - len(removed)
    pats = abcd_patterns(rows, cols, removed)
    rng = np.random.Generator(np.random.PCG64(seed))
    prev = [-1] * n
    gates: List[Gate] = []
    for t in range(cycles):
        for q in range(n):
            if prev[q] < 0:
                g = int(rng.integers(3))
            else:
                choices = [x for x in range(3) if x != prev[q]]
                g = choices[int(rng.integers(2))]
            prev[q] = g
            gates.append(Gate((q,), ONE_QUBIT_GATES[g].copy(), t, ONE_QUBIT_NAMES[g]))
        for (a, b) in pats[t % 4]:
            gates.append(Gate((a, b), two_qubit.copy(), t, "fsim"))
    return Circuit(n, gates, rows, cols, removed, seed)


def closed_bitstrings(n_qubits: int, open_qubits: Sequence[int], n_batch: int,
                      seed: int) -> np.ndarray:
    """`n_batch` distinct closed strings as full n-bit masks (open bits zero).

    Bit i of a uniform draw over 2^(n-l) goes to the i-th closed qubit in
    ascending order.
    """
    open_set = set(int(q) for q in open_qubits)
    closed = [q for q in range(n_qubits) if q not in open_set]
    nc = len(closed)
    if n_batch > (1 << nc):
        raise ValueError("more closed strings requested than exist")
    rng = np.random.Generator(np.random.PCG64(seed))
    seen = set()
    out = np.zeros(n_batch, dtype=np.uint64)
    i = 0
    while i < n_batch:
        v = int(rng.integers(0, 1 << nc, dtype=np.uint64)) if nc > 0 else 0
        if v in seen:
            continue
        seen.add(v)
        mask = 0
        for j, q in enumerate(closed):
            if (v >> j) & 1:
                mask |= 1 << q
        out[i] = mask
        i += 1
    return out


# The three workloads.  Sizes follow the paper's 30-qubit, 14-layer study
# (Fig. 3) and the 53-qubit, 20-cycle run with 10 open qubits (Methods D);
# the circuits are seeded stand-ins, not the Sycamore circuit files.
WORKLOADS = {
    "rqc12": dict(rows=3, cols=4, cycles=8, n_removed=0, n_open=12, n_batch=1,
                  n_sliced=0, max_log2=30),
    "rqc30": dict(rows=5, cols=6, cycles=14, n_removed=0, n_open=6, n_batch=256,
                  n_sliced=8, max_log2=26),
    "rqc53": dict(rows=6, cols=9, cycles=20, n_removed=1, n_open=10, n_batch=256,
                  n_sliced=-1, max_log2=28),
}
# The eight sliced wires (qubit, j) of the 30-qubit workload, wire t being
# bit t of the slice index (the set the planner picks for it at a
# 2^26-element cap); the slice prefix [0, 2^(8-D)) is the fraction 2^-D.
RQC30_SLICED_WIRES = [(19, 9), (20, 9), (21, 9), (14, 7), (22, 9), (24, 5), (15, 7), (25, 7)]
# candidate set of the 30-qubit sampling study: 2^20 closed strings (seeded)
# times the 64 values of the open qubits
XEB_MCMC_STRINGS = 1 << 20
XEB_MCMC_SEED = 2024
CIRCUIT_SEED = 2406
BITSTRING_SEED = 18889
REMOVAL_SEED = 53


def standard_workload(name: str, circuit_seed: int = CIRCUIT_SEED,
                      bitstring_seed: int = BITSTRING_SEED):
    """(circuit, open_qubits, closed_bits, spec) for a named workload.

    The open qubits are the last l qubits in row-major order.
    """
    spec = dict(WORKLOADS[name])
    circ = random_circuit(spec["rows"], spec["cols"], spec["cycles"], circuit_seed,
                          spec["n_removed"], REMOVAL_SEED)
    n = circ.n_qubits
    open_q = list(range(n - spec["n_open"], n))
    closed = closed_bitstrings(n, open_q, spec["n_batch"], bitstring_seed)
    return circ, np.array(open_q, np.int32), closed, spec


def random_complex(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """i.i.d. standard complex normal entries (kernel tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return ((re + 1j * im) / math.sqrt(2.0)).astype(dtype)


MIX_GRIDS = ((5, 6, 0), (6, 6, 0), (6, 7, 0), (7, 7, 0), (6, 9, 1))


def mixed_workload(n_circuits: int = 8, n_subtasks: int = 512, seed: int = 4096,
                   small: bool = False):
    """Uneven batch of sliced subtasks: `n_circuits` seeded circuits (grids
    5x6 .. 6x9-1, 12..20 cycles, 6..10 open qubits, 16..256 closed strings,
    intermediate cap 2^24..2^27) and `n_subtasks` (circuit, slice draw) pairs;
    the slice draw is reduced modulo the plan's slice count by the caller.
    `small` uses 4x4..5x5 grids, 8..12 cycles and caps 2^14..2^16 (tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    circuits = []
    for i in range(n_circuits):
        if small:
            r, c, rem = [(4, 4, 0), (4, 5, 0), (5, 5, 0)][int(rng.integers(3))]
            cyc = int(rng.integers(8, 13))
            n_open = int(rng.integers(3, 6))
            nb = int(rng.choice([4, 16]))
            cap = int(rng.integers(14, 17))
        else:
            r, c, rem = MIX_GRIDS[int(rng.integers(len(MIX_GRIDS)))]
            cyc = int(rng.integers(12, 21))
            n_open = int(rng.integers(6, 11))
            nb = int(rng.choice([16, 64, 256]))
            cap = int(rng.integers(24, 28))
        circ = random_circuit(r, c, cyc, int(rng.integers(1, 1 << 30)), rem,
                              int(rng.integers(1, 1 << 30)))
        n = circ.n_qubits
        openq = list(range(n - n_open, n))
        cb = closed_bitstrings(n, openq, nb, int(rng.integers(1, 1 << 30)))
        circuits.append(dict(circuit=circ, open_qubits=np.array(openq, np.int32),
                             closed_bits=cb, max_log2=cap, grid=(r, c, rem), cycles=cyc))
    subtasks = [(int(rng.integers(n_circuits)), int(rng.integers(0, 1 << 62)))
                for _ in range(n_subtasks)]
    return circuits, subtasks
