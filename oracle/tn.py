"""Oracle O3 (test infrastructure only): plain complex128 tensor-network
contraction of one sliced sub-network.

Follows Methods A and C: the circuit becomes a network whose tensors are the
gates, the closed output qubits are capped with the bits of the sampled
strings (one batch label "b" shared by every cap, so each closed string is a
separate network that shares all other tensors), the open output qubits stay
as legs, and slicing fixes the value of chosen wires; the sliced network is
contracted pairwise, each pair by a transpose and a batched matrix product.
The value of a network does not depend on the order of its pairwise
contractions, so a tree supplied by the caller only sets memory and time.

Leaf identity (shared with the library only as a naming convention): the
k-th two-qubit gate of the circuit, with the single-qubit gates that follow it
on its two qubits up to their next two-qubit gate (or the end) folded onto its
output legs, and, where it is a qubit's first two-qubit gate, that qubit's
earlier single-qubit gates applied to |0> folded onto its input leg, is leaf
k.  A qubit with no two-qubit gate is leaf n2q + q.  Wire (q, j), j >= 1, is
the leg between the (j-1)-th and j-th two-qubit gates on q.
"""

from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

Label = object


def canonical_network(circuit, open_qubits: Sequence[int], closed_bits: Sequence[int]):
    """Leaves {id: (labels, data)} of the network, in complex128."""
    n = circuit.n_qubits
    open_set = set(int(q) for q in open_qubits)
    cb = np.asarray(closed_bits, dtype=np.uint64)
    n2q_total = sum(1 for g in circuit.gates if len(g.qubits) == 2)
    eye = np.eye(2, dtype=np.complex128)
    zero = np.array([1.0, 0.0], dtype=np.complex128)

    pending = [eye.copy() for _ in range(n)]
    count = [0] * n
    last_leaf: List[Optional[int]] = [None] * n
    leaves: Dict[int, Tuple[List[Label], np.ndarray]] = {}

    def attach_out(leaf_id: int, q: int, m: np.ndarray) -> None:
        labels, data = leaves[leaf_id]
        ax = labels.index(("out", q))
        data = np.moveaxis(np.tensordot(m, data, axes=([1], [ax])), 0, ax)
        leaves[leaf_id] = (labels, data)

    k = 0
    for g in circuit.gates:
        if len(g.qubits) == 1:
            q = g.qubits[0]
            pending[q] = g.matrix @ pending[q]
            continue
        qa, qb = g.qubits
        for q in (qa, qb):
            if last_leaf[q] is not None:
                attach_out(last_leaf[q], q, pending[q])
                pending[q] = eye.copy()
        # axes: out_a, out_b, in_a, in_b
        data = g.matrix.reshape(2, 2, 2, 2).astype(np.complex128)
        labels: List[Label] = [("out", qa), ("out", qb), ("in", qa), ("in", qb)]
        for q in (qa, qb):
            ax = labels.index(("in", q))
            if count[q] == 0:
                v = pending[q] @ zero
                data = np.tensordot(data, v, axes=([ax], [0]))
                labels.pop(ax)
                pending[q] = eye.copy()
            else:
                labels[ax] = ("w", q, count[q])
        leaves[k] = (labels, data)
        # the previous leaf's out leg on q becomes wire (q, count[q])
        for q in (qa, qb):
            if last_leaf[q] is not None:
                pl, pd = leaves[last_leaf[q]]
                pl = list(pl)
                pl[pl.index(("out", q))] = ("w", q, count[q])
                leaves[last_leaf[q]] = (pl, pd)
            last_leaf[q] = k
            count[q] += 1
        k += 1
    assert k == n2q_total

    for q in range(n):
        if last_leaf[q] is not None:
            attach_out(last_leaf[q], q, pending[q])
        else:
            v = pending[q] @ zero
            leaves[n2q_total + q] = ([("out", q)], v)
            last_leaf[q] = n2q_total + q

    # output legs: open -> ("o", q); closed -> capped with <c_b(q)|, label "b"
    for q in range(n):
        lid = last_leaf[q]
        labels, data = leaves[lid]
        labels = list(labels)
        ax = labels.index(("out", q))
        if q in open_set:
            labels[ax] = ("o", q)
        else:
            bits = ((cb >> np.uint64(q)) & np.uint64(1)).astype(np.int64)
            if "b" in labels:
                bax = labels.index("b")
                data = np.moveaxis(data, (bax, ax), (0, 1))
                rest = [x for i, x in enumerate(labels) if i not in (bax, ax)]
                data = data[np.arange(len(cb)), bits]
                labels = ["b"] + rest
            else:
                data = np.moveaxis(np.take(data, bits, axis=ax), ax, 0)
                labels = ["b"] + [x for i, x in enumerate(labels) if i != ax]
        leaves[lid] = (labels, data)
    return leaves


def wire_list(leaves) -> List[Tuple[int, int]]:
    """All internal wires (q, j) present in the network."""
    ws = set()
    for labels, _ in leaves.values():
        for x in labels:
            if isinstance(x, tuple) and x[0] == "w":
                ws.add((x[1], x[2]))
    return sorted(ws)


def fix_wires(leaves, wires: Sequence[Tuple[int, int]], values: Sequence[int]):
    """Sliced sub-network: wire (q, j) fixed to value v in both tensors it joins."""
    out = {}
    fixed = {("w", int(q), int(j)): int(v) for (q, j), v in zip(wires, values)}
    seen = {x: 0 for x in fixed}
    for lid, (labels, data) in leaves.items():
        labels = list(labels)
        for lab, v in fixed.items():
            if lab in labels:
                ax = labels.index(lab)
                data = np.take(data, v, axis=ax)
                labels.pop(ax)
                seen[lab] += 1
        out[lid] = (labels, data)
    for lab, c in seen.items():
        if c != 2:
            raise ValueError(f"wire {lab} joins {c} tensors, expected 2")
    return out


def contract_pair(la, A, lb, B, keep):
    """Pairwise contraction; labels in both are summed unless kept (batch)."""
    common = [x for x in la if x in lb]
    batch = [x for x in common if x in keep]
    summed = [x for x in common if x not in keep]
    fa = [x for x in la if x not in common]
    fb = [x for x in lb if x not in common]
    da = dict(zip(la, A.shape))
    db = dict(zip(lb, B.shape))
    pa = [la.index(x) for x in batch + fa + summed]
    pb = [lb.index(x) for x in batch + summed + fb]
    zb = int(np.prod([da[x] for x in batch], dtype=np.int64))
    m = int(np.prod([da[x] for x in fa], dtype=np.int64))
    kk = int(np.prod([da[x] for x in summed], dtype=np.int64))
    nn = int(np.prod([db[x] for x in fb], dtype=np.int64))
    A2 = np.ascontiguousarray(np.transpose(A, pa)).reshape(zb, m, kk)
    B2 = np.ascontiguousarray(np.transpose(B, pb)).reshape(zb, kk, nn)
    C = np.matmul(A2, B2)
    shape = [da[x] for x in batch] + [da[x] for x in fa] + [db[x] for x in fb]
    return batch + fa + fb, C.reshape(shape)


def _keep_labels(open_qubits):
    return {"b"} | {("o", int(q)) for q in open_qubits}


def contract_tree(leaves, steps: Sequence[Tuple[int, int]], id_base: int, keep):
    """Contract following steps (a, b); intermediate i has id id_base + i.

    Checks that the steps form one full binary tree over exactly the leaves.
    """
    nodes = dict(leaves)
    used = set()
    for i, (a, b) in enumerate(steps):
        a, b = int(a), int(b)
        if a in used or b in used or a not in nodes or b not in nodes or a == b:
            raise ValueError(f"step {i}: invalid operands {a}, {b}")
        used.add(a)
        used.add(b)
        la, A = nodes.pop(a)
        lb, B = nodes.pop(b)
        nodes[id_base + i] = contract_pair(la, A, lb, B, keep)
    if len(nodes) != 1:
        raise ValueError(f"tree leaves {len(nodes)} nodes uncontracted")
    return next(iter(nodes.values()))


def greedy_steps(leaves, keep) -> Tuple[List[Tuple[int, int]], int]:
    """The oracle's own simple order for small networks: repeatedly contract
    the pair with the smallest result among pairs sharing a label."""
    shapes = {lid: (list(l), dict(zip(l, d.shape))) for lid, (l, d) in leaves.items()}
    id_base = max(leaves) + 1
    steps = []
    nxt = id_base
    while len(shapes) > 1:
        best = None
        ids = sorted(shapes)
        for i, a in enumerate(ids):
            la, da = shapes[a]
            for b in ids[i + 1:]:
                lb, db = shapes[b]
                common = [x for x in la if x in lb]
                out = [x for x in la if x not in lb or x in keep] + \
                      [x for x in lb if x not in la]
                size = 1
                for x in out:
                    size *= da.get(x, db.get(x, 1))
                key = (0 if common else 1, size)
                if best is None or key < best[1]:
                    best = ((a, b), key)
        (a, b) = best[0]
        la, da = shapes.pop(a)
        lb, db = shapes.pop(b)
        out = [x for x in la if x not in lb or x in keep] + [x for x in lb if x not in la]
        dd = dict(da)
        dd.update(db)
        shapes[nxt] = (out, {x: dd[x] for x in out})
        steps.append((a, b))
        nxt += 1
    return steps, id_base


def amplitudes(circuit, open_qubits, closed_bits, sliced_wires=(), slice_values=(),
               steps=None, id_base=None) -> np.ndarray:
    """A_sigma[b, j] of one sliced sub-network (all wires free if none fixed)."""
    leaves = canonical_network(circuit, open_qubits, closed_bits)
    if sliced_wires:
        leaves = fix_wires(leaves, sliced_wires, slice_values)
    keep = _keep_labels(open_qubits)
    if steps is None:
        steps, id_base = greedy_steps(leaves, keep)
    labels, data = contract_tree(leaves, steps, id_base, keep)
    B = len(closed_bits)
    order = []
    if "b" in labels:
        order.append(labels.index("b"))
    for q in reversed(list(open_qubits)):
        order.append(labels.index(("o", int(q))))
    if len(order) != len(labels):
        raise ValueError("root carries unexpected labels")
    res = np.transpose(data, order).reshape(-1, 1 << len(open_qubits))
    if res.shape[0] == 1 and B > 1:
        res = np.repeat(res, B, axis=0)
    return res


def slice_values(sigma: int, n_sliced: int) -> List[int]:
    """Sliced wire t takes bit t of the slice index."""
    return [(sigma >> t) & 1 for t in range(n_sliced)]
