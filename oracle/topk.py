"""Oracle O4/O5 (test infrastructure only): top-k post-selection and XEB.

Top-k (Methods A): from the candidate sequence, keep the k strings with the
largest p(s) = |phi(s)|^2.  Readings fixed here: p is re*re + im*im in
float64 with every product and the sum rounded separately (no fused
multiply-add), and ties are broken by the smaller position j inside the
group, so the selection is unique.

XEB (Eq. 1): F = N/|S| * sum_{s in S} q(s) - 1 with N = 2^n and q the exact
probability.  Expected top-k XEB under Porter-Thomas (Eq. 2, Appendix A):
ln(|S~|/k); the exact finite-size value for i.i.d. Exp(1) values Nq is
H_|S~| - H_k (harmonic numbers), which tends to the logarithm.
"""

from __future__ import annotations

import math

import numpy as np


def probabilities(amps: np.ndarray) -> np.ndarray:
    a = np.asarray(amps, dtype=np.complex128)
    re = np.ascontiguousarray(a.real)
    im = np.ascontiguousarray(a.imag)
    rr = re * re
    ii = im * im
    return rr + ii


def topk(amps: np.ndarray, group_size: int, k: int):
    """Per group of `group_size` consecutive entries: (idx[g, k], p[g, k]).

    Order: p descending, then index ascending.  idx is the position inside
    the group.
    """
    p = probabilities(np.asarray(amps).reshape(-1))
    if p.size % group_size:
        raise ValueError("size not a multiple of group_size")
    g = p.size // group_size
    if not (0 < k <= group_size):
        raise ValueError("k out of range")
    p = p.reshape(g, group_size)
    idx = np.empty((g, k), np.int64)
    val = np.empty((g, k), np.float64)
    j = np.arange(group_size)
    for r in range(g):
        order = np.lexsort((j, -p[r]))[:k]
        idx[r] = order
        val[r] = p[r, order]
    return idx, val


def topk_bruteforce(amps: np.ndarray, group_size: int, k: int):
    """Same selection by a full Python sort of (-p, j) tuples (pin for topk)."""
    p = probabilities(np.asarray(amps).reshape(-1)).reshape(-1, group_size)
    idx = []
    val = []
    for r in range(p.shape[0]):
        keyed = sorted(((-float(p[r, j]), j) for j in range(group_size)))[:k]
        idx.append([j for _, j in keyed])
        val.append([-v for v, _ in keyed])
    return np.array(idx, np.int64), np.array(val, np.float64)


def xeb(q_of_samples: np.ndarray, n_qubits: int) -> float:
    """Eq. 1 with the exact probabilities q of the selected samples."""
    q = np.asarray(q_of_samples, dtype=np.float64)
    return float((2.0 ** n_qubits) * q.mean() - 1.0)


def harmonic(n: int) -> float:
    if n <= 0:
        return 0.0
    if n < 10_000_000:
        return float(np.sum(1.0 / np.arange(1, n + 1, dtype=np.float64)))
    g = 0.5772156649015329
    return math.log(n) + g + 1.0 / (2 * n) - 1.0 / (12.0 * n * n)


def expected_topk_xeb(n_candidates: int, k: int) -> float:
    """E[XEB] of the top k of n_candidates i.i.d. Exp(1) values of Nq."""
    return harmonic(n_candidates) - harmonic(k)


def porter_thomas_topk_xeb(n_candidates: int, k: int) -> float:
    """Eq. 2: ln(|S~| / k)."""
    return math.log(n_candidates / k)
