"""Top-k post-selection at any size (Methods A: the k largest p over all of
S~ or per group), through the C ABI, bit-exact against the oracle's lexsort
selection (order p descending, then position ascending; p = re*re + im*im in
float64 without fused rounding) on the same amplitudes.

Inputs are i.i.d. complex normal amplitudes (Porter-Thomas p), with planted
ties: duplicated amplitudes, amplitudes of equal modulus and different phase
(equal p up to rounding only when the products round alike), quantised
amplitudes (many exact ties at the selection threshold), all-equal and zero
groups; sizes that are not powers of two and k up to the whole group.
"""

import sys

import numpy as np
import pytest

import workloads as wl
from oracle import topk

pytestmark = [pytest.mark.gpu]

torch = pytest.importorskip("torch")


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


def _check(lf, a, gs, k, label):
    _say(f"select {label}: n={a.size} group={gs} k={k}")
    d = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    idx, prob = lf.postselect_topk(d, gs, k)
    torch.cuda.synchronize()
    i_ref, p_ref = topk.topk(a, gs, k)
    got_i, got_p = idx.cpu().numpy(), prob.cpu().numpy()
    assert np.array_equal(got_p.view(np.uint64), p_ref.view(np.uint64)), label
    assert np.array_equal(got_i, i_ref), label


@pytest.mark.parametrize("n,k", [(1 << 20, 1), (1 << 20, 100), (1 << 20, 1025), (1 << 20, 4096),
                                 (1 << 20, 1 << 15), (100_003, 777), (70_001, 70_001),
                                 (1 << 17, 1 << 17)])
def test_global_select_random(lf, n, k):
    a = wl.random_complex(n, seed=n + k)
    _check(lf, a, n, k, "random")


def test_global_select_planted_ties(lf):
    n, k = 1 << 20, 5000
    a = wl.random_complex(n, seed=7)
    a[5::97] = a[3]                       # exact duplicates
    a[11::101] = a[2] * 1j                # equal modulus, rotated by i (same p exactly)
    _check(lf, a, n, k, "duplicates")


def test_global_select_quantised_ties(lf):
    # amplitudes on a coarse grid: thousands of exact ties at every p, so
    # the threshold class is cut by position
    n = 1 << 19
    rng = np.random.Generator(np.random.PCG64(11))
    a = (rng.integers(-3, 4, n) + 1j * rng.integers(-3, 4, n)).astype(np.complex128) / 8
    for k in (1, 3000, 40_000, n - 1):
        _check(lf, a, n, k, "quantised")


def test_select_degenerate_groups(lf):
    n = 1 << 18
    a = np.full(n, 0.25 + 0.5j, np.complex128)
    _check(lf, a, n, 2000, "all equal")
    z = np.zeros(n, np.complex128)
    _check(lf, z, n, 3000, "all zero")
    z[n - 1] = 1e-300                      # one tiny positive p among zeros (p underflows to 0)
    z[17] = 1e-150
    _check(lf, z, n, 2, "tiny")


@pytest.mark.parametrize("groups,gs,k", [(3, 1 << 17, 3000), (5, 2048, 2000), (7, 70_000, 1),
                                         (2, 1 << 16, 1024), (4, 1 << 16, 1025)])
def test_select_per_group(lf, groups, gs, k):
    a = wl.random_complex(groups * gs, seed=groups * 1000 + k)
    a[::7] = a[1]
    _check(lf, a, gs, k, "per group")


def test_select_small_and_radix_paths_agree(lf):
    # the same selection through both implementations (group_size 2^16:
    # one workgroup per group; k 1025 selects by radix over the same data)
    gs = 1 << 16
    a = wl.random_complex(gs, seed=99)
    d = torch.from_numpy(a).cuda()
    i1, p1 = lf.postselect_topk(d, gs, 1024)
    i2, p2 = lf.postselect_topk(d, gs, 1025)
    torch.cuda.synchronize()
    assert torch.equal(i1[0], i2[0, :1024]) and torch.equal(p1[0], p2[0, :1024])


def test_probabilities_at(lf):
    a = wl.random_complex(5000, seed=3)
    d = torch.from_numpy(a).cuda()
    idx = torch.tensor([0, 4999, 17, -1, 5000, 17], dtype=torch.int64, device="cuda")
    q = lf.probabilities_at(d, idx).cpu().numpy()
    ref = topk.probabilities(a[[0, 4999, 17]])
    assert np.array_equal(q[[0, 1, 2]], ref) and q[5] == ref[2]
    assert np.isnan(q[3]) and np.isnan(q[4])
