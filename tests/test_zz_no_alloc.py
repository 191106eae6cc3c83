"""The allocation-free top-k entry point (lf_postselect_topk_noalloc)
against the allocating one (lf_postselect_topk), through the C ABI: the same
indices and probabilities bit for bit, on two calls in a row (the second on a
smaller input, so stale scratch contents from the first would show), on both
implementations (one workgroup per group, and the radix path whose scratch
is the library's fixed device array); sizes beyond the fixed scratch are
rejected before any work."""

import ctypes
import sys

import numpy as np
import pytest

import workloads as wl

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


def _both(lf, a, gs, k):
    from paper_2406_18889_amd import api
    d = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g = d.numel() // gs
    i_ref, p_ref = lf.postselect_topk(d, gs, k)
    oi = torch.full((g, k), -7, dtype=torch.int64, device="cuda")
    op = torch.full((g, k), -7.0, dtype=torch.float64, device="cuda")
    api.postselect_topk_noalloc(d, gs, k, oi, op)
    torch.cuda.synchronize()
    return i_ref, p_ref, oi, op


@pytest.mark.parametrize("first,second", [
    ((1 << 20, 1 << 20, 40_000), (300_001, 300_001, 1500)),     # radix path, then smaller
    ((3 << 17, 1 << 17, 5000), (1 << 16, 1 << 16, 1025)),      # three groups, then one
    ((256 * 1024, 1024, 4), (64 * 1024, 1024, 1)),             # one workgroup per group
])
def test_noalloc_matches_allocating_entry_point(lf, first, second):
    for j, (n, gs, k) in enumerate((first, second)):
        a = wl.random_complex(n, seed=1000 + n + k)
        a[3::113] = a[1]  # ties
        _say(f"noalloc call {j}: n={n} group={gs} k={k}")
        i_ref, p_ref, oi, op = _both(lf, a, gs, k)
        assert torch.equal(oi, i_ref)
        assert torch.equal(op.view(torch.int64), p_ref.view(torch.int64))


def test_noalloc_rejects_k_beyond_fixed_scratch(lf):
    from paper_2406_18889_amd import _lib
    lib = _lib.load()
    n = 4_300_000
    d = torch.zeros(n, dtype=torch.complex128, device="cuda")
    oi = torch.empty(n, dtype=torch.int64, device="cuda")
    op = torch.empty(n, dtype=torch.float64, device="cuda")
    st = lib.lf_postselect_topk_noalloc(ctypes.c_void_p(d.data_ptr()), 1, n, n,
                                        ctypes.c_void_p(oi.data_ptr()), ctypes.c_void_p(op.data_ptr()),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.LF_INVALID_ARGUMENT
    assert b"scratch" in lib.lf_last_error()
