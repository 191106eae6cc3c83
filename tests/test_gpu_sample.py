"""The Metropolis sampling baseline of Methods B (lf_mcmc_sample), through
the C ABI, on small candidate sets whose distribution is known: the sample
frequencies follow p restricted to the candidates, normalised (total
variation distance against the exact distribution, which shrinks like
1/sqrt(samples)); candidates of zero probability are never visited after
burn-in; a seed reproduces its samples bit for bit; acceptance counts match
the samples' moves."""

import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = [pytest.mark.gpu]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_18889_amd as lf
    from paper_2406_18889_amd import _lib
    _lib.load()
    return lf


def test_mcmc_samples_follow_p_over_candidates(lf):
    a = wl.random_complex(64, seed=5)
    a[[2, 18, 34]] = 0.0                               # zero-probability candidates
    p = (a.real ** 2 + a.imag ** 2)
    base = np.array([0, 16, 32, 48], np.int64)         # 4 groups of 8 strings, stride 2
    cand = (base[:, None] + 2 * np.arange(8)[None, :]).reshape(-1)
    assert np.unique(cand).size == cand.size
    target = p[cand] / p[cand].sum()
    d = torch.from_numpy(a).cuda()
    chains, per = 4096, 64
    pos, acc = lf.mcmc_sample(d, torch.from_numpy(base).cuda(), 8, 2, chains, 64, 8, per, seed=7)
    pos2, acc2 = lf.mcmc_sample(d, torch.from_numpy(base).cuda(), 8, 2, chains, 64, 8, per, seed=7)
    pos3, _ = lf.mcmc_sample(d, torch.from_numpy(base).cuda(), 8, 2, chains, 64, 8, per, seed=8)
    torch.cuda.synchronize()
    assert torch.equal(pos, pos2) and torch.equal(acc, acc2)
    assert not torch.equal(pos, pos3)
    x = pos.cpu().numpy()
    assert np.isin(x, cand).all()
    freq = np.array([(x == c).sum() for c in cand], np.float64) / x.size
    tv = 0.5 * np.abs(freq - target).sum()
    sys.stdout.write(f"mcmc: total variation {tv:.4f} over {x.size} samples, acceptance "
                     f"{acc.sum().item() / (chains * (64 + per * 8)):.3f}\n")
    assert tv < 0.02
    assert freq[target == 0].sum() == 0
    # every chain's samples change only by accepted moves
    moves = (np.diff(x.reshape(chains, per), axis=1) != 0).sum(axis=1)
    assert (moves <= acc.cpu().numpy()).all()
