"""Sliced tensor-network amplitudes of random quantum circuits and top-k
post-selection (arXiv 2406.18889) on MI355X: a C-ABI HIP library
(include/leapfrog.h) with a thin Python binding.
"""

from .api import (Plan, autotune_load, autotune_save, build_network,  # noqa: F401
                  contract_batch, contract_pair, contract_slices, postselect_topk,
                  probabilities_at, mcmc_sample)
from ._lib import LeapfrogError  # noqa: F401
