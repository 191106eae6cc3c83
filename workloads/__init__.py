"""Seeded synthetic inputs shared by the product path and the oracle.

This package generates inputs only: random circuits of the family the paper
samples (Fig. 1: random single-qubit gates from {sqrt X, sqrt Y, sqrt W}
followed by two-qubit gates on nearest neighbours), the closed bitstrings of
Methods A, and i.i.d. complex tensors for kernel tests.  It holds none of the
contraction, slicing or post-selection arithmetic.
"""

from .circuits import (  # noqa: F401
    Circuit,
    Gate,
    SQRT_X,
    SQRT_Y,
    SQRT_W,
    fsim,
    FSIM_DEFAULT,
    CIRCUIT_SEED,
    BITSTRING_SEED,
    grid_sites,
    abcd_patterns,
    random_circuit,
    closed_bitstrings,
    standard_workload,
    WORKLOADS,
    random_complex,
    mixed_workload,
    RQC30_SLICED_WIRES,
    XEB_MCMC_STRINGS,
    XEB_MCMC_SEED,
)
