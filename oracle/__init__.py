"""The oracle: plain, slow, obviously correct CPU reference for the sliced
tensor-network amplitude path and its top-k post-selection.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check in the entry
module and the CPU-baseline leg of the benchmark may import or run anything
here; the product library never does, and shares no code with it.

Modules:
  sv    complex128 state vector with optional wire projectors (C, OpenMP)
  tn    complex128 contraction of one sliced sub-network (numpy)
  topk  top-k selection, XEB (Eq. 1) and its Porter-Thomas expectations
  mlp   float64 reference of the cost-model network (forward, backward)

The independent recount of per-step work from an exported plan (multiply-adds
and the largest tensor, from the oracle's own network) is written out in the
CPU tests of the boundary, next to the plan it checks.
"""
