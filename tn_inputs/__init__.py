"""Seeded synthetic inputs shared by the oracle-side tests and the GPU-side tests.

This package holds no contraction arithmetic. It builds tensor networks in the
form of the problem statement (Sec. 2: tensors T_v, ordered index tuples t_v,
index dimensions |D(e)|, optional open output indices) and contraction trees as
SSA pairs (the l(v), r(v) tuples of Sec. 2, leaves numbered first). The tree is
an input to both the oracle and the GPU library: each side recomputes its own
incidence sets, widths and costs from it.

Modules:
  network   -- the Network container and validation of its shape
  circuits  -- random grid circuits (transition amplitude, eq. trans-amp)
  graphs    -- random 3-regular graph networks with iid complex Gaussian tensors
  greedy    -- Hyper-Greedy tree sampler (Sec. 3.4, eqs. greedy-cost-function
               and greedy-boltzmann-factor)
  slicing   -- greedy choice of sliced indices (Sec. 4.7.1, Slicing)
  configs   -- the five benchmark workloads with their seeds
"""

from .network import Network, Tree  # noqa: F401
