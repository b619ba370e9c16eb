"""MI355X (gfx950) execution of fixed tensor-network contraction trees.

The library `libtn.so` (C ABI, declared in include/tn.h) plans and runs a
pairwise contraction tree, optionally sliced, on one GPU.  This package holds
its thin Python binding (`binding`), the autograd wrapper (`autograd`) and the
FLOP conventions used for reporting (`metrics`).  Every step of the
contraction runs in the library's HIP kernels; there is no CPU fallback.
"""

__all__ = ["binding", "autograd", "metrics"]
