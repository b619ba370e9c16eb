"""FLOP conventions for reporting (Sec. 2 and table tab:benchmark).

A pairwise contraction at node v costs 2^{vc(v)} multiply-adds (eq. vertexcon);
for complex tensors each is counted as 8 real FLOPs (6 for the product, 2 for
the sum), so a tree of cost C is 8 C FLOPs.  The benchmark table's FLOPs
efficiency is 8 C_s / time divided by the device's peak rate.
"""

from __future__ import annotations


def complex_flops(log2_cost: float) -> float:
    """8 C for a tree (or sliced tree) of cost C = 2**log2_cost."""
    return 8.0 * 2.0 ** log2_cost


def efficiency(flops: float, seconds: float, peak_flops_per_s: float) -> float:
    return flops / seconds / peak_flops_per_s
