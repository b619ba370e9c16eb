"""Greedy choice of sliced indices (Sec. 4.7.1).

Given a tree, indices are removed one at a time.  Each step considers the
indices of the currently widest nodes and takes the one whose removal gives
the lowest total sliced cost C_s = d_sliced * C(tree without the sliced
indices), with a small seeded random perturbation of the score; repeating the
whole procedure a few times and keeping the best sliced set is the
randomisation the paper describes.  Output indices are never sliced (the
paper slices scalar amplitudes; a sliced output would be concatenated, not
summed).
"""

from __future__ import annotations

import math

import numpy as np

from .greedy import _bits, tree_masks
from .network import Network, Tree


def choose_slices(net: Network, tree: Tree, target_width: int, seed: int = 0,
                  trials: int = 4, noise: float = 0.02):
    assert all(d == 2 for d in net.idx_dim), "greedy slicer assumes |D(e)| = 2"
    kept, union = tree_masks(net, tree)
    n = net.n_leaves
    out_mask = 0
    for e in net.out_idx:
        out_mask |= 1 << e
    internal = list(range(n, 2 * n - 1))
    W0 = max(m.bit_count() for m in kept)
    C0 = sum(2 ** union[v].bit_count() for v in internal)
    rng = np.random.default_rng(seed)
    best = None
    for t in range(trials):
        S = 0
        k = 0
        while True:
            widths = [(m & ~S).bit_count() for m in kept]
            W = max(widths)
            if W <= target_width:
                break
            cand = 0
            for v, w in enumerate(widths):
                if w == W:
                    cand |= kept[v]
            cand &= ~S & ~out_mask
            if cand == 0:
                raise ValueError("cannot reach target width without slicing outputs")
            # E[e] = sum over nodes whose union holds e of 2^{|union \ S|};
            # slicing e makes the total cost 2 * d * (C - E[e] / 2)
            E = {}
            for v in internal:
                u = union[v] & ~S
                c = 2 ** u.bit_count()
                for e in _bits(u & cand):
                    E[e] = E.get(e, 0) + c
            Ccur = sum(2 ** (union[v] & ~S).bit_count() for v in internal)
            best_e, best_s = None, None
            for e in _bits(cand):
                new_c = 2 * Ccur - E.get(e, 0)
                s = math.log2(new_c) + (noise * rng.gumbel() if t > 0 else 0.0)
                if best_s is None or s < best_s:
                    best_s, best_e = s, e
            S |= 1 << best_e
            k += 1
        Cs = sum(2 ** (union[v] & ~S).bit_count() for v in internal) * (2 ** k)
        rec = dict(sliced=sorted(_bits(S)), W=W0, W_s=max((m & ~S).bit_count() for m in kept),
                   log2_C=math.log2(C0), log2_Cs=math.log2(Cs), d_sliced=2 ** k)
        if best is None or rec["log2_Cs"] < best["log2_Cs"]:
            best = rec
    return best


def extend_slices(net: Network, tree: Tree, sliced, log2_cost_target: float):
    """Add indices to `sliced` (greedily, the one whose removal lowers the
    per-slice cost most) until one slice of the tree costs at most
    2**log2_cost_target.  The result slices the same tree further: every
    slice of it is a sub-slice of a slice of the original set."""
    kept, union = tree_masks(net, tree)
    n = net.n_leaves
    out_mask = 0
    for e in net.out_idx:
        out_mask |= 1 << e
    S = 0
    for e in sliced:
        S |= 1 << e
    order = list(sliced)
    internal = list(range(n, 2 * n - 1))
    while True:
        per = [2 ** (union[v] & ~S).bit_count() for v in internal]
        C = sum(per)
        if C <= 2.0 ** log2_cost_target:
            return order
        E = {}
        for v, c in zip(internal, per):
            for e in _bits(union[v] & ~S & ~out_mask):
                E[e] = E.get(e, 0) + c
        if not E:
            return order
        best = max(sorted(E), key=lambda e: E[e])
        S |= 1 << best
        order.append(best)
