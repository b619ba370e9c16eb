"""Rank simplification (Sec. 3.7), on the network's structure only.

A greedy contraction path that targets rank reduction only (eq.
greedy-cost-function with alpha = 0, no Boltzmann noise: the pair with the
smallest output first) is followed, performing only the pairwise
contractions whose output rank is not larger than the larger of the two
input ranks; without hyperedges that absorbs every rank-1 and rank-2 tensor
into a neighbour, as the paper notes.  Leaves listed in `protect` (tensors
whose gradient is wanted, or whose values change between uses of the tree)
are never merged.

Nothing is contracted here: the merges become the first pairwise nodes of
the tree over the original leaves (`compose`), so the GPU runs them like
every other contraction, and a path finder sees the merged tensors through
`structure_network`.
"""

from __future__ import annotations

import heapq
import math

import numpy as np

from .greedy import _bits
from .network import Network, Tree


class RankSimplified:
    """Result of `rank_simplify`: the merges as SSA pairs over the original
    leaves (internal node n + k is merge k), and the surviving tensors: their
    node ids and index masks."""

    def __init__(self, n_leaves, pairs, survivors, masks):
        self.n_leaves = n_leaves
        self.pairs = pairs          # list of (left, right) node ids
        self.survivors = survivors  # node ids of the tensors left, in a fixed order
        self.masks = masks          # their index sets as bitmasks


def rank_simplify(net: Network, protect=()) -> RankSimplified:
    n = net.n_leaves
    protect = set(int(v) for v in protect)
    log2w = [math.log2(d) for d in net.idx_dim]
    out_mask = 0
    for e in net.out_idx:
        out_mask |= 1 << e
    masks, count, holders = {}, {}, {}
    for v, ix in enumerate(net.leaf_idx):
        m = 0
        for e in ix:
            m |= 1 << e
            count[e] = count.get(e, 0) + 1
            holders.setdefault(e, set()).add(v)
        masks[v] = m

    def kept(mi, mj):
        keep = 0
        for e in _bits(mi | mj):
            rem = count[e] - ((mi >> e) & 1) - ((mj >> e) & 1)
            if rem > 0 or (out_mask >> e) & 1:
                keep |= 1 << e
        return keep

    def lsize(m):
        return sum(log2w[e] for e in _bits(m))

    def candidate(i, j):
        """(log2 size of the output, output mask) if merging i, j qualifies."""
        if i in protect or j in protect:
            return None
        mi, mj = masks[i], masks[j]
        mk = kept(mi, mj)
        if mk.bit_count() > max(mi.bit_count(), mj.bit_count()):
            return None
        return lsize(mk), mk

    heap = []

    def push_pairs(t):
        nb = set()
        for e in _bits(masks[t]):
            nb |= holders[e]
        nb.discard(t)
        for o in sorted(nb):
            c = candidate(min(o, t), max(o, t))
            if c is not None:
                heapq.heappush(heap, (c[0], min(o, t), max(o, t)))

    for v in range(n):
        push_pairs(v)
    pairs = []
    nxt = n
    while heap:
        cost, i, j = heapq.heappop(heap)
        if i not in masks or j not in masks:
            continue
        c = candidate(i, j)           # index counts may have changed since the pair was scored
        if c is None:
            continue
        if abs(c[0] - cost) > 1e-9:
            heapq.heappush(heap, (c[0], i, j))
            continue
        mi, mj, mk = masks[i], masks[j], c[1]
        for e in _bits(mi | mj):
            count[e] -= ((mi >> e) & 1) + ((mj >> e) & 1)
            holders[e].discard(i)
            holders[e].discard(j)
            if (mk >> e) & 1:
                count[e] += 1
                holders[e].add(nxt)
        del masks[i], masks[j]
        masks[nxt] = mk
        pairs.append((i, j))
        push_pairs(nxt)
        nxt += 1
    survivors = sorted(masks)
    return RankSimplified(n, pairs, survivors, [masks[s] for s in survivors])


def structure_network(net: Network, simp: RankSimplified) -> Network:
    """Network of the surviving tensors (index structure only; no leaf data):
    what a path finder sees after the simplification.  Index ids are the
    original ones."""
    leaf_idx = [list(_bits(m)) for m in simp.masks]
    return Network([None] * len(leaf_idx), leaf_idx, list(net.idx_dim), list(net.out_idx),
                   meta=dict(simplified_from=net.n_leaves))


def compose(simp: RankSimplified, tree: Tree) -> Tree:
    """Tree over the original leaves: the merges first, then `tree` (a tree
    over the surviving tensors, in their order) on top."""
    n = simp.n_leaves
    p = len(simp.pairs)
    m = len(simp.survivors)
    left = [a for a, _ in simp.pairs]
    right = [b for _, b in simp.pairs]

    def node(x):
        x = int(x)
        return simp.survivors[x] if x < m else n + p + (x - m)

    left += [node(x) for x in tree.left]
    right += [node(x) for x in tree.right]
    meta = dict(tree.meta)
    meta["rank_simplified_merges"] = p
    return Tree(np.array(left, np.int32), np.array(right, np.int32), meta=meta)
