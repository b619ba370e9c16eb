"""Sub-network below one tree node, as an input of its own (structure only).

The tensor at node v of a contraction tree (Sec. 2) is the contraction of
the leaves below v with the indices v keeps left open: those that are open
outputs of the whole network or also occur on a leaf outside v's subtree.
This builds that sub-network (its leaves, its tree in the same pairwise
order, its open indices in ascending original index id) so that a GPU plan
can produce the node's value, with some indices fixed to given values
(the slice of Sec. 4.7.1 the node belongs to): their axes are taken out of
the leaves, as a sliced contraction's leaf view does.
"""

from __future__ import annotations

import numpy as np

from .network import Network, Tree


def subtree_network(net: Network, tree: Tree, node: int, fixed: dict | None = None):
    """(sub-network, sub-tree, open index ids in the original numbering) of
    the subtree rooted at `node`; `fixed` maps index id -> value."""
    fixed = dict(fixed or {})
    n = net.n_leaves
    left = [int(x) for x in tree.left]
    right = [int(x) for x in tree.right]
    below, internal = [], []
    stack = [node]
    while stack:
        v = stack.pop()
        if v < n:
            below.append(v)
        else:
            internal.append(v)
            stack.append(right[v - n])
            stack.append(left[v - n])
    inside = set(below)
    occ_in, occ_out = set(), set()
    for v, ix in enumerate(net.leaf_idx):
        (occ_in if v in inside else occ_out).update(ix)
    outs = set(net.out_idx)
    open_idx = sorted(e for e in occ_in if e not in fixed and (e in outs or e in occ_out))
    leaves, idx = [], []
    for v in below:
        t = np.asarray(net.leaves[v])
        ix = list(net.leaf_idx[v])
        for e in [e for e in ix if e in fixed]:
            t = np.take(t, fixed[e], axis=ix.index(e))
            ix.remove(e)
        leaves.append(np.ascontiguousarray(t))
        idx.append(ix)
    remap = {}
    for ix in idx:
        for e in ix:
            remap.setdefault(e, len(remap))
    dims = [net.idx_dim[e] for e in sorted(remap, key=remap.get)]
    sub = Network(leaves, [[remap[e] for e in ix] for ix in idx], dims, [remap[e] for e in open_idx])
    # internal nodes in ascending id order are a valid pairwise order (each
    # node's children come before it); renumber leaves first, then them
    new_id = {v: i for i, v in enumerate(below)}
    for v in sorted(internal):
        new_id[v] = len(new_id)
    order = sorted(internal)
    sl = [new_id[left[v - n]] for v in order]
    sr = [new_id[right[v - n]] for v in order]
    return sub, Tree(np.array(sl, np.int32), np.array(sr, np.int32)), open_idx


def slice_values(sliced, dims, slice_id):
    """Index id -> value of slice `slice_id` over `sliced` (mixed radix, first
    index most significant)."""
    vals = {}
    s = int(slice_id)
    for e, d in zip(reversed(list(sliced)), reversed(list(dims))):
        vals[e] = s % int(d)
        s //= int(d)
    return vals
