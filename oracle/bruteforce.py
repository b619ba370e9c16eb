"""Direct evaluation of a network as nested sums (Sec. 4.7.1: a network is
|E| nested summations of the product of the entries of its tensors).

TEST INFRASTRUCTURE ONLY.  Enumerates every assignment of every index,
multiplies the leaf entries selected by each assignment and accumulates into
the entry of the open output indices.  Exponential in the number of indices:
for tiny networks only (<= ~22 binary indices).
"""

from __future__ import annotations

import numpy as np


def contract(net, max_assignments: int = 1 << 23) -> np.ndarray:
    dims = [int(d) for d in net.idx_dim]
    total = int(np.prod(dims, dtype=object))
    if total > max_assignments:
        raise ValueError(f"{total} assignments is too many for brute force")
    # every assignment of every index: column e holds x_e
    grids = np.indices(dims, dtype=np.int64).reshape(len(dims), -1)
    prod = np.ones(grids.shape[1], dtype=np.complex128)
    for t, ix in zip(net.leaves, net.leaf_idx):
        sel = tuple(grids[e] for e in ix)
        prod = prod * np.asarray(t, dtype=np.complex128)[sel]
    out_shape = tuple(dims[e] for e in net.out_idx)
    if not out_shape:
        return np.asarray(prod.sum())
    flat = np.ravel_multi_index(tuple(grids[e] for e in net.out_idx), out_shape)
    res = np.zeros(int(np.prod(out_shape)), dtype=np.complex128)
    np.add.at(res, flat, prod)
    return res.reshape(out_shape)
