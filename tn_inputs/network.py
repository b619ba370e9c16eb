"""Network and tree containers (problem statement, Sec. 2).

A network is a list of leaf tensors T_v, each with an ordered index tuple t_v
(its axis order, outermost first, row-major), a dimension |D(e)| for every
index e, and an optional ordered list of open output indices.  An index shared
by more than two leaves, or shared by one leaf and the output, is a hyperedge
(Sec. 3.5); the containers accept them.

A tree is the pair of tuples l, r of Sec. 2 in SSA form: internal node
n_leaves + k has children left[k], right[k]; the last node is the root.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Network:
    leaves: list            # list of complex ndarrays; leaves[v].shape == tuple(idx_dim[e] for e in leaf_idx[v])
    leaf_idx: list          # list of lists of int index ids (t_v)
    idx_dim: list           # dimension of each index id
    out_idx: list = field(default_factory=list)   # open indices, in output axis order
    meta: dict = field(default_factory=dict)

    @property
    def n_leaves(self) -> int:
        return len(self.leaf_idx)

    @property
    def n_idx(self) -> int:
        return len(self.idx_dim)

    def check(self) -> None:
        """Shape checks only (no arithmetic): leaf shapes agree with dims."""
        assert len(self.leaves) == len(self.leaf_idx)
        for v, (t, ix) in enumerate(zip(self.leaves, self.leaf_idx)):
            assert tuple(t.shape) == tuple(self.idx_dim[e] for e in ix), (v, t.shape, ix)
            assert len(set(ix)) == len(ix), f"leaf {v} repeats an index"

    def flat(self):
        """Flattened int64 arrays in the layout the C entry points take."""
        rank = np.array([len(ix) for ix in self.leaf_idx], dtype=np.int32)
        cat = [e for ix in self.leaf_idx for e in ix]
        leaf_idx = np.array(cat, dtype=np.int64)
        idx_dim = np.array(self.idx_dim, dtype=np.int64)
        out_idx = np.array(self.out_idx, dtype=np.int64)
        return rank, leaf_idx, idx_dim, out_idx

    def with_leaves(self, leaves) -> "Network":
        return Network(list(leaves), self.leaf_idx, self.idx_dim, self.out_idx, dict(self.meta))

    def astype(self, dtype) -> "Network":
        return self.with_leaves([np.ascontiguousarray(t, dtype=dtype) for t in self.leaves])


@dataclass
class Tree:
    left: np.ndarray        # int32, n_leaves - 1
    right: np.ndarray       # int32, n_leaves - 1
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return 2 * len(self.left) + 1
