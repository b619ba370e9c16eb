"""Random regular graph networks (Sec. 4.1).

Each vertex of a random k-regular graph carries a rank-k tensor, each edge an
index of size 2.  The paper samples graphs uniformly (Viger-Latapy); here a
seeded pairing (configuration) model with rejection of self-loops and
multi-edges gives a uniform simple k-regular graph.  Entries are iid complex
Gaussian with Re, Im ~ N(0, 1/2), scaled by 2**(-3/4) per tensor so that for
|V| = 120, |E| = 180 the contraction has E|Z|^2 = 1.
"""

from __future__ import annotations

import numpy as np

from .network import Network


def random_regular_edges(n: int, k: int, seed: int, max_tries: int = 10000):
    rng = np.random.default_rng(seed)
    assert (n * k) % 2 == 0
    for _ in range(max_tries):
        stubs = np.repeat(np.arange(n), k)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        a, b = pairs[:, 0], pairs[:, 1]
        if np.any(a == b):
            continue
        key = np.minimum(a, b) * n + np.maximum(a, b)
        if len(np.unique(key)) != len(key):
            continue
        edges = sorted((int(min(x, y)), int(max(x, y))) for x, y in pairs)
        return edges
    raise RuntimeError("pairing model did not produce a simple graph")


def rrg_network(n: int = 120, k: int = 3, seed: int = 0, scale: float | None = None) -> Network:
    edges = random_regular_edges(n, k, seed)
    inc = [[] for _ in range(n)]
    for e, (u, v) in enumerate(edges):
        inc[u].append(e)
        inc[v].append(e)
    rng = np.random.default_rng(seed + 1_000_003)
    if scale is None:
        scale = 2.0 ** (-0.75)
    leaves = []
    for v in range(n):
        shape = (2,) * len(inc[v])
        t = (rng.normal(0.0, np.sqrt(0.5), size=shape)
             + 1j * rng.normal(0.0, np.sqrt(0.5), size=shape)) * scale
        leaves.append(t.astype(np.complex128))
    net = Network(leaves, inc, [2] * len(edges), [],
                  meta=dict(kind="rrg", n=n, k=k, seed=seed, edges=edges))
    net.check()
    return net


def random_network(n_leaves: int, n_idx: int, max_rank: int, seed: int, n_out: int = 0,
                   dims=(2,), hyper: bool = False) -> Network:
    """Small random connected network for tests: every index joins >= 2 leaves
    (or one leaf and the output); with `hyper`, some indices join 3 leaves."""
    rng = np.random.default_rng(seed)
    while True:
        leaf_idx = [[] for _ in range(n_leaves)]
        idx_dim = []
        out_idx = []
        # spanning chain keeps it connected
        order = rng.permutation(n_leaves)
        for a, b in zip(order[:-1], order[1:]):
            e = len(idx_dim)
            idx_dim.append(int(rng.choice(dims)))
            leaf_idx[a].append(e)
            leaf_idx[b].append(e)
        while len(idx_dim) < n_idx:
            ends = 3 if (hyper and rng.random() < 0.3) else 2
            vs = rng.choice(n_leaves, size=ends, replace=False)
            if any(len(leaf_idx[v]) >= max_rank for v in vs):
                if all(len(ix) >= max_rank for ix in leaf_idx):
                    break
                continue
            e = len(idx_dim)
            idx_dim.append(int(rng.choice(dims)))
            for v in vs:
                leaf_idx[v].append(e)
        for _ in range(n_out):
            v = int(rng.integers(n_leaves))
            e = len(idx_dim)
            idx_dim.append(int(rng.choice(dims)))
            leaf_idx[v].append(e)
            out_idx.append(e)
        if all(len(ix) <= max_rank + n_out for ix in leaf_idx):
            break
    for ix in leaf_idx:
        rng.shuffle(ix)
    rng.shuffle(out_idx)
    leaves = []
    for ix in leaf_idx:
        shape = tuple(idx_dim[e] for e in ix)
        leaves.append((rng.normal(size=shape) + 1j * rng.normal(size=shape)).astype(np.complex128))
    net = Network(leaves, [list(map(int, ix)) for ix in leaf_idx], idx_dim, [int(e) for e in out_idx],
                  meta=dict(kind="random", seed=seed))
    net.check()
    return net


def pairwise_network(h: int, m: int, n: int, k: int, seed: int, dims=(2, 4)) -> Network:
    """Two leaves A(H, M, K) and B(H, K, N) with open outputs (H, M, N), each in
    a random axis order.  h, m, n, k are log2 sizes of the classes; indices
    have dimensions drawn from `dims` (powers of two) to fill each class."""
    rng = np.random.default_rng(seed)

    def split(bits):
        out = []
        while bits > 0:
            choices = [d for d in dims if int(np.log2(d)) <= bits]
            d = int(rng.choice(choices))
            out.append(d)
            bits -= int(np.log2(d))
        return out

    idx_dim = []
    cls = {}
    for name, bits in (("H", h), ("M", m), ("N", n), ("K", k)):
        ids = []
        for d in split(bits):
            ids.append(len(idx_dim))
            idx_dim.append(d)
        cls[name] = ids
    a_idx = cls["H"] + cls["M"] + cls["K"]
    b_idx = cls["H"] + cls["K"] + cls["N"]
    out = cls["H"] + cls["M"] + cls["N"]
    a_idx = [a_idx[i] for i in rng.permutation(len(a_idx))]
    b_idx = [b_idx[i] for i in rng.permutation(len(b_idx))]
    out = [out[i] for i in rng.permutation(len(out))]
    leaves = []
    for ix in (a_idx, b_idx):
        shape = tuple(idx_dim[e] for e in ix)
        leaves.append((rng.normal(size=shape) + 1j * rng.normal(size=shape)).astype(np.complex128))
    net = Network(leaves, [a_idx, b_idx], idx_dim, out, meta=dict(kind="pairwise", hmnk=(h, m, n, k)))
    net.check()
    return net
