"""Hyper-Greedy contraction-tree sampler (Sec. 3.4).

Pairs of tensors that share an index are scored with
    cost(T_i, T_j) = size(T_k) - alpha * (size(T_i) + size(T_j))      (eq. greedy-cost-function)
and a pair is drawn with probability proportional to exp(-cost / tau)
(eq. greedy-boltzmann-factor).  The Boltzmann draw uses the Gumbel-max form:
every candidate pair gets key = cost - tau * g with g ~ Gumbel(0, 1) when it
is created, and the smallest key is taken (tau = 0 is plain greedy).
Repeating this with sampled (alpha, tau) and keeping the best tree is the
Hyper-Greedy optimiser (Sec. 3.6 tunes the parameters; here they are drawn at
random from a seeded generator).

The sizes here only steer the search.  The tree is handed to the oracle and to
the GPU library, which recompute their own incidence sets from it.
"""

from __future__ import annotations

import heapq
import math

import numpy as np

from .network import Network, Tree


def _bits(mask: int):
    while mask:
        low = mask & -mask
        yield low.bit_length() - 1
        mask ^= low


class _Greedy:
    def __init__(self, net: Network, sliced=()):
        self.net = net
        self.log2w = [math.log2(d) for d in net.idx_dim]
        self.unit = all(d == 2 for d in net.idx_dim)
        self.out_mask = 0
        for e in net.out_idx:
            self.out_mask |= 1 << e
        self.sliced_mask = 0
        for e in sliced:
            self.sliced_mask |= 1 << e

    def log2size(self, mask: int) -> float:
        if self.unit:
            return float(mask.bit_count())
        return sum(self.log2w[e] for e in _bits(mask))

    def run(self, alpha: float, tau: float, rng) -> Tree:
        net = self.net
        n = net.n_leaves
        sets = {}
        holders = {}
        count = {}
        for v, ix in enumerate(net.leaf_idx):
            m = 0
            for e in ix:
                m |= 1 << e
                holders.setdefault(e, set()).add(v)
                count[e] = count.get(e, 0) + 1
            sets[v] = m
        out_mask = self.out_mask

        def kept(mi, mj):
            both = mi | mj
            keep = 0
            for e in _bits(both):
                rem = count[e] - ((mi >> e) & 1) - ((mj >> e) & 1)
                if rem > 0 or (out_mask >> e) & 1:
                    keep |= 1 << e
            return keep

        def score(i, j):
            mi, mj = sets[i], sets[j]
            mk = kept(mi, mj)
            sk = 2.0 ** self.log2size(mk)
            si = 2.0 ** self.log2size(mi)
            sj = 2.0 ** self.log2size(mj)
            c = sk - alpha * (si + sj)
            if tau > 0:
                c -= tau * rng.gumbel()
            return c

        heap = []
        seen = set()
        for e, hs in holders.items():
            hl = sorted(hs)
            for a in range(len(hl)):
                for b in range(a + 1, len(hl)):
                    key = (hl[a], hl[b])
                    if key not in seen:
                        seen.add(key)
                        heap.append((score(*key), key[0], key[1]))
        heapq.heapify(heap)
        alive = set(range(n))
        left, right = [], []
        nxt = n
        while len(alive) > 1:
            pair = None
            while heap:
                _, i, j = heapq.heappop(heap)
                if i in alive and j in alive:
                    pair = (i, j)
                    break
            if pair is None:
                # disconnected parts left: join the two smallest (outer product)
                order = sorted(alive, key=lambda t: (self.log2size(sets[t]), t))
                pair = (order[0], order[1])
            i, j = pair
            mi, mj = sets[i], sets[j]
            mk = kept(mi, mj)
            for e in _bits(mi | mj):
                count[e] -= ((mi >> e) & 1) + ((mj >> e) & 1)
                holders[e].discard(i)
                holders[e].discard(j)
                if (mk >> e) & 1:
                    count[e] += 1
                    holders[e].add(nxt)
            k = nxt
            nxt += 1
            sets[k] = mk
            alive.discard(i)
            alive.discard(j)
            alive.add(k)
            left.append(i)
            right.append(j)
            del sets[i], sets[j]
            nbrs = set()
            for e in _bits(mk):
                nbrs |= holders[e]
            nbrs.discard(k)
            for o in sorted(nbrs):
                a, b = (o, k)
                heapq.heappush(heap, (score(a, b), a, b))
        return Tree(np.array(left, dtype=np.int32), np.array(right, dtype=np.int32),
                    meta=dict(alpha=alpha, tau=tau))


def tree_masks(net: Network, tree: Tree):
    """Per-node kept-index bitmasks and, for internal nodes, the union of the
    children's kept sets (the indices counted by eq. vertexcon)."""
    n = net.n_leaves
    total = {}
    out_mask = 0
    for e in net.out_idx:
        out_mask |= 1 << e
    kept = [0] * (2 * n - 1)
    cnt = [None] * (2 * n - 1)
    for v, ix in enumerate(net.leaf_idx):
        m = 0
        c = {}
        for e in ix:
            m |= 1 << e
            total[e] = total.get(e, 0) + 1
            c[e] = 1
        kept[v] = m
        cnt[v] = c
    union = [0] * (2 * n - 1)
    for k, (l, r) in enumerate(zip(tree.left, tree.right)):
        v = n + k
        cl, cr = cnt[l], cnt[r]
        c = dict(cl)
        for e, x in cr.items():
            c[e] = c.get(e, 0) + x
        m = 0
        cv = {}
        for e, x in c.items():
            if x < total[e] or (out_mask >> e) & 1:
                m |= 1 << e
                cv[e] = x
        kept[v] = m
        union[v] = kept[l] | kept[r]
        cnt[v] = cv
        cnt[l] = cnt[r] = None
    return kept, union


def width_cost(net: Network, tree: Tree, sliced_mask: int = 0):
    """(W, log2 C) for the tree with the given indices removed (eqs. edgecon,
    vertexcon); log2 C sums over internal nodes only."""
    kept, union = tree_masks(net, tree)
    n = net.n_leaves
    log2w = [math.log2(d) for d in net.idx_dim]
    unit = all(d == 2 for d in net.idx_dim)
    keep = ~sliced_mask

    def lsz(m):
        m &= keep
        if unit:
            return m.bit_count()
        return sum(log2w[e] for e in _bits(m))

    W = max(lsz(m) for m in kept)
    C = 0.0
    for v in range(n, 2 * n - 1):
        C += 2.0 ** lsz(union[v])
    return W, math.log2(C) if C > 0 else float("-inf")


def find_tree(net: Network, seed: int = 0, trials: int = 32, alphas=(0.0, 1.5),
              taus=(1e-3, 1.0), target: str = "C", slice_width: int | None = None,
              slice_trials: int = 4, verbose: bool = False):
    """Best of `trials` Boltzmann-greedy trees.  Trial 0 is plain greedy with
    alpha = 0.5, tau = 0.  With `slice_width`, every candidate tree is sliced to
    that width (Sec. 4.7.1) and scored by its total sliced cost C_s."""
    from .slicing import choose_slices

    rng = np.random.default_rng(seed)
    g = _Greedy(net)
    best = None
    for t in range(trials):
        if t == 0:
            alpha, tau = 0.5, 0.0
        else:
            alpha = float(rng.uniform(*alphas))
            tau = float(math.exp(rng.uniform(math.log(taus[0]), math.log(taus[1]))))
        tree = g.run(alpha, tau, rng)
        if slice_width is not None:
            sl = choose_slices(net, tree, slice_width, seed=int(rng.integers(1 << 30)),
                               trials=slice_trials)
            score = (sl["log2_Cs"], sl["W"])
            tree.meta.update(sliced=sl["sliced"], W_s=sl["W_s"], log2_Cs=sl["log2_Cs"])
            W, lc = sl["W"], sl["log2_C"]
        else:
            W, lc = width_cost(net, tree)
            score = (lc, W) if target == "C" else (W, lc)
        tree.meta.update(W=W, log2_C=lc, trial=t)
        if verbose:
            print(f"trial {t}: alpha={alpha:.3f} tau={tau:.3g} W={W} log10C={lc*math.log10(2):.2f}"
                  + (f" log10Cs={tree.meta['log2_Cs']*math.log10(2):.2f}" if slice_width else ""))
        if best is None or score < best[0]:
            best = (score, tree)
    return best[1]
