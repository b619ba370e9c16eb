"""QAOA energy terms as tensor networks (Sec. 4.4, QAOA energy evaluation).

The p-layer MAX-CUT ansatz on a graph G is
    |gamma, beta> = U_B(beta_p) U_C(gamma_p) ... U_B(beta_1) U_C(gamma_1) |+>^N
with U_C(gamma) = prod_{(j,k) in E} exp(-i gamma Z_j Z_k) and
U_B(beta) = prod_j exp(-i beta X_j); the energy is the sum over edges of
<gamma, beta| Z_j Z_k |gamma, beta> (unit weights).  Each term is built as its
own network, <+| U^dagger Z_j Z_k U |+> restricted to the reverse light cone of
{j, k}: going back from the observable, a mixer layer keeps the rotations on
the current cone, and a cost layer keeps the ZZ gates that touch the cone (the
layer's gates commute, so the others cancel against their adjoints) and then
adds their qubits to the cone.  Qubits outside the final cone contribute
<+|+> = 1 and are left out.

Gate tensors: ZZ as the rank-4 leaf (o_a, o_b, i_a, i_b) of
diag(e^{-i gamma}, e^{i gamma}, e^{i gamma}, e^{-i gamma}); the mixer as
[[cos beta, -i sin beta], [-i sin beta, cos beta]] (out, in); the bra side uses
the conjugate transposes.  Seeded parameters and graphs only: no method
arithmetic here.
"""

from __future__ import annotations

import numpy as np

from .graphs import random_regular_edges
from .network import Network


def zz_gate(gamma: float) -> np.ndarray:
    ph = np.exp(-1j * gamma * np.array([1, -1, -1, 1]))
    return np.diag(ph).reshape(2, 2, 2, 2)


def mixer_gate(beta: float) -> np.ndarray:
    c, s = np.cos(beta), np.sin(beta)
    return np.array([[c, -1j * s], [-1j * s, c]])


def light_cone(edges, p: int, j: int, k: int):
    """Kept gates per layer, backwards from Z_j Z_k: returns (cost[l], mixer[l])
    for l = 0..p-1 (time order), and the cone at time 0."""
    cone = {j, k}
    cost, mixer = [None] * p, [None] * p
    for l in range(p - 1, -1, -1):
        mixer[l] = sorted(cone)
        kept = [e for e in edges if e[0] in cone or e[1] in cone]
        cost[l] = kept
        for a, b in kept:
            cone.add(a)
            cone.add(b)
    return cost, mixer, sorted(cone)


def term_network(edges, gammas, betas, j: int, k: int) -> Network:
    """<+| U^dagger Z_j Z_k U |+> on the light cone of (j, k): a scalar network."""
    p = len(gammas)
    cost, mixer, cone0 = light_cone(edges, p, j, k)
    leaves, leaf_idx = [], []
    n_idx = 0
    wire = {}
    plus = np.array([1.0, 1.0], dtype=np.complex128) / np.sqrt(2.0)
    for q in cone0:
        wire[q] = n_idx
        n_idx += 1
        leaves.append(plus.copy())
        leaf_idx.append([wire[q]])
    gates = []                                    # (kind, qubits, matrix (out, in)), ket side in time order
    for l in range(p):
        for a, b in cost[l]:
            gates.append(("2q", (a, b), zz_gate(gammas[l])))
        for q in mixer[l]:
            gates.append(("1q", (q,), mixer_gate(betas[l])))
    z = np.diag([1.0, -1.0]).astype(np.complex128)
    full = gates + [("1q", (j,), z), ("1q", (k,), z)]
    # bra side: adjoints in reverse order
    for kind, qs, u in reversed(gates):
        if kind == "1q":
            full.append((kind, qs, u.conj().T))
        else:
            full.append((kind, qs, u.reshape(4, 4).conj().T.reshape(2, 2, 2, 2)))
    for kind, qs, u in full:
        if kind == "1q":
            (q,) = qs
            o = n_idx
            n_idx += 1
            leaves.append(np.array(u, dtype=np.complex128))
            leaf_idx.append([o, wire[q]])
            wire[q] = o
        else:
            a, b = qs
            oa, ob = n_idx, n_idx + 1
            n_idx += 2
            leaves.append(np.array(u, dtype=np.complex128))
            leaf_idx.append([oa, ob, wire[a], wire[b]])
            wire[a], wire[b] = oa, ob
    for q in cone0:
        leaves.append(plus.copy())
        leaf_idx.append([wire[q]])
    net = Network(leaves, leaf_idx, [2] * n_idx, [],
                  meta=dict(kind="qaoa_term", term=(j, k), p=p, cone=tuple(cone0)))
    net.check()
    return net


def instance(n: int, p: int, seed: int):
    """Seeded MAX-CUT instance: a random 3-regular graph on n vertices and
    parameters gamma, beta drawn uniformly from [0, pi)."""
    edges = random_regular_edges(n, 3, seed)
    rng = np.random.default_rng(seed + 7)
    gammas = rng.uniform(0.0, np.pi, size=p)
    betas = rng.uniform(0.0, np.pi, size=p)
    return edges, gammas, betas


def term_networks(n: int, p: int, seed: int):
    edges, gammas, betas = instance(n, p, seed)
    return edges, [term_network(edges, gammas, betas, j, k) for j, k in edges]
