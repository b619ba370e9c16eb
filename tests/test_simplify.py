"""Rank simplification (Sec. 3.7; tn_inputs/simplify.py), structure only:
what the paper states about it and that the composed tree contracts to the
same value.  No GPU."""

import numpy as np
import pytest

from oracle import statevector as sv
from tn_inputs.circuits import circuit_network, gate_leaves, random_circuit
from tn_inputs.graphs import random_network
from tn_inputs.greedy import find_tree, tree_masks
from tn_inputs.simplify import compose, rank_simplify, structure_network


def _ranks(net, simp):
    """Ranks of the inputs and output of every merge, from the composed
    tree's kept sets (tn_inputs.greedy.tree_masks, an independent count)."""
    st = find_tree(structure_network(net, simp), seed=0, trials=1)
    full = compose(simp, st)
    kept, _ = tree_masks(net, full)
    n = net.n_leaves
    out = []
    for k, (a, b) in enumerate(simp.pairs):
        out.append((kept[a].bit_count(), kept[b].bit_count(), kept[n + k].bit_count()))
    return full, out


@pytest.mark.parametrize("decompose", ["none", "swap_diag"])
def test_merges_never_raise_rank(decompose):
    net = circuit_network(4, 5, 10, 3, 0b10110011101001011101, open_qubits=(6, 13), decompose=decompose)
    simp = rank_simplify(net)
    assert len(simp.pairs) > 0
    _, ranks = _ranks(net, simp)
    for ra, rb, ro in ranks:
        assert ro <= max(ra, rb)


def test_no_hyperedges_absorbs_rank_one_and_two():
    """Without hyperedges the procedure absorbs every rank-1 and rank-2
    tensor into a neighbour (the paper's remark): no survivor has rank <= 2."""
    net = circuit_network(4, 4, 8, 1, 0b1011001110100101, open_qubits=(5,))
    simp = rank_simplify(net)
    assert len(simp.survivors) > 1
    assert min(m.bit_count() for m in simp.masks) >= 3
    # a random network with rank-1/2 tensors, no hyperedges
    rn = random_network(14, 20, 4, seed=9, n_out=1, dims=(2,), hyper=False)
    s2 = rank_simplify(rn)
    if len(s2.survivors) > 1:
        assert min(m.bit_count() for m in s2.masks) >= 3


def test_protected_leaves_are_not_merged():
    net = circuit_network(4, 4, 8, 2, 0b0110100110010110)
    wrt = gate_leaves(net, "2q")
    simp = rank_simplify(net, protect=wrt)
    merged = {x for pair in simp.pairs for x in pair}
    assert not merged & set(wrt)
    assert set(wrt) <= set(simp.survivors)


@pytest.mark.parametrize("decompose", ["none", "swap_diag"])
def test_composed_tree_contracts_to_the_same_value(oracle_lib, decompose):
    """The composed tree (merges, then a tree found on the simplified
    structure) is a tree of the original network: its oracle value equals
    the statevector's amplitudes (open qubits) and the unsimplified tree's."""
    R, C, m, seed, b = 3, 4, 8, 4, 0b101101001110
    opens = (1, 6)
    net = circuit_network(R, C, m, seed, b, open_qubits=opens, decompose=decompose)
    simp = rank_simplify(net)
    st = find_tree(structure_network(net, simp), seed=1, trials=2)
    full = compose(simp, st)
    assert len(full.left) == net.n_leaves - 1
    got = oracle_lib.contract(net, full)
    plain = oracle_lib.contract(net, find_tree(net, seed=1, trials=2))
    assert np.max(np.abs(got - plain)) < 1e-12
    # statevector: amplitudes with the open qubits free
    ref = sv.amplitude(R * C, random_circuit(R, C, m, seed), b, open_qubits=opens)
    assert np.max(np.abs(got - ref)) < 1e-12
