"""CPU pin of the projection used by the full-size GPU parity tests: zeroing
the entries x_e != x of one leaf per extra index turns a slice of the network
into a sub-slice of the same tree with those indices sliced as well."""

import numpy as np

from tests.gpu_util import project, rel, sub_slice_id
from tn_inputs.circuits import circuit_network
from tn_inputs.greedy import find_tree
from tn_inputs.slicing import extend_slices


def test_projection_equals_sub_slice(oracle_lib):
    net = circuit_network(3, 4, 8, 2, 0b110010011010, open_qubits=(5, 6))
    tree = find_tree(net, seed=0, trials=2, slice_width=9)
    sliced = tree.meta["sliced"]
    ext = extend_slices(net, tree, sliced, 12.0)
    extra = ext[len(sliced):]
    assert len(extra) >= 2
    rng = np.random.default_rng(0)
    for s in (0, 3):
        s = s % (2 ** len(sliced))
        vals = [int(x) for x in rng.integers(0, 2, size=len(extra))]
        got = oracle_lib.contract(project(net, extra, vals), tree, sliced=sliced, slice_ids=[s])
        ref = oracle_lib.contract(net, tree, sliced=ext,
                                  slice_ids=[sub_slice_id(s, vals, [net.idx_dim[e] for e in extra])])
        assert rel(got, ref) < 1e-12
