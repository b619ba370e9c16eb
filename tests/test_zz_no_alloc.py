"""The allocation-free entry point (tn_contract_sliced_noalloc) against the
workspace entry point (tn_contract_sliced) it mirrors, through the C ABI:
two calls in a row on the shared static scratch, the second with a smaller
network, each bitwise equal to the workspace call's result (same kernels in
the same order) and within the complex64 tolerance of the oracle evaluated
on the same complex64 leaves.  Also: a plan whose workspace exceeds the
static scratch is refused with TN_E_WORKSPACE."""

import numpy as np
import pytest

from tests.gpu_util import TOL_C64, c64_leaves, note, rel, to_dev
from tn_inputs.circuits import circuit_network
from tn_inputs.graphs import pairwise_network
from tn_inputs.greedy import find_tree
from tn_inputs.network import Tree

pytestmark = pytest.mark.gpu


def _run_pair(plan, net, ids):
    import torch
    leaves = to_dev(net, "c64_4m")
    ws_out = plan.contract_sliced(leaves, slice_ids=ids)
    out = torch.empty(plan.out_shape, dtype=torch.complex128, device="cuda")
    out.fill_(float("nan"))
    na_out = plan.contract_sliced_noalloc(leaves, out, slice_ids=ids)
    torch.cuda.synchronize()
    return ws_out.cpu().numpy(), na_out.cpu().numpy()


def test_noalloc_matches_workspace_entry(oracle_lib):
    from paper_2002_01935_amd.binding import Plan

    big = circuit_network(5, 4, 12, 7, 0b10110011101001011101, open_qubits=(6, 9, 13))
    btree = find_tree(big, seed=2, trials=4, slice_width=16)
    bsl = list(btree.meta["sliced"])
    small = circuit_network(3, 4, 8, 1, 0b101100111010, open_qubits=(4,))
    stree = find_tree(small, seed=0, trials=2, slice_width=7)
    ssl = list(stree.meta["sliced"])
    cases = [(big, btree, bsl, 2), (small, stree, ssl, 1)]
    for k, (net, tree, sl, inflight) in enumerate(cases):
        plan = Plan(net, tree, sliced=sl, precision="c64_4m", max_inflight_slices=inflight)
        ws = plan.info()["workspace_bytes"]
        d = plan.info()["d_sliced"]
        ids = list(range(d)) if k == 1 else list(range(1, d, 2))
        note("noalloc call", k, "leaves", net.n_leaves, "sliced", len(sl), "workspace", ws, "ids", len(ids))
        assert ws <= 64 << 20
        a, b = _run_pair(plan, net, ids)
        assert np.array_equal(a, b), (k, a.ravel()[:4], b.ravel()[:4])
        ref = oracle_lib.contract(c64_leaves(net), tree, sliced=sl, slice_ids=ids)
        assert rel(b, ref) < TOL_C64
    note("noalloc: both calls bitwise equal to tn_contract_sliced")


def test_noalloc_rejects_large_workspace():
    import torch

    from paper_2002_01935_amd.binding import Plan, TNError

    net = pairwise_network(0, 12, 12, 1, seed=3)   # 2^24-element output: 128 MiB arena
    plan = Plan(net, Tree(np.array([0], np.int32), np.array([1], np.int32)), precision="c64_4m")
    assert plan.info()["workspace_bytes"] > 64 << 20
    out = torch.empty(plan.out_shape, dtype=torch.complex128, device="cuda")
    with pytest.raises(TNError) as ei:
        plan.contract_sliced_noalloc(to_dev(net, "c64_4m"), out)
    assert ei.value.code == -4
    note("noalloc: oversize plan refused:", str(ei.value))
