"""Full-size parity in the launch configuration bench.py times (autotuned
tiles, graph replay, one in-flight slice; bench.py replays cfg3's slices
eight at a time, and results do not depend on the number in flight:
tests/test_gpu_parity.py test_sliced_subsets_and_batches): a whole slice of
cfg5 and cfg5h (width 30) and of cfg3 (width 27) runs on the GPU with a few more indices
projected out of the leaves (tests/gpu_util.project), and the oracle
evaluates the matching sub-slice of the same tree on the same complex64
leaves.

Tolerance (complex64, 4M): 1e-5 relative, normwise and max-componentwise.
The error of the exact result against the complex128 circuit (the input's
own complex64 rounding, about 1.1e-5 on these circuits, plus the
contraction's error) is reported beside it.  3M: the same bound; BF16x3:
its stated bound.  The root's two children, each planned on the GPU as a
network of its own (tn_inputs.subnet), are held to the same bound against
the oracle's value of the same subtree."""

import numpy as np
import pytest

from tests.gpu_util import (TOL_BF16X3, TOL_C64, c64_leaves, check, note, project, rel, rel_inf, sub_slice_id,
                            to_dev)
from tn_inputs import configs
from tn_inputs.slicing import extend_slices
from tn_inputs.subnet import slice_values, subtree_network

pytestmark = pytest.mark.gpu

# (workload, log2 cost of the oracle's sub-slice, position in the seeded slice
# subset, seed of the projected values)
CASES = {"cfg5": ("cfg5", 33.0, 7, 1), "cfg5h": ("cfg5h", 33.0, 11, 3), "cfg3": ("cfg3", 31.0, 3, 2)}
_memo = {}


def _case(name):
    if name not in _memo:
        wl, target, pos, seed_vals = CASES[name]
        net, tree, sliced = configs.load(wl)
        ids = configs.slice_subset(2 ** len(sliced), seed=0, size=256)
        s = ids[pos]
        ext = extend_slices(net, tree, sliced, target)
        extra = ext[len(sliced):]
        vals = [int(x) for x in np.random.default_rng(seed_vals).integers(0, 2, size=len(extra))]
        sid = sub_slice_id(s, vals, [net.idx_dim[e] for e in extra])
        _memo[name] = (net, tree, sliced, s, ext, extra, vals, sid)
    return _memo[name]


def _gpu_slice(name, prec):
    import torch

    from paper_2002_01935_amd.binding import Plan
    net, tree, sliced, s, ext, extra, vals, sid = _case(name)
    pnet = project(net, extra, vals)
    plan = Plan(net, tree, sliced=sliced, precision=prec, max_inflight_slices=1)
    ws = plan.workspace()
    plan.tune(ws)
    note(name, prec, "slice", s, "extra", len(extra), "workspace GiB", plan.info()["workspace_bytes"] / 2 ** 30)
    got = plan.contract_sliced(to_dev(pnet, prec), slice_ids=[s], workspace=ws).cpu().numpy()
    torch.cuda.synchronize()
    del ws
    return got


def _refs(name, oracle_lib):
    key = ("ref", name)
    if key not in _memo:
        net, tree, sliced, s, ext, extra, vals, sid = _case(name)
        ref = oracle_lib.contract(c64_leaves(net), tree, sliced=ext, slice_ids=[sid])
        ref128 = oracle_lib.contract(net, tree, sliced=ext, slice_ids=[sid])
        note(name, "input rounding: exact value of the complex64 leaves vs the complex128 circuit",
             "%.3e" % rel(ref, ref128))
        _memo[key] = (ref, ref128)
    return _memo[key]


@pytest.mark.parametrize("name,prec", [("cfg5", "c64_4m"), ("cfg5", "c64_3m"), ("cfg5", "c64_bf16x3"),
                                       ("cfg5h", "c64_4m"), ("cfg3", "c64_4m")])
def test_full_slice(oracle_lib, name, prec):
    got = _gpu_slice(name, prec)
    ref, ref128 = _refs(name, oracle_lib)
    note(name, prec, "vs the complex128 circuit: rel %.3e max-componentwise %.3e"
         % (rel(got, ref128), rel_inf(got, ref128)))
    check(got, ref, TOL_BF16X3 if prec == "c64_bf16x3" else TOL_C64, name, prec, "vs oracle on the same leaves")


@pytest.mark.parametrize("name", ["cfg5", "cfg5h", "cfg3"])
def test_root_children(oracle_lib, name):
    """Values of the root's two children for the same sub-slice: each child
    subtree planned and contracted on the GPU (complex64 4M, its indices that
    the sub-slice fixes taken out of the leaves), against the oracle's value
    of that subtree (oracle/contract.subtree_value)."""
    import torch

    from paper_2002_01935_amd.binding import Plan
    net, tree, sliced, s, ext, extra, vals, sid = _case(name)
    fixed = slice_values(ext, [net.idx_dim[e] for e in ext], sid)
    n = net.n_leaves
    net64 = c64_leaves(net)
    for side, child in (("left", int(tree.left[-1])), ("right", int(tree.right[-1]))):
        if child < n:
            continue
        sub, stree, open_idx = subtree_network(net, tree, child, fixed)
        plan = Plan(sub, stree, precision="c64_4m")
        ws = plan.workspace()
        plan.tune(ws)
        got = plan.contract_sliced(to_dev(sub, "c64_4m"), workspace=ws).cpu().numpy()
        torch.cuda.synchronize()
        del ws
        ref, kept = oracle_lib.subtree_value(net64, tree, child, ext, sid)
        assert kept == open_idx
        note(name, side, "child node", child, "open indices", len(open_idx), "elements", ref.size)
        check(got, ref, TOL_C64, name, side, "child")
