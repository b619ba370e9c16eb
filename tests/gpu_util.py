"""Helpers for the GPU tests: run a network through libtn and compare with the
oracle.  Inputs come from tn_inputs; expected values from oracle/ only."""

import sys

import numpy as np

TOL_C64 = 1e-5
TOL_C128 = 1e-10
# BF16x3: each real product carries ~2^-16 relative error (lo*lo dropped, lo
# rounded); the stated bound for whole contractions is this measured ceiling
TOL_BF16X3 = 3e-4
# 3M: Im = T3 - T1 - T2 loses componentwise accuracy when |Im| << |Re|
TOL_3M = 1e-4


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def note(*msg):
    print(*msg, flush=True)
    sys.stdout.flush()


def to_dev(net, precision):
    import torch
    dt = torch.complex128 if precision == "c128" else torch.complex64
    return [torch.from_numpy(np.ascontiguousarray(t)).to(device="cuda", dtype=dt).contiguous() for t in net.leaves]


def gpu_sliced(net, tree, sliced=(), slice_ids=None, precision="c64_4m", max_inflight=0, plan=None):
    import torch
    from paper_2002_01935_amd.binding import Plan
    p = plan or Plan(net, tree, sliced=sliced, precision=precision, max_inflight_slices=max_inflight)
    leaves = to_dev(net, precision)
    out = p.contract_sliced(leaves, slice_ids=slice_ids)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def gpu_contract(net, tree, precision="c64_4m"):
    import torch
    from paper_2002_01935_amd.binding import Plan
    p = Plan(net, tree, precision=precision)
    out = p.contract(to_dev(net, precision))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def project(net, extra, values):
    """Network whose contraction equals one sub-slice: for each extra index e
    with value x, the entries of the first leaf holding e with x_e != x are
    set to zero (multiplying the network by a delta on e)."""
    leaves = [np.array(t, copy=True) for t in net.leaves]
    for e, x in zip(extra, values):
        v = next(v for v, ix in enumerate(net.leaf_idx) if e in ix)
        ax = net.leaf_idx[v].index(e)
        sel = [slice(None)] * leaves[v].ndim
        for y in range(net.idx_dim[e]):
            if y != x:
                sel[ax] = y
                leaves[v][tuple(sel)] = 0
    return net.with_leaves(leaves)


def sub_slice_id(slice_id, extra_values, extra_dims):
    """Slice id in the extended sliced set (original list, then the extra
    indices): mixed radix with the first index most significant."""
    sid = int(slice_id)
    for x, d in zip(extra_values, extra_dims):
        sid = sid * int(d) + int(x)
    return sid
