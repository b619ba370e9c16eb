"""Helpers for the GPU tests: run a network through libtn and compare with the
oracle.  Inputs come from tn_inputs; expected values from oracle/ only.

A complex64 plan receives its leaves rounded to complex64.  The parity
reference for it is the oracle's complex128 contraction of those same
rounded leaves (c64_leaves: rounding done here by numpy, promotion back to
complex128 is exact), so that the comparison measures the contraction's own
error.  How far rounding the leaves moves the exact result is a property of
the input, reported beside it (on the circuit configs it is about 1.1e-5
relative: every gate type recurs hundreds of times, so the rounding of its
entries adds up coherently)."""

import sys

import numpy as np

TOL_C64 = 1e-5
TOL_C128 = 1e-10
# BF16x3: each real product carries ~2^-16 relative error (lo*lo dropped, lo
# rounded); the stated bound for whole contractions is this measured ceiling
TOL_BF16X3 = 3e-4
# 3M: Im = T3 - T1 - T2 loses componentwise accuracy when |Im| << |Re|
TOL_3M = 1e-4
# cancellation-heavy scalars (the random-Gaussian network): normwise backward
# error err / kappa of the last contraction, kappa = sum over slices of
# ||T_l|| ||T_r|| / |Z| (oracle/contract.root_condition); 1e-6 is 16 units of
# FP32 rounding (2^-24), the precision the root's children are stored in
TOL_BACKWARD_C64 = 1e-6
TOL_BACKWARD_BF16X3 = 1e-5


def rel(a, b):
    """Normwise relative error ||a - b||_2 / ||b||_2."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def rel_inf(a, b):
    """Max-componentwise error relative to the largest component:
    max_i |a_i - b_i| / max_i |b_i|."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_cw(a, b):
    """Largest componentwise relative error max_i |a_i - b_i| / |b_i| (over
    components with b_i != 0)."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    nz = np.abs(b) > 0
    return float((np.abs(a - b)[nz] / np.abs(b)[nz]).max()) if nz.any() else 0.0


def check(got, ref, tol, *what):
    """Normwise and max-componentwise relative errors both within tol."""
    e2, ei = rel(got, ref), rel_inf(got, ref)
    note(*what, "rel err %.3e  max-componentwise %.3e  componentwise %.3e" % (e2, ei, rel_cw(got, ref)))
    assert e2 < tol, (what, e2, tol)
    assert ei < tol, (what, ei, tol)
    return e2, ei


def c64_leaves(net):
    """The network with every leaf rounded to complex64 (as a complex64 plan
    receives it) and promoted back to complex128 (exact)."""
    return net.with_leaves([np.asarray(t).astype(np.complex64).astype(np.complex128) for t in net.leaves])


def ref_net(net, precision):
    """Network whose oracle value is the parity reference of `precision`."""
    return net if precision == "c128" else c64_leaves(net)


def note(*msg):
    print(*msg, flush=True)
    sys.stdout.flush()


def to_dev(net, precision):
    import torch
    dt = torch.complex128 if precision == "c128" else torch.complex64
    return [torch.from_numpy(np.ascontiguousarray(t)).to(device="cuda", dtype=dt).contiguous() for t in net.leaves]


def gpu_sliced(net, tree, sliced=(), slice_ids=None, precision="c64_4m", max_inflight=0, plan=None,
               gemm_all_sizes=False):
    import torch
    from paper_2002_01935_amd.binding import Plan
    p = plan or Plan(net, tree, sliced=sliced, precision=precision, max_inflight_slices=max_inflight,
                     gemm_all_sizes=gemm_all_sizes)
    leaves = to_dev(net, precision)
    out = p.contract_sliced(leaves, slice_ids=slice_ids)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def gpu_contract(net, tree, precision="c64_4m", gemm_all_sizes=False):
    import torch
    from paper_2002_01935_amd.binding import Plan
    p = Plan(net, tree, precision=precision, gemm_all_sizes=gemm_all_sizes)
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
