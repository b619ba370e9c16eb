"""ctypes driver for the complex128 loop-nest oracle (oracle.c).

TEST INFRASTRUCTURE ONLY.  See oracle.c for what is computed and the readings
of the paper it takes.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True, path: str = _LIB, defines=()) -> str:
    """Compile oracle.c with gcc (OpenMP); returns the library path.
    `defines` (e.g. ORACLE_PLANT_SIGN) are for the mutation tests only."""
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-Wno-unused-function"] + [f"-D{d}" for d in defines] + [_SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, path)
    return path


def use_library(path: str | None) -> None:
    """Switch this module to another build of oracle.c (mutation tests);
    None returns to the normal build."""
    global _lib
    _lib = None if path is None else _open(path)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _open(_LIB)
    return _lib


def _open(path):
    if True:
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.oracle_contract.argtypes = [i32, P, P, i32, P, i32, P, P, P, i32, P, P, i64, P, P, i32]
        lib.oracle_contract.restype = ctypes.c_int
        lib.oracle_grad.argtypes = [i32, P, P, i32, P, i32, P, P, P, i32, P, P, P, i32, P, P, i64, P, i32]
        lib.oracle_grad.restype = ctypes.c_int
        lib.oracle_width_cost.argtypes = [i32, P, P, i32, P, i32, P, P, P, i32, P, P, P]
        lib.oracle_width_cost.restype = ctypes.c_int
        lib.oracle_last_error.restype = ctypes.c_char_p
    return lib


class OracleError(RuntimeError):
    pass


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size > 0 else None


def _prep(net, tree, sliced):
    rank, leaf_idx, idx_dim, out_idx = net.flat()
    left = np.ascontiguousarray(tree.left, dtype=np.int32)
    right = np.ascontiguousarray(tree.right, dtype=np.int32)
    sl = np.ascontiguousarray(np.array(list(sliced), dtype=np.int64))
    return rank, leaf_idx, idx_dim, out_idx, left, right, sl


def _n_threads(n):
    if n is not None:
        return int(n)
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def contract(net, tree, sliced=(), slice_ids=None, n_threads=None) -> np.ndarray:
    """Oracle value of the network (complex128, shape of the open outputs in
    out_idx order), summed over `slice_ids` (all slices when None)."""
    lib = _load()
    rank, leaf_idx, idx_dim, out_idx, left, right, sl = _prep(net, tree, sliced)
    data = [np.ascontiguousarray(t, dtype=np.complex128) for t in net.leaves]
    ptrs = (ctypes.c_void_p * len(data))(*[d.ctypes.data for d in data])
    shape = tuple(int(net.idx_dim[e]) for e in net.out_idx)
    out = np.zeros(shape if shape else (1,), dtype=np.complex128)
    ids = None if slice_ids is None else np.ascontiguousarray(np.array(slice_ids, dtype=np.int64))
    rc = lib.oracle_contract(net.n_leaves, _ptr(rank), _ptr(leaf_idx), net.n_idx, _ptr(idx_dim),
                             len(net.out_idx), _ptr(out_idx), _ptr(left), _ptr(right), len(sl), _ptr(sl),
                             ptrs, 0 if ids is None else len(ids), _ptr(ids),
                             out.ctypes.data_as(ctypes.c_void_p), _n_threads(n_threads))
    if rc != 0:
        raise OracleError(lib.oracle_last_error().decode())
    return out.reshape(shape)


def grad(net, tree, grad_out, wrt, sliced=(), slice_ids=None, n_threads=None):
    """Leaf gradients sum_o conj(dR_o/dT[k]) * grad_out[o] for leaves `wrt`."""
    lib = _load()
    rank, leaf_idx, idx_dim, out_idx, left, right, sl = _prep(net, tree, sliced)
    data = [np.ascontiguousarray(t, dtype=np.complex128) for t in net.leaves]
    ptrs = (ctypes.c_void_p * len(data))(*[d.ctypes.data for d in data])
    go = np.ascontiguousarray(np.asarray(grad_out, dtype=np.complex128))
    wrt = np.ascontiguousarray(np.array(list(wrt), dtype=np.int32))
    outs = [np.zeros(net.leaves[int(v)].shape, dtype=np.complex128) for v in wrt]
    gptrs = (ctypes.c_void_p * max(1, len(outs)))(*[o.ctypes.data for o in outs])
    ids = None if slice_ids is None else np.ascontiguousarray(np.array(slice_ids, dtype=np.int64))
    rc = lib.oracle_grad(net.n_leaves, _ptr(rank), _ptr(leaf_idx), net.n_idx, _ptr(idx_dim),
                         len(net.out_idx), _ptr(out_idx), _ptr(left), _ptr(right), len(sl), _ptr(sl),
                         ptrs, go.ctypes.data_as(ctypes.c_void_p), len(wrt), _ptr(wrt), gptrs,
                         0 if ids is None else len(ids), _ptr(ids), _n_threads(n_threads))
    if rc != 0:
        raise OracleError(lib.oracle_last_error().decode())
    return outs


def width_cost(net, tree, sliced=()):
    """(W, log2 C) per eqs. edgecon / vertexcon, computed by the oracle."""
    lib = _load()
    rank, leaf_idx, idx_dim, out_idx, left, right, sl = _prep(net, tree, sliced)
    W = ctypes.c_double()
    C = ctypes.c_double()
    rc = lib.oracle_width_cost(net.n_leaves, _ptr(rank), _ptr(leaf_idx), net.n_idx, _ptr(idx_dim),
                               len(net.out_idx), _ptr(out_idx), _ptr(left), _ptr(right), len(sl),
                               _ptr(sl), ctypes.byref(W), ctypes.byref(C))
    if rc != 0:
        raise OracleError(lib.oracle_last_error().decode())
    return math.log2(W.value), (math.log2(C.value) if C.value > 0 else float("-inf"))


def subtree_value(net, tree, node, sliced=(), slice_id=None):
    """Oracle value of the tensor at tree node `node`, as (array, index list):
    the sub-network of the leaves below `node`, with its kept indices (those
    that are outputs or occur on a leaf outside the subtree) left open.  With
    `sliced`, the sliced indices are fixed to the values of `slice_id`
    (mixed radix, first sliced index most significant)."""
    from tn_inputs.network import Network, Tree

    n = net.n_leaves
    left = [int(x) for x in tree.left]
    right = [int(x) for x in tree.right]

    def leaves_under(v):
        if v < n:
            return [v]
        return leaves_under(left[v - n]) + leaves_under(right[v - n])

    below = leaves_under(node)
    inside = set(below)
    val = {}
    if sliced:
        sid = int(slice_id)
        for e in reversed(list(sliced)):
            val[e] = sid % net.idx_dim[e]
            sid //= net.idx_dim[e]
    count_in, count_out = {}, {}
    for v, ix in enumerate(net.leaf_idx):
        for e in ix:
            d = count_in if v in inside else count_out
            d[e] = d.get(e, 0) + 1
    outs = set(net.out_idx)
    kept = sorted(e for e in count_in if e not in val and (e in outs or e in count_out))
    leaves, idx = [], []
    for v in below:
        t = np.asarray(net.leaves[v])
        ix = list(net.leaf_idx[v])
        for e in [e for e in ix if e in val]:
            t = np.take(t, val[e], axis=ix.index(e))
            ix.remove(e)
        leaves.append(t)
        idx.append(ix)
    remap = {}
    for ix in idx:
        for e in ix:
            remap.setdefault(e, len(remap))
    sub = Network(leaves, [[remap[e] for e in ix] for ix in idx], [net.idx_dim[e] for e in sorted(remap, key=remap.get)],
                  [remap[e] for e in kept])
    # the subtree's internal nodes in SSA order, renumbered
    order = {}
    for k, v in enumerate(below):
        order[v] = k
    sl, sr = [], []

    def build(v):
        if v < n:
            return order[v]
        a, b = build(left[v - n]), build(right[v - n])
        sl.append(a)
        sr.append(b)
        return len(below) + len(sl) - 1

    build(node)
    sub_tree = Tree(np.array(sl, np.int32), np.array(sr, np.int32))
    return contract(sub, sub_tree), kept


def root_condition(net, tree, sliced=(), slice_ids=None):
    """kappa = sum over slices of ||T_l|| * ||T_r|| / ||R||, for the root's two
    children T_l, T_r and the result R: the factor by which relative
    perturbations of the last pairwise contraction's inputs can grow in its
    output (||l . r|| <= ||l|| ||r||)."""
    n = net.n_leaves
    root = 2 * n - 2
    l, r = int(tree.left[-1]), int(tree.right[-1])
    ids = list(range(int(np.prod([net.idx_dim[e] for e in sliced], dtype=np.int64)))) if slice_ids is None else list(slice_ids)
    if not sliced:
        ids = [None]
    num = 0.0
    for s in ids:
        a, _ = subtree_value(net, tree, l, sliced, s)
        b, _ = subtree_value(net, tree, r, sliced, s)
        num += float(np.linalg.norm(a)) * float(np.linalg.norm(b))
    R = contract(net, tree, sliced=sliced, slice_ids=None if slice_ids is None else slice_ids)
    del root
    return num / float(np.linalg.norm(R))
