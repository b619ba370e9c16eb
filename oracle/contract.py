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
