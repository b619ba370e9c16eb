"""Thin ctypes binding of libtn (include/tn.h): argument marshalling only.

Every step of a contraction runs in libtn's HIP kernels.  PyTorch supplies
device memory (leaves, outputs, gradients, workspace) and the stream
(torch.cuda.current_stream()).  If libtn.so is missing this module raises on
import: there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np
# torch first: it carries its own HIP / HSA runtime libraries, and libtn.so must
# bind to the HIP runtime torch has loaded (one runtime per process); loading
# libtn.so first would bring in a second HSA runtime that finds no device.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtn.so")

TN_C64_4M, TN_C64_3M, TN_C64_BF16X3, TN_C128 = 0, 1, 2, 3
TN_FLAG_GEMM_ALL_SIZES = 1
PRECISIONS = {"c64_4m": TN_C64_4M, "c64_3m": TN_C64_3M, "c64_bf16x3": TN_C64_BF16X3, "c128": TN_C128}
KERNEL_CLASSES = {0: "row", 1: "splitk", 2: "gemm", 3: "gemm_splitk"}

EXPORTS = [
    "tn_plan", "tn_plan_info", "tn_plan_backward_info", "tn_plan_num_nodes", "tn_plan_node_info",
    "tn_plan_tune", "tn_contract", "tn_contract_sliced", "tn_contract_backward", "tn_plan_destroy",
    "tn_last_error", "tn_contract_sliced_timed", "tn_plan_set_tile", "tn_plan_node_kernel",
    "tn_plan_tune_trials", "tn_contract_sliced_noalloc", "tn_batch", "tn_batch_info", "tn_batch_prepare",
    "tn_batch_contract", "tn_batch_destroy", "tn_plan_backward_kernels",
]
OP_KINDS = {0: "row", 1: "splitk", 2: "reduce", 3: "gemm", 4: "accum", 5: "permute", 6: "counter", 7: "split"}


class TNError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libtn error {code}: {msg}")
        self.code = code


class _Options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("max_inflight_slices", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("workspace_cap", ctypes.c_uint64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2002_01935_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.tn_plan.argtypes = [i32, P, P, i32, P, i32, P, P, P, i32, P, P, ctypes.POINTER(P)]
    lib.tn_plan_info.argtypes = [P, P, P, P, P, P, P]
    lib.tn_plan_backward_info.argtypes = [P, i32, P, P, P]
    lib.tn_plan_num_nodes.argtypes = [P, P]
    lib.tn_plan_node_info.argtypes = [P, i32, P, P, P, P, P, P, P]
    lib.tn_plan_tune.argtypes = [P, P, u64, P]
    lib.tn_plan_set_tile.argtypes = [P, i32, P]
    lib.tn_contract.argtypes = [P, P, P, P, u64, P]
    lib.tn_contract_sliced.argtypes = [P, P, i64, P, P, P, u64, P]
    lib.tn_contract_backward.argtypes = [P, P, P, i32, P, P, i64, P, P, u64, P]
    lib.tn_contract_sliced_timed.argtypes = [P, P, i64, P, P, P, u64, P, i32, P, P, P, P, P, P]
    lib.tn_plan_node_kernel.argtypes = [P, i32, P, ctypes.c_char_p, i32]
    lib.tn_plan_backward_kernels.argtypes = [P, i32, P, i32, P, ctypes.c_char_p, i32]
    lib.tn_plan_tune_trials.argtypes = [P, i32, P, P, P, P, P]
    lib.tn_contract_sliced_noalloc.argtypes = [P, P, i64, P, P, P]
    lib.tn_batch.argtypes = [i32, P, ctypes.POINTER(P)]
    lib.tn_batch_info.argtypes = [P, P, P, P, P]
    lib.tn_batch_prepare.argtypes = [P, P, u64, P]
    lib.tn_batch_contract.argtypes = [P, P, P, P, u64, P]
    lib.tn_batch_destroy.argtypes = [P]
    lib.tn_batch_destroy.restype = None
    lib.tn_plan_destroy.argtypes = [P]
    lib.tn_plan_destroy.restype = None
    lib.tn_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("tn_plan_destroy", "tn_last_error", "tn_batch_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


lib = _load()


def _check(rc):
    if rc != 0:
        raise TNError(rc, lib.tn_last_error().decode())


def _arr(a, dtype):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    return a, (a.ctypes.data_as(ctypes.c_void_p) if a.size else None)


def _stream(stream):
    """A torch.cuda.Stream, a raw hipStream_t handle (int), or None for the
    current stream."""
    if stream is not None:
        return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _on_stream(stream, make):
    """Run `make()` (a torch allocation) with `stream` current, so that the
    caching allocator ties the new tensor to the stream the library enqueues
    its work on; None = the current stream."""
    if stream is None or not hasattr(stream, "cuda_stream"):
        if stream is not None:
            raise ValueError("pass a torch.cuda.Stream, or preallocate every buffer for a raw stream handle")
        return make()
    with torch.cuda.stream(stream):
        return make()


def _dev_ptrs(tensors):
    return (ctypes.c_void_p * max(1, len(tensors)))(*[t.data_ptr() for t in tensors])


class Plan:
    """A compiled contraction plan (tn_plan).  `net` needs .flat() -> (rank,
    leaf_idx, idx_dim, out_idx) and n_leaves / n_idx; `tree` needs .left and
    .right (SSA pairs, leaves first)."""

    def __init__(self, net, tree, sliced=(), precision="c64_4m", max_inflight_slices=0,
                 workspace_cap=0, autotune=False, gemm_all_sizes=False):
        rank, leaf_idx, idx_dim, out_idx = net.flat()
        self.n_leaves = int(len(rank))
        self.out_shape = tuple(int(idx_dim[e]) for e in out_idx)
        self.leaf_shapes = []
        off = 0
        for r in rank:
            self.leaf_shapes.append(tuple(int(idx_dim[e]) for e in leaf_idx[off:off + r]))
            off += r
        self.precision = precision
        self.prec = PRECISIONS[precision]
        keep = []
        args = []
        for a, dt in ((rank, np.int32), (leaf_idx, np.int64), (idx_dim, np.int64), (out_idx, np.int64),
                      (tree.left, np.int32), (tree.right, np.int32), (list(sliced), np.int64)):
            arr, ptr = _arr(a, dt)
            keep.append(arr)
            args.append(ptr)
        flags = TN_FLAG_GEMM_ALL_SIZES if gemm_all_sizes else 0
        opt = _Options(self.prec, int(bool(autotune)), int(max_inflight_slices), flags, int(workspace_cap))
        handle = ctypes.c_void_p()
        _check(lib.tn_plan(self.n_leaves, args[0], args[1], int(len(idx_dim)), args[2], int(len(out_idx)),
                           args[3], args[4], args[5], int(len(keep[6])), args[6], ctypes.byref(opt),
                           ctypes.byref(handle)))
        self.handle = handle
        self.sliced = list(sliced)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:   # lib is None during interpreter shutdown
            lib.tn_plan_destroy(h)
            self.handle = None

    @property
    def storage_dtype(self):
        import torch
        return torch.complex128 if self.prec == TN_C128 else torch.complex64

    def info(self) -> dict:
        W, Ws = ctypes.c_int32(), ctypes.c_int32()
        lc, fl = ctypes.c_double(), ctypes.c_double()
        d, ws = ctypes.c_int64(), ctypes.c_uint64()
        _check(lib.tn_plan_info(self.handle, ctypes.byref(W), ctypes.byref(Ws), ctypes.byref(lc),
                                ctypes.byref(fl), ctypes.byref(d), ctypes.byref(ws)))
        return dict(W=W.value, W_s=Ws.value, log2_C=lc.value, flops_per_slice=fl.value,
                    d_sliced=d.value, workspace_bytes=ws.value)

    def backward_info(self, wrt) -> dict:
        w, wp = _arr(list(wrt), np.int32)
        ws, fl = ctypes.c_uint64(), ctypes.c_double()
        _check(lib.tn_plan_backward_info(self.handle, len(w), wp, ctypes.byref(ws), ctypes.byref(fl)))
        return dict(workspace_bytes=ws.value, flops_per_slice=fl.value)

    def backward_kernels(self, wrt) -> list:
        """Kernel names of the reverse program's contractions for leaves `wrt`,
        in program order (tn_plan_backward_kernels)."""
        w, wp = _arr(list(wrt), np.int32)
        n = ctypes.c_int32()
        _check(lib.tn_plan_backward_kernels(self.handle, len(w), wp, 0, ctypes.byref(n), None, 0))
        cap, width = n.value, 96
        buf = ctypes.create_string_buffer(max(cap, 1) * width)
        _check(lib.tn_plan_backward_kernels(self.handle, len(w), wp, cap, ctypes.byref(n), buf, width))
        raw = buf.raw
        return [raw[i * width:(i + 1) * width].split(b"\0", 1)[0].decode() for i in range(min(cap, n.value))]

    def nodes(self) -> list:
        n = ctypes.c_int32()
        _check(lib.tn_plan_num_nodes(self.handle, ctypes.byref(n)))
        out = []
        for k in range(n.value):
            vals = [ctypes.c_int32() for _ in range(5)] + [ctypes.c_double(), ctypes.c_double()]
            _check(lib.tn_plan_node_info(self.handle, k, *[ctypes.byref(v) for v in vals]))
            kc, h, m, nn, kk, fl, by = [v.value for v in vals]
            tile = ctypes.c_int32()
            name = ctypes.create_string_buffer(96)
            _check(lib.tn_plan_node_kernel(self.handle, k, ctypes.byref(tile), name, len(name)))
            out.append(dict(kclass=KERNEL_CLASSES[kc], logH=h, logM=m, logN=nn, logK=kk, flops=fl, bytes=by,
                            tile=tile.value, kernel=name.value.decode()))
        return out

    def tune_trials(self) -> list:
        """Autotune trials of the last tune(): shape (h, m, n, k, split bits,
        direct-to-LDS eligible), tile, log2 of the trial's summed range and
        the median time in ms."""
        n = ctypes.c_int32()
        _check(lib.tn_plan_tune_trials(self.handle, 0, ctypes.byref(n), None, None, None, None))
        cap = n.value
        keys = np.zeros(6 * max(cap, 1), np.int32)
        tiles = np.zeros(max(cap, 1), np.int32)
        kb = np.zeros(max(cap, 1), np.int32)
        ms = np.zeros(max(cap, 1), np.float32)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(lib.tn_plan_tune_trials(self.handle, cap, ctypes.byref(n), vp(keys), vp(tiles), vp(kb), vp(ms)))
        return [dict(shape=[int(x) for x in keys[6 * i:6 * i + 6]], tile=int(tiles[i]), k_bits=int(kb[i]),
                     ms=float(ms[i])) for i in range(min(cap, n.value))]

    # ---------------------------------------------------------------- device calls

    def _check_leaves(self, leaves):
        import torch
        if len(leaves) != self.n_leaves:
            raise ValueError(f"expected {self.n_leaves} leaves, got {len(leaves)}")
        for v, t in enumerate(leaves):
            if not t.is_cuda or not t.is_contiguous() or t.dtype != self.storage_dtype:
                raise ValueError(f"leaf {v} must be a contiguous {self.storage_dtype} CUDA tensor")
            if tuple(t.shape) != self.leaf_shapes[v] and t.numel() != int(np.prod(self.leaf_shapes[v], dtype=np.int64)):
                raise ValueError(f"leaf {v} has shape {tuple(t.shape)}, expected {self.leaf_shapes[v]}")
        return torch

    def workspace(self, nbytes=None, stream=None):
        n = self.info()["workspace_bytes"] if nbytes is None else int(nbytes)
        return _on_stream(stream, lambda: torch.empty(max(n, 1), dtype=torch.uint8, device="cuda"))

    def tune(self, workspace, stream=None):
        _check(lib.tn_plan_tune(self.handle, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                _stream(stream)))

    def set_tile(self, tile) -> int:
        """Pin matrix-core tile variant `tile` wherever it applies; returns the
        number of contractions changed (tn_plan_set_tile)."""
        n = ctypes.c_int32()
        _check(lib.tn_plan_set_tile(self.handle, int(tile), ctypes.byref(n)))
        return n.value

    def contract(self, leaves, out=None, workspace=None, stream=None):
        torch = self._check_leaves(leaves)
        if out is None:
            out = _on_stream(stream, lambda: torch.empty(self.out_shape, dtype=self.storage_dtype, device="cuda"))
        if workspace is None:
            workspace = self.workspace(stream=stream)
        _check(lib.tn_contract(self.handle, _dev_ptrs(leaves), ctypes.c_void_p(out.data_ptr()),
                               ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream(stream)))
        return out

    def contract_sliced(self, leaves, slice_ids=None, out=None, workspace=None, stream=None):
        torch = self._check_leaves(leaves)
        if out is None:
            out = _on_stream(stream, lambda: torch.empty(self.out_shape, dtype=torch.complex128, device="cuda"))
        if out.dtype != torch.complex128 or not out.is_contiguous():
            raise ValueError("out must be a contiguous complex128 CUDA tensor")
        if workspace is None:
            workspace = self.workspace(stream=stream)
        if slice_ids is None:
            n, ptr, keep = 0, None, None
        else:
            keep, ptr = _arr(list(slice_ids), np.int64)
            n = len(keep)
        _check(lib.tn_contract_sliced(self.handle, _dev_ptrs(leaves), n, ptr, ctypes.c_void_p(out.data_ptr()),
                                      ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream(stream)))
        return out

    def contract_sliced_noalloc(self, leaves, out, slice_ids=None, stream=None):
        """tn_contract_sliced over the library's static per-device scratch:
        no workspace, and the call allocates no device memory.  `out` is a
        caller-provided contiguous complex128 tensor; calls that overlap on
        one GPU race on the shared scratch."""
        self._check_leaves(leaves)
        if out.dtype != torch.complex128 or not out.is_contiguous() or not out.is_cuda:
            raise ValueError("out must be a contiguous complex128 CUDA tensor")
        if slice_ids is None:
            n, ptr, keep = 0, None, None
        else:
            keep, ptr = _arr(list(slice_ids), np.int64)
            n = len(keep)
        _check(lib.tn_contract_sliced_noalloc(self.handle, _dev_ptrs(leaves), n, ptr, ctypes.c_void_p(out.data_ptr()),
                                              _stream(stream)))
        return out

    def contract_sliced_timed(self, leaves, slice_ids=None, out=None, workspace=None, stream=None):
        """tn_contract_sliced run op by op with HIP events around every launch;
        returns (out, [dict(kind, node, ms, flops, bytes) per op])."""
        torch = self._check_leaves(leaves)
        if out is None:
            out = _on_stream(stream, lambda: torch.empty(self.out_shape, dtype=torch.complex128, device="cuda"))
        if workspace is None:
            workspace = self.workspace(stream=stream)
        if slice_ids is None:
            n, ptr, keep = 0, None, None
        else:
            keep, ptr = _arr(list(slice_ids), np.int64)
            n = len(keep)
        cap = 1 << 16
        ms = np.zeros(cap, np.float32)
        kind = np.zeros(cap, np.int32)
        node = np.zeros(cap, np.int32)
        fl = np.zeros(cap, np.float64)
        by = np.zeros(cap, np.float64)
        nops = ctypes.c_int32()
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(lib.tn_contract_sliced_timed(self.handle, _dev_ptrs(leaves), n, ptr, ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream(stream),
                                            cap, vp(ms), vp(kind), vp(node), vp(fl), vp(by), ctypes.byref(nops)))
        ops = [dict(kind=OP_KINDS.get(int(kind[i]), "?"), node=int(node[i]), ms=float(ms[i]), flops=float(fl[i]),
                    bytes=float(by[i])) for i in range(min(nops.value, cap))]
        return out, ops

    def backward(self, leaves, grad_out, wrt, grads=None, slice_ids=None, workspace=None, stream=None):
        torch = self._check_leaves(leaves)
        wrt = [int(v) for v in wrt]
        if grads is None:
            grads = _on_stream(stream, lambda: [torch.empty(self.leaf_shapes[v], dtype=self.storage_dtype,
                                                            device="cuda") for v in wrt])
        go = _on_stream(stream, lambda: grad_out.to(device="cuda", dtype=torch.complex128).contiguous())
        if workspace is None:
            workspace = self.workspace(self.backward_info(wrt)["workspace_bytes"], stream=stream)
        w, wp = _arr(wrt, np.int32)
        if slice_ids is None:
            n, ptr, keep = 0, None, None
        else:
            keep, ptr = _arr(list(slice_ids), np.int64)
            n = len(keep)
        _check(lib.tn_contract_backward(self.handle, _dev_ptrs(leaves), ctypes.c_void_p(go.data_ptr()), len(w), wp,
                                        _dev_ptrs(grads), n, ptr, ctypes.c_void_p(workspace.data_ptr()),
                                        workspace.numel(), _stream(stream)))
        return grads


class Batch:
    """Many unsliced plans of one precision contracted by one graph launch
    (tn_batch): tiny contractions in an interpreter kernel (one workgroup per
    network), large ones with the ordinary kernels."""

    def __init__(self, plans):
        self.plans = list(plans)   # kept for shapes and dtypes only
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        handle = ctypes.c_void_p()
        _check(lib.tn_batch(len(self.plans), arr, ctypes.byref(handle)))
        self.handle = handle

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:
            lib.tn_batch_destroy(h)
            self.handle = None

    def info(self) -> dict:
        ws, lv, nt, nl = ctypes.c_uint64(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.tn_batch_info(self.handle, ctypes.byref(ws), ctypes.byref(lv), ctypes.byref(nt), ctypes.byref(nl)))
        return dict(workspace_bytes=ws.value, levels=lv.value, tiny_ops=nt.value, launches=nl.value)

    def workspace(self, stream=None):
        n = self.info()["workspace_bytes"]
        return _on_stream(stream, lambda: torch.empty(max(n, 1), dtype=torch.uint8, device="cuda"))

    def prepare(self, workspace, stream=None):
        _check(lib.tn_batch_prepare(self.handle, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                    _stream(stream)))

    def contract(self, leaves, workspace, outs=None, stream=None):
        """leaves[j] = the leaf tensors of plan j; returns the outputs."""
        if len(leaves) != len(self.plans):
            raise ValueError(f"expected leaves of {len(self.plans)} networks")
        flat = []
        for p, ls in zip(self.plans, leaves):
            p._check_leaves(ls)
            flat.extend(ls)
        if outs is None:
            outs = [_on_stream(stream, lambda p=p: torch.empty(p.out_shape, dtype=p.storage_dtype, device="cuda"))
                    for p in self.plans]
        _check(lib.tn_batch_contract(self.handle, _dev_ptrs(flat), _dev_ptrs(outs), ctypes.c_void_p(workspace.data_ptr()),
                                     workspace.numel(), _stream(stream)))
        return outs
