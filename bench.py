#!/usr/bin/env python
"""Throughput of sliced tensor-network contraction on one MI355X.

Default workload: 54-qubit 6x9 grid circuit, 12 cycles, six open qubits (64
correlated amplitudes), tree sliced to width 30 (2^30 complex64 = 8 GiB
intermediates), complex64 with FP32 matrix cores (4M).  A step is one
tn_contract_sliced call over `--slices-per-step` seeded slice ids (FP64 sum of
their 64-amplitude roots); the whole hot path (plan, slice instantiation,
permute-fused loads, vector-ALU and matrix-core contractions, FP64 slice
accumulation, graph replay) runs in every step.

Printed as one JSON line:
  value       8 C_s / time over the timed steps (complex FLOPs, Sec. 2), TFLOP/s
  roofline    dominant kernel (the GEMM launch with the largest total time):
              algorithmic FLOPs of one launch / its average duration, timed
              with HIP events around every launch over the same number of
              steps, against the FP32 matrix-core peak (157.3 TFLOP/s)
  cpu_baseline  the CPU oracle on one sub-slice of the same tree (more
              indices sliced so that it runs in seconds), same FLOP convention,
              on all host threads and on one
  plain_fp64  the same tree and slice run node by node with materialised
              permutes and complex128 matmuls in PyTorch (one slice)
  variants    the same slices with 3M and BF16x3, each with its dominant
              launch's rate in the FLOPs its matrix cores execute
  adjoint     forward and reverse pass on cfg4 (all 180 fSim leaf gradients),
              with the oracle's forward and gradient of one sub-slice beside it

Other modes (one JSON line each): --node M,N,K [precision] [reps] (one
pairwise node), --qaoa [N] [p] [streams], --sample [n], --adjoint
[precision] (the cfg4 forward and reverse pass alone, for profiling),
--copy-calibration, --summarize-rocprof DIR.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"c64_4m": 157.3, "c64_3m": 157.3, "c64_bf16x3": 2500.0, "c128": 78.6}
# real FLOPs the matrix cores execute per 8C FLOPs of the tree: 4M and the
# vector-ALU complex128 path 1; 3M three real products (6C); BF16x3 three
# BF16 products of the 4M embedding (24C)
EXECUTED = {"c64_4m": 1.0, "c64_3m": 0.75, "c64_bf16x3": 3.0, "c128": 1.0}
KERNEL = {"c64_4m": "gemm_mfma_4m", "c64_3m": "gemm_mfma_3m", "c64_bf16x3": "gemm_mfma_bf16x3", "c128": "gemm_valu"}
WORKLOADS = {
    "cfg5": "6x9 grid circuit (54 qubits), 12 cycles, fSim(pi/2,pi/6) + sqrtX/Y/W, 6 open qubits "
            "(64 amplitudes), sliced to W_s=30, seeded slice ids",
    "cfg3": "7x7 grid circuit (49 qubits), 14 cycles, one amplitude, sliced to W_s=27, seeded slice ids",
    "cfg2": "random 3-regular graph, 120 rank-3 tensors, bond 2, sliced to W_s=20, all slices",
    "cfg4": "6x6 grid circuit (36 qubits), 12 cycles, one amplitude, W=28, unsliced",
    "cfg5h": "cfg5 circuit with every fSim written as SWAP times a diagonal gate (hyperedge wires, batched "
             "contractions), 64 amplitudes, sliced to W_s=30, seeded slice ids",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "rowops.h", "tn_internal.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_2002_01935_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, precision, workload, log2_hmnk):
    """HBM bytes per launch of the dominant kernel from the committed PMC
    record (profiles/traffic_*.json: FETCH_SIZE + WRITE_SIZE, each scaled by
    a plain copy's reading), or None when no record matches this kernel,
    node and the current kernel sources."""
    safe = "".join(c if c.isalnum() or c == "_" else "_" for c in kernel).strip("_")
    path = os.path.join(ROOT, "profiles", f"traffic_{safe}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if (rec.get("kernel") != kernel or rec.get("precision") != precision or rec.get("log2_hmnk") != log2_hmnk
            or rec.get("kernel_sources_sha256") != kernel_sources_sha256()):
        return None
    return rec["traffic_bytes_per_launch"]


def permute_any(x, perm, torch):
    """x.permute(perm).contiguous() for any rank: axes that stay adjacent are
    merged first; if more than 16 groups remain (the limit of the copy kernel
    in this PyTorch build), the permutation is applied as a sequence of
    windowed permutes (odd-even block transposition on groups of 7)."""
    shape = list(x.shape)
    target = list(perm)
    while True:
        # merge source axes that are adjacent and in order in the target
        groups = []
        for a in target:
            if groups and groups[-1][-1] + 1 == a:
                groups[-1].append(a)
            else:
                groups.append([a])
        order = sorted(range(len(groups)), key=lambda g: groups[g][0])   # source order of groups
        sizes = {g: int(math.prod(shape[a] for a in groups[g])) for g in range(len(groups))}
        y = x.reshape([sizes[g] for g in order])
        rank_in_target = {g: i for i, g in enumerate(range(len(groups)))}
        src_pos = {g: i for i, g in enumerate(order)}
        if len(groups) <= 16:
            return y.permute(*[src_pos[g] for g in range(len(groups))]).contiguous().reshape(
                [shape[a] for a in target])
        # one pass: sort windows of 14 consecutive source groups by target rank
        cur = list(order)
        for start in (0, 7):
            new = []
            i = 0
            while i < len(cur):
                if i >= start and (i - start) % 14 == 0:
                    new.extend(sorted(cur[i:i + 14], key=lambda g: rank_in_target[g]))
                    i += 14
                elif i < start:
                    new.append(cur[i])
                    i += 1
                else:
                    new.append(cur[i])
                    i += 1
            cur = new
            pre_dims = []
            # apply this window pass as permutes of at most 16 dims each
            yy = y
            i = 0
            dims = [sizes[g] for g in order]
            for w0 in range(start, len(order), 14):
                w1 = min(w0 + 14, len(order))
                win = order[w0:w1]
                want = sorted(win, key=lambda g: rank_in_target[g])
                lead = int(math.prod(dims[:w0])) if w0 else 1
                tail = int(math.prod(dims[w1:])) if w1 < len(order) else 1
                yy = yy.reshape([lead] + dims[w0:w1] + [tail])
                p = [0] + [1 + win.index(g) for g in want] + [len(win) + 1]
                yy = yy.permute(*p).contiguous()
                dims = dims[:w0] + [sizes[g] for g in want] + dims[w1:]
                order = order[:w0] + want + order[w1:]
                yy = yy.reshape(dims)
            y = yy
        # continue with the partially sorted tensor: its axes are now `order`
        x = y.reshape([shape[a] for g in order for a in groups[g]])
        shape = [shape[a] for g in order for a in groups[g]]
        flat = [a for g in order for a in groups[g]]
        target = [flat.index(a) for a in target]


def plain_fp64(net, tree, sliced, slice_id, torch):
    """Node-by-node complex128 contraction with materialised permutes and
    torch.matmul (the per-contraction baseline); returns (value, seconds)."""
    import numpy as np
    dev = "cuda"
    n = net.n_leaves
    # slice values: mixed radix, first sliced index most significant
    val = {}
    sid = slice_id
    for e in reversed(list(sliced)):
        val[e] = sid % net.idx_dim[e]
        sid //= net.idx_dim[e]
    leaves = []
    for t, ix in zip(net.leaves, net.leaf_idx):
        x = torch.from_numpy(np.ascontiguousarray(t)).to(dev, torch.complex128)
        keep = []
        for a, e in enumerate(ix):
            if e in val:
                x = x.select(len(keep), int(val[e]))
            else:
                keep.append(e)
        leaves.append((x.contiguous(), keep))
    total = {}
    for ix in net.leaf_idx:
        for e in ix:
            total[e] = total.get(e, 0) + 1
    outs = set(net.out_idx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vals = dict(enumerate(leaves))
    count = {v: {e: 1 for e in ix} for v, ix in enumerate(net.leaf_idx)}
    for k, (l, r) in enumerate(zip(tree.left, tree.right)):
        (A, ia), (B, ib) = vals.pop(int(l)), vals.pop(int(r))
        cl, cr = count.pop(int(l)), count.pop(int(r))
        c = dict(cl)
        for e, x in cr.items():
            c[e] = c.get(e, 0) + x
        kept = [e for e in ia + [e for e in ib if e not in ia] if e not in val and (e in outs or c[e] < total[e])]
        summed = [e for e in ia if e in ib and e not in kept]
        batch = [e for e in kept if e in ia and e in ib]
        ma = [e for e in ia if e not in ib]
        nb = [e for e in ib if e not in ia]
        d = lambda es: int(math.prod(net.idx_dim[e] for e in es))  # noqa: E731
        Ap = permute_any(A, [ia.index(e) for e in batch + ma + summed], torch).reshape(d(batch), d(ma), d(summed))
        Bp = permute_any(B, [ib.index(e) for e in batch + summed + nb], torch).reshape(d(batch), d(summed), d(nb))
        Cm = torch.matmul(Ap, Bp)
        order = batch + ma + nb
        Cm = Cm.reshape([net.idx_dim[e] for e in order]) if order else Cm.reshape(())
        vals[n + k] = (Cm, order)
        count[n + k] = {e: c[e] for e in order}
    (R, ir), = vals.values()
    R = permute_any(R, [ir.index(e) for e in net.out_idx], torch) if net.out_idx else R
    torch.cuda.synchronize()
    return R.cpu().numpy(), time.perf_counter() - t0


def summarize_rocprof(path):
    """Summary of rocprofv3 output under `path` (rocpd SQLite databases, or CSV
    files from --output-format csv): per (kernel, grid) group the dispatch
    count and mean / min / total duration from the kernel trace, and the
    per-dispatch mean of every PMC counter found (FETCH_SIZE, WRITE_SIZE in
    KiB).  Prints text for profiles/."""
    import csv
    import glob
    import sqlite3
    from collections import defaultdict

    def short(name):
        return name.split("(")[0].replace("void ", "").replace("tn::", "")[:70]

    trace = defaultdict(list)
    pmc = defaultdict(lambda: defaultdict(list))
    longest = []
    for f in sorted(glob.glob(os.path.join(path, "**", "*.db"), recursive=True)):
        con = sqlite3.connect(f)
        tabs = {r[0] for r in con.execute("select name from sqlite_master where type in ('table', 'view')")}
        if "kernels" in tabs:
            for name, gx, gy, gz, wx, dur in con.execute(
                    "select name, grid_x, grid_y, grid_z, workgroup_x, duration from kernels"):
                trace[(short(name), (gx, gy, gz, wx))].append(dur / 1e6)
            # the longest dispatches, with their counters when this is a PMC run
            for did, name, dur in con.execute(
                    "select dispatch_id, name, duration from kernels order by duration desc limit 6"):
                cs = {}
                if "counters_collection" in tabs:
                    for cname, val in con.execute(
                            "select counter_name, value from counters_collection where dispatch_id = ?", (did,)):
                        cs[cname] = float(val)
                longest.append((short(name), dur / 1e6, cs))
        if "counters_collection" in tabs:
            for name, gx, gy, gz, wx, cname, val in con.execute(
                    "select kernel_name, grid_size_x, grid_size_y, grid_size_z, workgroup_size_x, counter_name, value "
                    "from counters_collection"):
                pmc[(short(name), (gx, gy, gz, wx))][cname].append(float(val))
        con.close()
    for f in sorted(glob.glob(os.path.join(path, "**", "*kernel_trace.csv"), recursive=True)):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                g = tuple(int(r[k]) for k in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Workgroup_Size_X"))
                trace[(short(r["Kernel_Name"]), g)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
    for f in sorted(glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                g = tuple(int(r[k]) for k in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Workgroup_Size_X"))
                pmc[(short(r["Kernel_Name"]), g)][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = []
    if trace:
        total = sum(sum(v) for v in trace.values())
        out.append(f"kernel trace: {sum(len(v) for v in trace.values())} dispatches, {total:.1f} ms total")
        # `long` = dispatches within 10 % of the group's longest: the full-size
        # launches, apart from shortened ones of the same kernel and grid
        # (autotune trials run with the summed range cut)
        out.append(f"{'kernel':52s} {'grid x,y,z / wg':26s} {'calls':>6s} {'mean ms':>10s} {'min ms':>10s} "
                   f"{'total ms':>10s} {'share':>6s} {'long n':>6s} {'long mean':>10s}")
        for (k, g), v in sorted(trace.items(), key=lambda kv: -sum(kv[1]))[:30]:
            gs = f"{g[0]},{g[1]},{g[2]}/{g[3]}"
            lv = [x for x in v if x >= 0.9 * max(v)]
            out.append(f"{k[:52]:52s} {gs:26s} {len(v):6d} {sum(v) / len(v):10.3f} {min(v):10.3f} "
                       f"{sum(v):10.1f} {sum(v) / total:6.1%} {len(lv):6d} {sum(lv) / len(lv):10.3f}")
        fam = defaultdict(lambda: [0, 0.0])
        for (k, g), v in trace.items():
            f = fam[k.split("<")[0]]
            f[0] += len(v)
            f[1] += sum(v)
        out.append("by kernel (all template arguments and grids): " + "; ".join(
            f"{k} {n} calls {t:.1f} ms" for k, (n, t) in sorted(fam.items(), key=lambda kv: -kv[1][1])))
    if pmc:
        out.append("PMC counters (mean per dispatch, KiB for FETCH_SIZE / WRITE_SIZE):")
        agg = []
        for (k, g), cs in pmc.items():
            agg.append(((k, g), {c: sum(v) / len(v) for c, v in cs.items()}, max(len(v) for v in cs.values())))
        for (k, g), cs, n in sorted(agg, key=lambda a: -sum(a[1].values()))[:30]:
            vals = "  ".join(f"{c}={v:.6g}" for c, v in sorted(cs.items()))
            gs = f"{g[0]},{g[1]},{g[2]}/{g[3]}"
            out.append(f"{k[:52]:52s} {gs:26s} n={n:4d}  {vals}")
    if longest:
        out.append("longest dispatches (ms, counters of that dispatch):")
        for name, ms, cs in sorted(longest, key=lambda x: -x[1]):
            vals = "  ".join(f"{c}={v:.6g}" for c, v in sorted(cs.items()))
            out.append(f"{name[:52]:52s} {ms:10.3f}  {vals}")
    print("\n".join(out))


def copy_calibration():
    """A plain device copy of 1 GiB (read 1 GiB, write 1 GiB): run under
    rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE to scale those counters."""
    import torch
    x = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": x.numel() * 4, "dispatches": 3}))


def adjoint_bench(precision, torch, np, Plan, configs, reps=3, cpu_threads=0):
    """Reverse mode on cfg4 (6x6 grid, 12 cycles, width 28): the amplitude c,
    then dL/dconj(G) of L = |c|^2 for all 180 fSim leaves through
    tn_contract_backward (recomputation from checkpoints).  Times are medians of
    `reps` warm calls; FLOPs are the planner's 8C counts of the forward and of
    the backward program (recomputation included).  With `cpu_threads`, the
    complex128 oracle's forward and gradient of one sub-slice (8 more sliced
    indices) are timed too, and scaled by the number of sub-slices to the
    whole gradient (an extrapolation: every sub-slice has the same cost)."""
    from tn_inputs.circuits import gate_leaves
    net, tree, sliced = configs.load("cfg4")
    plan = Plan(net, tree, sliced=sliced, precision=precision)
    wrt = gate_leaves(net, "2q")
    binfo = plan.backward_info(wrt)
    ws = plan.workspace(max(binfo["workspace_bytes"], plan.info()["workspace_bytes"]))
    plan.tune(ws)
    leaves = [torch.from_numpy(np.ascontiguousarray(t)).to("cuda", plan.storage_dtype) for t in net.leaves]
    grads = [torch.empty(plan.leaf_shapes[v], dtype=plan.storage_dtype, device="cuda") for v in wrt]
    out = torch.empty(plan.out_shape, dtype=torch.complex128, device="cuda")
    tf, tb = [], []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = plan.contract_sliced(leaves, out=out, workspace=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plan.backward(leaves, (2 * c).reshape(()), wrt, grads=grads, workspace=ws)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if r:
            tf.append(t1 - t0)
            tb.append(t2 - t1)
    f_fl = plan.info()["flops_per_slice"] * plan.info()["d_sliced"]
    b_fl = binfo["flops_per_slice"] * plan.info()["d_sliced"]
    tfm, tbm = sorted(tf)[len(tf) // 2], sorted(tb)[len(tb) // 2]
    res = {"workload": "cfg4: 6x6 grid circuit, 12 cycles, one amplitude, W=28; d|amp|^2/d(all 180 fSim leaves)",
           "precision": precision, "forward_s": round(tfm, 4), "backward_s": round(tbm, 4),
           "forward_tflops": round(f_fl / tfm / 1e12, 2), "backward_tflops": round(b_fl / tbm / 1e12, 2),
           "backward_over_forward_flops": round(b_fl / f_fl, 2), "n_grads": len(wrt)}
    if cpu_threads:
        from oracle import contract as oc
        from tn_inputs.slicing import extend_slices
        ext = extend_slices(net, tree, sliced, 33.0)
        _, lc = oc.width_cost(net, tree, sliced=ext)
        t0 = time.perf_counter()
        oc.contract(net, tree, sliced=ext, slice_ids=[0], n_threads=cpu_threads)
        t1 = time.perf_counter()
        oc.grad(net, tree, np.array(1.0 + 0j), wrt, sliced=ext, slice_ids=[0], n_threads=cpu_threads)
        t2 = time.perf_counter()
        n_sub = 2 ** len(ext)
        res["cpu_oracle"] = {
            "kind": "oracle", "cores": cpu_threads, "forward_s": round(t1 - t0, 2), "gradient_s": round(t2 - t1, 2),
            "sample": f"one sub-slice of {n_sub} ({len(ext) - len(sliced)} extra sliced indices, forward "
                      f"8C = {8 * 2 ** lc:.3e}), complex128",
            "extrapolated_forward_plus_gradient_s": round((t2 - t0) * n_sub, 1)}
    return res


def node_bench(spec, precision, reps):
    """One pairwise contraction node, A[M][K] x B[N][K] -> C[M][N] (binary
    indices, canonical layouts, seeded complex normal entries), timed per
    launch with HIP events through tn_contract_sliced_timed: the dominant
    GEMM shape of a workload in isolation, for kernel profiles."""
    import numpy as np
    import torch

    from paper_2002_01935_amd.binding import Plan
    from tn_inputs.network import Network, Tree
    m, n, k = (int(x) for x in spec.split(","))
    M, K, N = list(range(m)), list(range(m, m + k)), list(range(m + k, m + k + n))
    g = torch.Generator().manual_seed(0)
    a = torch.randn(2 ** (m + k), dtype=torch.complex64, generator=g).numpy().reshape([2] * (m + k))
    b = torch.randn(2 ** (n + k), dtype=torch.complex64, generator=g).numpy().reshape([2] * (n + k))
    net = Network([a, b], [M + K, N + K], [2] * (m + n + k), M + N)
    tree = Tree(np.array([0], np.int32), np.array([1], np.int32))
    plan = Plan(net, tree, precision=precision)
    ws = plan.workspace()
    leaves = [torch.from_numpy(np.ascontiguousarray(t)).to("cuda", plan.storage_dtype) for t in net.leaves]
    out = torch.empty(plan.out_shape, dtype=torch.complex128, device="cuda")
    node = plan.nodes()[0]
    # the operands are leaves, which tn_plan_tune does not time: every tile
    # variant that applies is timed here instead
    per_tile = {}
    best = None
    for t in (range(15) if node["kclass"].startswith("gemm") else [0]):
        if t == 4 or (t and plan.set_tile(t) == 0 and t != 0):
            continue
        if t == 0:
            plan.set_tile(0)
        plan.contract_sliced_timed(leaves, out=out, workspace=ws)
        tbest = None
        for _ in range(reps):
            _, ops = plan.contract_sliced_timed(leaves, out=out, workspace=ws)
            # the contraction's own kernels (split-K includes its reduction),
            # not the FP64 accumulation of the root into the output
            cops = [o for o in ops if o["kind"] in ("row", "splitk", "reduce", "gemm", "split")]
            op = dict(max(cops, key=lambda o: o["flops"]), ms=sum(o["ms"] for o in cops))
            tbest = op if tbest is None or op["ms"] < tbest["ms"] else tbest
        per_tile[t] = round(tbest["ms"], 4)
        if best is None or tbest["ms"] < best[1]["ms"]:
            best = (t, tbest)
    t, best = best
    print(json.dumps({"mode": "node", "shape_mnk": [m, n, k], "precision": precision, "kernel_class": node["kclass"],
                      "kernel": best["kind"], "kernel_name": plan.nodes()[0].get("kernel"), "tile": t,
                      "ms": round(best["ms"], 4),
                      "tflops": round(best["flops"] / best["ms"] / 1e9, 2),
                      "gbs": round(best["bytes"] / best["ms"] / 1e6, 1), "ms_per_tile": per_tile, "reps": reps}))


def sampling_bench(n_samples):
    """Sampling driver (Sec. 4.7.3) on a 6x6 grid circuit, 12 cycles, with the
    central 2x3 block of qubits open (64 amplitudes per contraction): samples
    from psi at fidelity 1, one sliced contraction each (tree sliced to width
    28); prints the time per contraction and the projected time of 10^6
    samples at f = 0.002 (f M contractions)."""
    import numpy as np
    import torch

    from paper_2002_01935_amd.binding import Plan
    from paper_2002_01935_amd.sampling import CircuitSampler
    from tn_inputs.circuits import circuit_network, gate_leaves
    from tn_inputs.greedy import find_tree
    R, C, m = 6, 6, 12
    opened = (14, 15, 16, 20, 21, 22)
    net = circuit_network(R, C, m, 0, 0, open_qubits=opened)
    tree = find_tree(net, seed=0, trials=8, slice_width=28)
    plan = Plan(net, tree, sliced=tree.meta["sliced"], precision="c64_4m")
    ws = plan.workspace()
    plan.tune(ws)
    leaves = [torch.from_numpy(np.ascontiguousarray(t)).to("cuda", plan.storage_dtype) for t in net.leaves]
    closed = [q for q in range(R * C) if q not in opened]
    sampler = CircuitSampler(plan, leaves, R * C, closed, opened, gate_leaves(net, "out"), workspace=ws)
    sampler.conditional(0)                    # first call captures the graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    samples, nc = sampler.sample(n_samples, 1.0, np.random.default_rng(0))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    info = plan.info()
    per = el / max(nc, 1)
    print(json.dumps({"mode": "sample", "workload": "6x6 grid circuit, 12 cycles, qubits 14-16 and 20-22 open, "
                      "sliced to W_s=28", "W": info["W"], "W_s": info["W_s"], "d_sliced": info["d_sliced"],
                      "contractions": nc, "s_per_contraction": round(per, 4),
                      "tflops": round(info["flops_per_slice"] * info["d_sliced"] / per / 1e12, 2),
                      "projected_s_1e6_samples_f0.002": round(1e6 * 0.002 * per, 1),
                      "samples": [format(b, "09x") for b in samples]}))


def qaoa_bench(n, p, n_streams):
    """QAOA MAX-CUT energy (Sec. 4.5) on a seeded random 3-regular graph: one
    light-cone network per edge, each with its own tree and plan (complex64
    4M), contracted back to back on one stream, round-robin over `n_streams`
    streams (default priority, one workspace per plan), and all terms in one
    graph launch (tn_batch: tiny contractions in the interpreter kernel, one
    workgroup per term); plan by plan the many small networks are
    launch-latency bound."""
    import numpy as np
    import torch

    from paper_2002_01935_amd.binding import Plan
    from tn_inputs.greedy import find_tree
    from tn_inputs.qaoa import instance, term_network
    edges, gammas, betas = instance(n, p, 0)
    t0 = time.perf_counter()
    plans, leaves, wss, outs = [], [], [], []
    flops = 0.0
    for j, k in edges:
        net = term_network(edges, gammas, betas, j, k)
        tree = find_tree(net, seed=0, trials=4)
        pl = Plan(net, tree, precision="c64_4m")
        flops += pl.info()["flops_per_slice"]
        plans.append(pl)
        leaves.append([torch.from_numpy(np.ascontiguousarray(t)).to("cuda", pl.storage_dtype) for t in net.leaves])
        wss.append(pl.workspace())
        outs.append(torch.empty((), dtype=torch.complex64, device="cuda"))
    t_plan = time.perf_counter() - t0
    streams = [torch.cuda.Stream() for _ in range(n_streams)]

    def run(concurrent):
        for i, pl in enumerate(plans):
            s = streams[i % n_streams] if concurrent else torch.cuda.current_stream()
            with torch.cuda.stream(s):
                pl.contract(leaves[i], out=outs[i], workspace=wss[i], stream=s)
        torch.cuda.synchronize()

    res = {}
    for name, conc in (("one_stream", False), (f"{n_streams}_streams", True)):
        run(conc)                                  # captures the graphs
        ts = []
        for _ in range(3):
            t1 = time.perf_counter()
            run(conc)
            ts.append(time.perf_counter() - t1)
        res[name + "_s"] = round(sorted(ts)[1], 5)
    energy = float(sum(complex(o.item()).real for o in outs))
    # every term in one graph launch (tn_batch), on one stream
    from paper_2002_01935_amd.binding import Batch
    t0 = time.perf_counter()
    batch = Batch(plans)
    bws = batch.workspace()
    batch.prepare(bws)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t0
    bouts = batch.contract(leaves, bws)
    torch.cuda.synchronize()
    ts = []
    for _ in range(5):
        t1 = time.perf_counter()
        batch.contract(leaves, bws, outs=bouts)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t1)
    res["batched_one_stream_s"] = round(sorted(ts)[2], 5)
    binfo = batch.info()
    e_batch = float(sum(complex(o.item()).real for o in bouts))
    print(json.dumps({"mode": "qaoa", "workload": f"MAX-CUT QAOA, random 3-regular graph N={n}, p={p}, seed 0",
                      "terms": len(plans), "leaves_per_term_max": max(len(l) for l in leaves),
                      "flops_8C_total": flops, "plan_s": round(t_plan, 2), **res,
                      "batch": {"prepare_s": round(t_prep, 3), "launches_per_call": binfo["launches"],
                                "interpreter_levels": binfo["levels"], "interpreted_contractions": binfo["tiny_ops"],
                                "workspace_MiB": round(binfo["workspace_bytes"] / 2 ** 20, 1),
                                "launches_per_term_unbatched": round(sum(len(pl.nodes()) for pl in plans) / len(plans), 1)},
                      "tflops_best": round(flops / min(res.values()) / 1e12, 4), "energy": energy,
                      "energy_batched": e_batch}))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--qaoa":
        a = sys.argv[2:]
        qaoa_bench(int(a[0]) if a else 54, int(a[1]) if len(a) > 1 else 3, int(a[2]) if len(a) > 2 else 8)
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--sample":
        sampling_bench(int(sys.argv[2]) if len(sys.argv) > 2 else 3)
        return
    if len(sys.argv) > 2 and sys.argv[1] == "--node":
        prec = sys.argv[3] if len(sys.argv) > 3 else "c64_4m"
        node_bench(sys.argv[2], prec, int(sys.argv[4]) if len(sys.argv) > 4 else 3)
        return
    if len(sys.argv) > 2 and sys.argv[1] == "--summarize-rocprof":
        summarize_rocprof(sys.argv[2])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--copy-calibration":
        copy_calibration()
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--adjoint":
        import numpy as np
        import torch

        from paper_2002_01935_amd.binding import Plan
        from tn_inputs import configs
        prec = sys.argv[2] if len(sys.argv) > 2 else "c64_4m"
        print(json.dumps(adjoint_bench(prec, torch, np, Plan, configs)))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg5", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="c64_4m", choices=sorted(PEAK))
    ap.add_argument("--slices-per-step", type=int, default=None, help="default 2 (cfg3: 64)")
    ap.add_argument("--inflight", type=int, default=None,
                    help="slices contracted together per graph replay; default 1 (cfg3: 8)")
    ap.add_argument("--no-variants", action="store_true", help="skip timing the other precisions")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-timed-pass", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the cfg4 forward + backward timing")
    args = ap.parse_args()
    # cfg3's slices are small (about 26 ms each): eight share each graph
    # replay, so that its ~1100 launches per replay are spread over them
    spd, infl = {"cfg3": (64, 8)}.get(args.workload, (2, 1))
    args.slices_per_step = spd if args.slices_per_step is None else args.slices_per_step
    args.inflight = infl if args.inflight is None else args.inflight
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the sliced contraction is measured on a single MI355X "
              "(slices would shard across GPUs with one all-reduce of the result; not built here)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2002_01935_amd.binding import Plan
    from tn_inputs import configs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    net, tree, sliced = configs.load(args.workload)
    plan = Plan(net, tree, sliced=sliced, precision=args.precision, max_inflight_slices=args.inflight)
    info = plan.info()
    # seeded distinct slice ids: 256, or as many as the run contracts
    ids_all = configs.slice_subset(info["d_sliced"], seed=0,
                                   size=max(256, args.slices_per_step * (args.steps + args.warmup)))
    B = max(1, min(args.slices_per_step, len(ids_all)))
    log(f"workload {args.workload}: W={info['W']} W_s={info['W_s']} d_sliced={info['d_sliced']} "
        f"8C/slice={info['flops_per_slice']:.3e} workspace={info['workspace_bytes'] / 2**30:.1f} GiB")
    ws = plan.workspace()
    dt = plan.storage_dtype
    leaves = [torch.from_numpy(np.ascontiguousarray(t)).to("cuda", dt) for t in net.leaves]
    out = torch.empty(plan.out_shape, dtype=torch.complex128, device="cuda")
    if not args.no_tune:
        t0 = time.perf_counter()
        plan.tune(ws)
        log(f"autotune {time.perf_counter() - t0:.1f} s")

    def step_ids(s):
        return [ids_all[(s * B + j) % len(ids_all)] for j in range(B)]

    for w in range(args.warmup):
        plan.contract_sliced(leaves, slice_ids=step_ids(w), out=out, workspace=ws)
        torch.cuda.synchronize()
        log(f"warmup step {w} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        plan.contract_sliced(leaves, slice_ids=step_ids(args.warmup + s), out=out, workspace=ws)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {elapsed:.3f} s")
    n_slices = args.steps * B
    flops = info["flops_per_slice"] * n_slices
    tflops = flops / elapsed / 1e12
    per_slice = elapsed / n_slices
    n_amps = int(np.prod(plan.out_shape)) if plan.out_shape else 1

    roof = None
    if not args.no_timed_pass:
        agg = {}
        for s in range(args.steps):
            _, ops = plan.contract_sliced_timed(leaves, slice_ids=step_ids(args.warmup + s), out=out, workspace=ws)
            for i, o in enumerate(ops):
                a = agg.setdefault(i, dict(o, ms=0.0, launches=0))
                a["ms"] += o["ms"]
                a["launches"] += B
        total_ms = sum(a["ms"] for a in agg.values())
        by_kind = {}
        for a in agg.values():
            by_kind[a["kind"]] = by_kind.get(a["kind"], 0.0) + a["ms"]
        gemms = [a for a in agg.values() if a["kind"] == "gemm"]
        dom = max(gemms, key=lambda a: a["ms"])
        avg_s = dom["ms"] / 1e3 / dom["launches"]
        achieved = dom["flops"] / avg_s / 1e12
        peak = PEAK[args.precision]
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None,
                "kernel": KERNEL[args.precision],
                "node": dom["node"], "flops_per_launch": dom["flops"], "avg_launch_ms": round(avg_s * 1e3, 3),
                "time_share": round(dom["ms"] / total_ms, 4),
                "time_by_kernel_class": {k: round(v / total_ms, 4) for k, v in sorted(by_kind.items())}}
        nodes = plan.nodes()
        if 0 <= dom["node"] - net.n_leaves < len(nodes):
            nd = nodes[dom["node"] - net.n_leaves]
            roof["log2_hmnk"] = [nd["logH"], nd["logM"], nd["logN"], nd["logK"]]
            # the kernel and tile that ran, and the autotune trials of its shape
            roof["kernel"] = nd["kernel"]
            roof["tile"] = nd["tile"]
            h, m, n, k = roof["log2_hmnk"]
            # trial shapes are (h, m, n, k) of the GEMM as launched: A may be
            # either child, so m and n can appear swapped
            roof["autotune"] = [{"tile": t["tile"], "k_bits": t["k_bits"], "median_ms": round(t["ms"], 3)}
                                for t in plan.tune_trials()
                                if t["shape"][0] == h and t["shape"][3] == k and sorted(t["shape"][1:3]) == sorted([m, n])]
            roof["traffic"] = measured_traffic(nd["kernel"], args.precision, args.workload, roof["log2_hmnk"])
        log(f"dominant gemm node {dom['node']}: {avg_s * 1e3:.2f} ms/launch, {achieved:.1f} TFLOP/s")

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import contract as oc
        from tn_inputs.slicing import extend_slices
        target = 37.0
        ext = extend_slices(net, tree, sliced, target)
        _, lc = oc.width_cost(net, tree, sliced=ext)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        oc.contract(net, tree, sliced=ext, slice_ids=[0], n_threads=threads)
        tc = time.perf_counter() - t0
        cpu = {"value": round(8 * 2 ** lc / tc / 1e12, 6), "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
               "sample": f"one sub-slice of the same tree with {len(ext) - len(sliced)} extra sliced indices "
                         f"(8C = {8 * 2 ** lc:.3e} complex FLOPs) in {tc:.1f} s, complex128 loop nest"}
        log(f"cpu oracle: {cpu['value'] * 1e3:.3f} GFLOP/s on {threads} threads ({tc:.1f} s)")
        # the same oracle on one thread, on a sub-slice with a few more sliced indices
        ext1 = extend_slices(net, tree, sliced, target - 4.0)
        _, lc1 = oc.width_cost(net, tree, sliced=ext1)
        t0 = time.perf_counter()
        oc.contract(net, tree, sliced=ext1, slice_ids=[0], n_threads=1)
        tc1 = time.perf_counter() - t0
        cpu["single_thread"] = {"value": round(8 * 2 ** lc1 / tc1 / 1e12, 6), "unit": "TFLOP/s", "cores": 1,
                                "sample": f"one sub-slice with {len(ext1) - len(sliced)} extra sliced indices "
                                          f"(8C = {8 * 2 ** lc1:.3e}) in {tc1:.1f} s"}
        log(f"cpu oracle: {cpu['single_thread']['value'] * 1e3:.3f} GFLOP/s on 1 thread ({tc1:.1f} s)")
        cpu["host_cpus"] = os.cpu_count()
        try:
            cpu["cpu_model"] = next(ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo")
                                    if ln.startswith("model name"))
        except (OSError, StopIteration):
            pass

    plain = None
    plain_ref = None
    if not args.no_plain:
        try:
            ref, tp = plain_fp64(net, tree, sliced, ids_all[0], torch)
            plan1 = plan.contract_sliced(leaves, slice_ids=[ids_all[0]], out=out, workspace=ws).cpu().numpy()
            err = float(np.linalg.norm(plan1 - ref) / np.linalg.norm(ref))
            plain = {"s_per_slice": round(tp, 4), "speedup": round(tp / per_slice, 2),
                     "rel_err_vs_fp64_plain": err}
            if args.precision != "c128":
                # the same FP64 path on the complex64-rounded leaves the plan
                # receives: the contraction's own error, without the inputs'
                net64 = net.with_leaves([np.asarray(t).astype(np.complex64).astype(np.complex128)
                                         for t in net.leaves])
                ref64, _ = plain_fp64(net64, tree, sliced, ids_all[0], torch)
                plain["rel_err_vs_fp64_plain_same_leaves"] = float(np.linalg.norm(plan1 - ref64)
                                                                   / np.linalg.norm(ref64))
                plain["max_componentwise_err_same_leaves"] = float(np.abs(plan1 - ref64).max()
                                                                   / np.abs(ref64).max())
                plain["input_rounding_rel"] = float(np.linalg.norm(ref64 - ref) / np.linalg.norm(ref))
                plain_ref = ref64
            else:
                plain_ref = ref
            log(f"plain fp64 path: {tp:.2f} s/slice, speedup {tp / per_slice:.1f}x, {plain}")
        except torch.cuda.OutOfMemoryError as e:   # the plain path materialises every permute
            plain = {"error": f"out of memory: {e}"[:200]}
        torch.cuda.empty_cache()

    variants = None
    if not args.no_variants and args.precision == "c64_4m":
        variants = {}
        del ws
        torch.cuda.empty_cache()
        for prec in ("c64_3m", "c64_bf16x3"):
            vp = Plan(net, tree, sliced=sliced, precision=prec, max_inflight_slices=args.inflight)
            vws = vp.workspace()
            vp.tune(vws)
            vp.contract_sliced(leaves, slice_ids=step_ids(0), out=out, workspace=vws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s in range(args.steps):
                vp.contract_sliced(leaves, slice_ids=step_ids(args.warmup + s), out=out, workspace=vws)
            torch.cuda.synchronize()
            ve = time.perf_counter() - t0
            rec = {"value": round(info["flops_per_slice"] * n_slices / ve / 1e12, 3), "unit": "TFLOP/s",
                   "s_per_slice": round(ve / n_slices, 4)}
            # dominant matrix-core launch of one timed step, in executed FLOPs
            _, vops = vp.contract_sliced_timed(leaves, slice_ids=step_ids(args.warmup), out=out, workspace=vws)
            vg = max((o for o in vops if o["kind"] == "gemm"), key=lambda o: o["ms"])
            vt = vg["flops"] * EXECUTED[prec] / (vg["ms"] / 1e3 / B) / 1e12
            vnd = vp.nodes()[vg["node"] - net.n_leaves]
            vshape = [vnd["logH"], vnd["logM"], vnd["logN"], vnd["logK"]]
            rec["roofline"] = {"bound": "mfma", "kernel": vnd["kernel"], "tile": vnd["tile"], "node": vg["node"],
                               "achieved": round(vt, 2), "peak": PEAK[prec], "unit": "TFLOP/s",
                               "frac": round(vt / PEAK[prec], 4), "executed_per_8C": EXECUTED[prec],
                               "avg_launch_ms": round(vg["ms"] / B, 3), "log2_hmnk": vshape,
                               "autotune": [{"tile": t["tile"], "k_bits": t["k_bits"], "median_ms": round(t["ms"], 3)}
                                            for t in vp.tune_trials()
                                            if t["shape"][0] == vshape[0] and t["shape"][3] == vshape[3]
                                            and sorted(t["shape"][1:3]) == sorted(vshape[1:3])]}
            if plain_ref is not None:
                v1 = vp.contract_sliced(leaves, slice_ids=[ids_all[0]], out=out, workspace=vws).cpu().numpy()
                rec["rel_err_vs_fp64_plain_same_leaves"] = float(np.linalg.norm(v1 - plain_ref)
                                                                 / np.linalg.norm(plain_ref))
            variants[prec] = rec
            log(f"variant {prec}: {rec}")
            del vws, vp
            torch.cuda.empty_cache()

    adjoint = None
    if not args.no_adjoint and args.precision in ("c64_4m", "c64_3m", "c64_bf16x3"):
        try:
            del ws
        except NameError:
            pass
        torch.cuda.empty_cache()
        adjoint = adjoint_bench(args.precision, torch, np, Plan, configs,
                                cpu_threads=0 if args.no_cpu_baseline else
                                int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
        log(f"adjoint (cfg4): {adjoint}")

    res = {
        "metric": "TFLOP/s on contraction tree + s/amplitude at stated error vs FP64, vs plain path",
        "value": round(tflops, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64" if args.precision != "c128" else "c128",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "precision": args.precision,
                   "slices_per_step": B, "d_sliced": info["d_sliced"], "W": info["W"], "W_s": info["W_s"],
                   "flops_8C_per_slice": info["flops_per_slice"], "amplitudes": n_amps},
        "s_per_slice": round(per_slice, 4),
        "s_per_amplitude_extrapolated": round(per_slice * info["d_sliced"] / n_amps, 4),
        "roofline": roof, "cpu_baseline": cpu, "plain_fp64": plain, "variants": variants, "adjoint": adjoint,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
