"""Several host threads on one plan (the concurrency contract of include/tn.h):
each thread has its own workspace and stream; forward contractions, reverse
passes over two different leaf sets (which rebuild the plan's reverse program
and drop its cached graphs) and more workspaces than the graph cache holds
(evictions) run at the same time.  Every result must be bitwise equal to the
same call made alone on one thread.  Slices are independent (Sec. 4.7.1), so
nothing but the plan's shared state couples the threads."""

import threading

import numpy as np
import pytest

from tests.gpu_util import note, to_dev
from tn_inputs.circuits import circuit_network, gate_leaves
from tn_inputs.greedy import find_tree

pytestmark = pytest.mark.gpu


def _case():
    net = circuit_network(4, 4, 10, 3, 0b1011001110100101, open_qubits=(5, 10))
    tree = find_tree(net, seed=1, trials=4, slice_width=12)
    return net, tree, list(tree.meta["sliced"])


def test_threads_share_one_plan():
    import torch

    from paper_2002_01935_amd.binding import Plan

    net, tree, sl = _case()
    plan = Plan(net, tree, sliced=sl, precision="c64_4m", max_inflight_slices=2)
    leaves = to_dev(net, "c64_4m")
    d = plan.info()["d_sliced"]
    wrt_sets = [gate_leaves(net, "2q")[:6], gate_leaves(net, "2q")[6:9]]
    go = torch.tensor(np.linspace(0.2, 1.0, 4).reshape(2, 2) * (1 - 0.5j), dtype=torch.complex128)

    # references: each call alone, on the default stream
    ref_fwd = {}
    for i in range(4):
        ids = list(range(i, d, 4))
        ref_fwd[i] = plan.contract_sliced(leaves, slice_ids=ids).cpu().numpy()
    ref_bwd = {}
    for j, w in enumerate(wrt_sets):
        ref_bwd[j] = [g.cpu().numpy() for g in plan.backward(leaves, go, w)]
    torch.cuda.synchronize()
    note("threads: d_sliced", d, "references done")

    errors = []
    results = {}

    def worker(tid):
        try:
            s = torch.cuda.Stream()
            # per-thread workspaces, more of them in total than the plan's graph
            # cache holds, so graphs are evicted while other threads launch
            ws_f = [plan.workspace(stream=s) for _ in range(3)]
            ws_b = plan.workspace(max(plan.backward_info(w)["workspace_bytes"] for w in wrt_sets), stream=s)
            out = []
            for it in range(6):
                i = (tid + it) % 4
                ids = list(range(i, d, 4))
                r = plan.contract_sliced(leaves, slice_ids=ids, workspace=ws_f[it % 3], stream=s)
                j = (tid + it) % 2
                g = plan.backward(leaves, go, wrt_sets[j], workspace=ws_b, stream=s)
                s.synchronize()
                out.append((i, r.cpu().numpy(), j, [x.cpu().numpy() for x in g]))
            results[tid] = out
        except Exception as e:  # reported by the main thread
            errors.append((tid, repr(e)))

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    n = 0
    for tid, out in results.items():
        for i, r, j, g in out:
            assert np.array_equal(r, ref_fwd[i]), (tid, i)
            for a, b in zip(g, ref_bwd[j]):
                assert np.array_equal(a, b), (tid, j)
            n += 1
    note("threads: compared", n, "forward + reverse results bitwise")
    assert n == 4 * 6
