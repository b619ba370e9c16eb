"""Many independent networks in one graph launch (tn_batch): every network's
result against the oracle, per network.  Workloads: the QAOA energy terms
(Sec. 4.5; one light-cone network per edge), including the full-size
instance (N = 54, p = 3, 81 terms), and a mixed batch of random networks with
open outputs, hyperedges and dimension-4 indices whose larger contractions
(split-K rows and GEMMs) run between the interpreter's launches.  complex128
within 1e-10, complex64 within 1e-5 of the oracle on the same complex64
leaves; repeated calls and a second workspace give bitwise the same values."""

import numpy as np
import pytest

from tests.gpu_util import TOL_C64, TOL_C128, c64_leaves, note, rel, to_dev
from tn_inputs.graphs import random_network
from tn_inputs.greedy import find_tree
from tn_inputs.qaoa import instance, term_network

pytestmark = pytest.mark.gpu


def _run_batch(nets, trees, prec, oracle_lib, check_repeat=True):
    import torch

    from paper_2002_01935_amd.binding import Batch, Plan
    plans = [Plan(n, t, precision=prec) for n, t in zip(nets, trees)]
    batch = Batch(plans)
    info = batch.info()
    note("batch", prec, "networks", len(nets), info)
    ws = batch.workspace()
    batch.prepare(ws)
    leaves = [to_dev(n, prec) for n in nets]
    outs = batch.contract(leaves, ws)
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o in outs]
    tol = TOL_C128 if prec == "c128" else TOL_C64
    worst = 0.0
    for i, (n, t, g) in enumerate(zip(nets, trees, got)):
        ref = oracle_lib.contract(n if prec == "c128" else c64_leaves(n), t)
        e = rel(g, ref)
        worst = max(worst, e)
        assert g.shape == ref.shape, i
        assert e < tol, (i, e)
    note("batch", prec, "worst rel err over networks %.3e" % worst)
    if check_repeat:
        again = [o.cpu().numpy() for o in batch.contract(leaves, ws)]
        ws2 = batch.workspace()
        batch.prepare(ws2)
        other = [o.cpu().numpy() for o in batch.contract(leaves, ws2)]
        torch.cuda.synchronize()
        for a, b, c in zip(got, again, other):
            assert np.array_equal(a, b) and np.array_equal(a, c)
    return got, info


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
@pytest.mark.parametrize("n,p,seed", [(10, 2, 0), (16, 1, 3)])
def test_qaoa_terms_batched(oracle_lib, n, p, seed, prec):
    edges, gammas, betas = instance(n, p, seed)
    nets = [term_network(edges, gammas, betas, j, k) for j, k in edges]
    trees = [find_tree(net, seed=0, trials=2) for net in nets]
    _run_batch(nets, trees, prec, oracle_lib)


def test_qaoa_full_size_batched(oracle_lib):
    """N = 54, p = 3: 81 terms, widths 12-20, in one graph launch."""
    edges, gammas, betas = instance(54, 3, 0)
    nets = [term_network(edges, gammas, betas, j, k) for j, k in edges]
    trees = [find_tree(net, seed=0, trials=4) for net in nets]
    got, info = _run_batch(nets, trees, "c64_4m", oracle_lib, check_repeat=False)
    assert info["launches"] < sum(len(n.leaves) for n in nets) // 10
    energy = sum(complex(np.asarray(g).ravel()[0]).real for g in got)
    note("batched full-size energy", energy)


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
def test_mixed_networks_batched(oracle_lib, prec):
    """Networks of different sizes in one batch: the small ones entirely in
    the interpreter, the larger ones with split-K and GEMM contractions
    between its launches (more than one level)."""
    nets, trees = [], []
    for i in range(6):
        net = random_network(9 + i, 14 + 2 * i, 4, seed=500 + i, n_out=2, dims=(2, 4), hyper=True)
        nets.append(net)
        trees.append(find_tree(net, seed=i, trials=2))
    from tn_inputs.circuits import circuit_network
    for i, (r, c) in enumerate([(4, 4), (4, 5)]):
        net = circuit_network(r, c, 10, 20 + i, 0b1011001110100101 >> i, open_qubits=(5,))
        nets.append(net)
        trees.append(find_tree(net, seed=0, trials=2))
    got, info = _run_batch(nets, trees, prec, oracle_lib)
    assert info["levels"] >= 2, info
