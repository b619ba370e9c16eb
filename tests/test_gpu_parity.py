"""GPU parity: libtn (HIP, gfx950) against the complex128 oracle on seeded
inputs.  Tolerances: 1e-10 relative for complex128, 1e-5 for complex64."""

import numpy as np
import pytest

from tests.gpu_util import (TOL_3M, TOL_BACKWARD_BF16X3, TOL_BACKWARD_C64, TOL_BF16X3, TOL_C128, TOL_C64, c64_leaves,
                            gpu_contract, gpu_sliced, note, rel)
from tn_inputs.circuits import circuit_network
from tn_inputs.graphs import pairwise_network, random_network, rrg_network
from tn_inputs.greedy import find_tree
from tn_inputs.network import Network, Tree

pytestmark = pytest.mark.gpu

TWO = Tree(np.array([0], np.int32), np.array([1], np.int32))

# (h, m, n, k) log2 class sizes: dot, outer, row kernel both orientations,
# split-K with and without chunks, matrix-core GEMM (partial and full tiles,
# K = 0, batch), the few-summed-values GEMM (one to three summed bits, with
# and without batches), and tiny cases
SHAPES = [(0, 0, 0, 0), (0, 0, 0, 10), (0, 3, 2, 0), (0, 10, 2, 3), (0, 2, 10, 3), (0, 1, 1, 16),
          (0, 4, 4, 8), (3, 2, 2, 2), (0, 5, 5, 0), (0, 6, 6, 4), (0, 7, 9, 5), (0, 10, 10, 8),
          (2, 6, 6, 3), (0, 12, 5, 1), (0, 8, 7, 11), (1, 9, 3, 6), (0, 5, 8, 2),
          (0, 5, 5, 1), (2, 6, 7, 2), (1, 9, 5, 2), (0, 6, 11, 1), (3, 5, 6, 1)]


TOLS = {"c64_4m": TOL_C64, "c128": TOL_C128, "c64_bf16x3": TOL_BF16X3, "c64_3m": TOL_3M}


@pytest.mark.parametrize("prec", ["c64_4m", "c128", "c64_bf16x3", "c64_3m"])
@pytest.mark.parametrize("shape", SHAPES)
def test_pairwise(oracle_lib, shape, prec):
    net = pairwise_network(*shape, seed=sum(shape) * 7 + len(prec))
    ref = oracle_lib.contract(net, TWO)
    tol = TOLS[prec]
    # the default kernel choice, and the matrix-core kernels for GEMM-shaped
    # nodes of every size (by default those under 2^25 multiply-adds take the
    # row kernel)
    for all_sizes in (False, True):
        note("pairwise", shape, prec, "gemm_all_sizes", all_sizes)
        got = gpu_sliced(net, TWO, precision=prec, gemm_all_sizes=all_sizes)
        assert got.shape == ref.shape
        assert rel(got, ref) < tol
        got2 = gpu_contract(net, TWO, precision=prec, gemm_all_sizes=all_sizes)
        assert rel(got2, ref) < tol


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
@pytest.mark.parametrize("seed", range(4))
def test_random_trees_hyper_outputs(oracle_lib, seed, prec):
    net = random_network(9, 14, 4, seed=100 + seed, n_out=2, dims=(2, 4), hyper=True)
    tree = find_tree(net, seed=seed, trials=2)
    ref = oracle_lib.contract(net, tree)
    note("random tree", seed, prec)
    got = gpu_sliced(net, tree, precision=prec)
    assert rel(got, ref) < (TOL_C128 if prec == "c128" else TOL_C64)


def test_cfg1_amplitudes_c128(oracle_lib):
    """3x3 grid, 8 cycles, complex128, greedy tree, no slicing: GPU amplitude
    against the oracle for 32 seeded bitstrings (same tree for all)."""
    net0 = circuit_network(3, 3, 8, 0, 0)
    tree = find_tree(net0, seed=0, trials=1)
    rng = np.random.default_rng(0)
    for b in [int(rng.integers(0, 2 ** 9))] + list(range(31)):
        net = circuit_network(3, 3, 8, 0, b)
        ref = oracle_lib.contract(net, tree)
        got = gpu_contract(net, tree, precision="c128")
        assert abs(complex(got) - complex(ref)) <= TOL_C128 * abs(complex(ref))


@pytest.mark.parametrize("prec", ["c64_4m", "c128", "c64_bf16x3", "c64_3m"])
def test_swap_diag_circuit_sliced(oracle_lib, prec):
    """fSim as SWAP . diag: wires become hyperedges and most contractions get
    batch indices (H), matrix-core GEMMs included; 4x5 grid, 12 cycles, three
    open qubits, sliced to width 16, all slices summed."""
    net = circuit_network(4, 5, 12, 5, 0b1011001110100101, open_qubits=(2, 9, 13), decompose="swap_diag")
    tree = find_tree(net, seed=0, trials=4, slice_width=16)
    sl = list(tree.meta["sliced"])
    ref = oracle_lib.contract(net, tree, sliced=sl)
    note("swap_diag", prec, "W", tree.meta["W"], "sliced", sl)
    got = gpu_sliced(net, tree, sliced=sl, precision=prec)
    assert got.shape == ref.shape
    assert rel(got, ref) < TOLS[prec]


def _canonical_pair(h, m, n, k, seed):
    """A(H, M, K) x B(H, N, K) with the summed bits lowest in both operands."""
    H = list(range(h))
    M = list(range(h, h + m))
    K = list(range(h + m, h + m + k))
    N = list(range(h + m + k, h + m + k + n))
    rng = np.random.default_rng(seed)
    a = (rng.normal(size=(2,) * (h + m + k)) + 1j * rng.normal(size=(2,) * (h + m + k)))
    b = (rng.normal(size=(2,) * (h + n + k)) + 1j * rng.normal(size=(2,) * (h + n + k)))
    return Network([a, b], [H + M + K, H + N + K], [2] * (h + m + n + k), H + M + N)


@pytest.mark.parametrize("shape", [(12, 1, 2), (14, 2, 1), (10, 3, 0), (11, 4, 2), (6, 2, 3), (9, 4, 5)])
def test_row_staged_stores(oracle_lib, shape):
    """Row kernel whose output rows are staged through LDS (the in-thread values
    lowest in C, the row bits right above them)."""
    m, n, k = shape
    M, K, N = list(range(m)), list(range(m, m + k)), list(range(m + k, m + k + n))
    rng = np.random.default_rng(sum(shape))
    a = rng.normal(size=(2,) * (m + k)) + 1j * rng.normal(size=(2,) * (m + k))
    b = rng.normal(size=(2,) * (n + k)) + 1j * rng.normal(size=(2,) * (n + k))
    net = Network([a, b], [M + K, N + K], [2] * (m + n + k), M + N)
    ref = oracle_lib.contract(net, TWO)
    for prec in ("c64_4m", "c128"):
        assert rel(gpu_sliced(net, TWO, precision=prec), ref) < TOLS[prec]
        assert rel(gpu_contract(net, TWO, precision=prec), ref) < TOLS[prec]


TILE_CASES = {"c64_4m": [0, 1, 2, 3, 5, 6, 7, 8, 9, 14], "c64_3m": [0, 1, 2, 3, 7, 8, 9], "c64_bf16x3": [0, 1, 2, 3, 10, 11, 12, 13]}


@pytest.mark.parametrize("prec", sorted(TILE_CASES))
def test_every_tile_variant(oracle_lib, prec):
    """Each matrix-core tile variant pinned with tn_plan_set_tile, on pairwise
    nodes with the summed bits lowest (full and partial tiles, batch bits, K of
    two stages and of many) and on a hyperedge circuit whose intermediates the
    planner lays out."""
    nets = [(_canonical_pair(*s, seed=i), TWO, ()) for i, s in
            enumerate([(0, 8, 9, 5), (2, 7, 6, 4), (0, 10, 10, 8), (1, 5, 9, 12), (0, 9, 8, 4)])]
    cnet = circuit_network(4, 5, 12, 5, 0b1011001110100101, open_qubits=(2, 9, 13), decompose="swap_diag")
    ctree = find_tree(cnet, seed=0, trials=4, slice_width=16)
    nets.append((cnet, ctree, list(ctree.meta["sliced"])))
    from paper_2002_01935_amd.binding import Plan
    for ni, (net, tree, sl) in enumerate(nets):
        ref = oracle_lib.contract(net, tree, sliced=sl)
        for t in TILE_CASES[prec]:
            plan = Plan(net, tree, sliced=sl, precision=prec, gemm_all_sizes=True)
            changed = plan.set_tile(t)   # 0 when no contraction can take it, or t is already every op's default
            note("tile", prec, t, "net", ni, "changed", changed)
            got = gpu_sliced(net, tree, sliced=sl, precision=prec, plan=plan)
            assert rel(got, ref) < TOLS[prec], (prec, t, ni)


# (h, m, n, k) of 2^28 multiply-adds (operands split into bf16 planes before
# the GEMM): two stages of 8 summed values, many; batch bits; canonical and
# scattered axes (8 summed values or fewer take the few-summed-values kernel)
PRESPLIT = [("canonical", (0, 10, 10, 8)), ("canonical two stages", (0, 12, 12, 4)),
            ("canonical h", (2, 9, 9, 8)), ("scattered", (0, 10, 9, 9)), ("scattered h", (1, 9, 10, 8))]


def test_presplit_tile_variants(oracle_lib):
    """Every BF16x3 variant on pre-split operands (10-13) pinned with
    tn_plan_set_tile, against the oracle, within the BF16x3 bound."""
    from paper_2002_01935_amd.binding import Plan
    for i, (name, shp) in enumerate(PRESPLIT):
        net = (_canonical_pair(*shp, seed=90 + i) if name.startswith("canonical")
               else pairwise_network(*shp, seed=90 + i, dims=(2,)))
        ref = oracle_lib.contract(net, TWO)
        for t in (10, 11, 12, 13):
            plan = Plan(net, TWO, precision="c64_bf16x3")
            # the variants on pre-split planes are the only ones such a node takes
            assert plan.nodes()[0]["kernel"].startswith("gemm_mfma_bf16x3_dl"), name
            plan.set_tile(t)
            assert plan.nodes()[0]["tile"] == t, (name, t)
            note("presplit", name, shp, "tile", t, plan.nodes()[0]["kernel"])
            got = gpu_sliced(net, TWO, precision="c64_bf16x3", plan=plan)
            e = rel(got, ref)
            note("presplit", name, "tile", t, "rel err %.3e" % e)
            assert e < TOL_BF16X3, (name, t, e)


BACK = {"c64_4m": TOL_BACKWARD_C64, "c64_3m": TOL_BACKWARD_C64, "c64_bf16x3": TOL_BACKWARD_BF16X3}


def _cfg2_check(oracle_lib, net, tree, sl, prec, ref128, tag):
    """complex128 within 1e-10 of the oracle; a single precision within its
    relative bound of the oracle on the same complex64 leaves or, the scalar
    being the result of heavy cancellation, with a normwise backward error
    err / kappa of the last contraction within TOL_BACKWARD_*."""
    got = complex(gpu_sliced(net, tree, sliced=sl, precision=prec))
    if prec == "c128":
        err = abs(got - ref128) / abs(ref128)
        note(tag, prec, "rel err", err)
        assert err <= TOL_C128
        return err, None
    n64 = c64_leaves(net)
    ref = complex(oracle_lib.contract(n64, tree, sliced=sl))
    kappa = oracle_lib.root_condition(n64, tree, sl)
    err = abs(got - ref) / abs(ref)
    note(tag, prec, "rel err %.3e kappa %.1f backward %.3e (vs complex128 leaves %.3e)"
         % (err, kappa, err / kappa, abs(got - ref128) / abs(ref128)))
    assert err <= TOLS[prec] or err / kappa <= BACK[prec], (tag, prec, err, kappa)
    return err, kappa


@pytest.mark.parametrize("seed", [0, 1])
def test_cfg2_rrg(oracle_lib, seed):
    """120-vertex random 3-regular network, every precision."""
    net = rrg_network(120, 3, seed=seed)
    tree = find_tree(net, seed=seed, trials=8, slice_width=20)
    sl = tree.meta["sliced"]
    ref128 = complex(oracle_lib.contract(net, tree, sliced=sl))
    note("cfg2", seed, "W_s", tree.meta["W_s"], "sliced", sl)
    for prec in ("c128", "c64_4m", "c64_bf16x3", "c64_3m"):
        _cfg2_check(oracle_lib, net, tree, sl, prec, ref128, "cfg2 seed %d" % seed)


def test_cfg2_error_study(oracle_lib):
    """The 120-vertex random 3-regular network over seeds 0-9 in every
    precision (bounds as in test_cfg2_rrg); prints the median and maximum
    relative and backward errors per precision."""
    errs = {p: [] for p in ("c128", "c64_4m", "c64_3m", "c64_bf16x3")}
    backs = {p: [] for p in errs}
    for seed in range(10):
        net = rrg_network(120, 3, seed=seed)
        tree = find_tree(net, seed=seed, trials=8, slice_width=20)
        sl = tree.meta["sliced"]
        ref128 = complex(oracle_lib.contract(net, tree, sliced=sl))
        for prec in errs:
            err, kappa = _cfg2_check(oracle_lib, net, tree, sl, prec, ref128, "cfg2 study seed %d" % seed)
            errs[prec].append(err)
            if kappa:
                backs[prec].append(err / kappa)
    for prec, e in errs.items():
        note("cfg2 study", prec, "rel err median", float(np.median(e)), "max", max(e),
             "backward max", max(backs[prec]) if backs[prec] else None)


def test_sliced_subsets_and_batches(oracle_lib):
    net = random_network(10, 16, 4, seed=7, n_out=1, dims=(2,), hyper=False)
    tree = find_tree(net, seed=1, trials=2)
    cand = [e for e in range(net.n_idx) if e not in net.out_idx]
    sliced = cand[:4]
    ref_all = oracle_lib.contract(net, tree, sliced=sliced)
    ids = [3, 0, 9, 14, 5]
    ref_sub = oracle_lib.contract(net, tree, sliced=sliced, slice_ids=ids)
    outs = []
    for nb in (1, 2, 3, 16):
        note("slices batch", nb)
        got = gpu_sliced(net, tree, sliced=sliced, precision="c128", max_inflight=nb)
        assert rel(got, ref_all) < TOL_C128
        sub = gpu_sliced(net, tree, sliced=sliced, slice_ids=ids, precision="c128", max_inflight=nb)
        assert rel(sub, ref_sub) < TOL_C128
        outs.append(gpu_sliced(net, tree, sliced=sliced, precision="c64_4m", max_inflight=nb))
    # fixed-order FP64 slice sum: identical bits whatever the batch size
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_repeat_is_bitwise_identical():
    net = rrg_network(60, 3, seed=3)
    tree = find_tree(net, seed=0, trials=2, slice_width=12)
    sl = tree.meta["sliced"]
    from paper_2002_01935_amd.binding import Plan
    p = Plan(net, tree, sliced=sl)
    a = gpu_sliced(net, tree, plan=p)
    b = gpu_sliced(net, tree, plan=p)
    assert np.array_equal(a, b)


SPLIT_SHAPES = [(0, 8, 7, 11), (1, 6, 8, 12), (0, 7, 6, 14), (2, 5, 5, 13)]


@pytest.mark.parametrize("prec", ["c64_4m", "c64_3m", "c64_bf16x3", "c128"])
def test_gemm_split_k(oracle_lib, prec):
    """GEMM nodes with few output tiles and a long sum: the summed range is
    split across the grid and the partial tiles summed in a fixed order.
    Random axis orders (split bits scattered in both operands), canonical
    operands (direct-to-LDS kernels), unsliced direct writes of the output,
    and a sliced summed index with two slices in flight (one partial buffer
    per slice)."""
    from paper_2002_01935_amd.binding import Plan
    cases = [(pairwise_network(*s, seed=31 + i), f"perm {s}") for i, s in enumerate(SPLIT_SHAPES)]
    cases += [(_canonical_pair(0, 7, 7, 12, seed=5), "canonical"), (_canonical_pair(1, 6, 7, 11, seed=6), "canonical h")]
    if prec == "c64_bf16x3":
        # at least 2^28 multiply-adds: operands split into bf16 planes by the
        # split pass (scattered axes, batch bits), then split-K on the planes
        cases += [(pairwise_network(0, 7, 8, 14, seed=77), "presplit perm"),
                  (pairwise_network(2, 6, 7, 13, seed=78), "presplit perm h")]
    for net, name in cases:
        note("split-k", prec, name)
        plan = Plan(net, TWO, precision=prec, gemm_all_sizes=True)
        assert [n["kclass"] for n in plan.nodes()] == ["gemm_splitk"], name
        ref = oracle_lib.contract(net, TWO)
        assert rel(gpu_sliced(net, TWO, precision=prec, plan=plan), ref) < TOLS[prec], name
        assert rel(gpu_contract(net, TWO, precision=prec, gemm_all_sizes=True), ref) < TOLS[prec], name
    net = pairwise_network(0, 8, 7, 12, seed=40, dims=(2,))
    k_idx = [e for e in range(net.n_idx) if e not in net.out_idx]
    sl = k_idx[:1]
    plan = Plan(net, TWO, sliced=sl, precision=prec, max_inflight_slices=2, gemm_all_sizes=True)
    assert [n["kclass"] for n in plan.nodes()] == ["gemm_splitk"]
    ref = oracle_lib.contract(net, TWO, sliced=sl)
    note("split-k sliced", prec)
    assert rel(gpu_sliced(net, TWO, sliced=sl, precision=prec, max_inflight=2, plan=plan), ref) < TOLS[prec]


@pytest.mark.parametrize("prec", ["c64_4m", "c128", "c64_3m", "c64_bf16x3"])
def test_degenerate_networks(oracle_lib, prec):
    """A single leaf (the result is the leaf permuted to the output order), an
    index of dimension 1 between two leaves (an outer product in disguise),
    a scalar from two vectors, and a network whose only summed index has
    dimension 1 next to a real contraction."""
    one = Tree(np.zeros(0, np.int32), np.zeros(0, np.int32))
    rng = np.random.default_rng(11)

    def cn(*shape):
        return rng.normal(size=shape) + 1j * rng.normal(size=shape)

    cases = [
        (Network([cn(2, 4, 2)], [[0, 1, 2]], [2, 4, 2], [2, 0, 1]), one),
        (Network([cn(8, 1), cn(1, 4)], [[0, 1], [1, 2]], [8, 1, 4], [0, 2]), TWO),
        (Network([cn(64), cn(64)], [[0], [0]], [64], []), TWO),
        (Network([cn(2, 1, 16), cn(16, 1, 4)], [[0, 1, 2], [2, 3, 4]], [2, 1, 16, 1, 4], [0, 1, 3, 4]), TWO),
    ]
    for i, (net, tree) in enumerate(cases):
        note("degenerate", prec, i)
        ref = oracle_lib.contract(net, tree)
        got = gpu_sliced(net, tree, precision=prec)
        assert got.shape == ref.shape, i
        assert rel(got, ref) < TOLS[prec], i
        assert rel(gpu_contract(net, tree, precision=prec), ref) < TOLS[prec], i


def test_graph_replays_match_eager(oracle_lib, monkeypatch):
    """The sliced contraction replays one captured HIP graph per batch of
    in-flight slices.  Several calls, each replaying the graph more than once,
    with unrelated eager PyTorch work and synchronisations in between, give
    bitwise the result of the same kernels launched eagerly (TN_NO_GRAPH=1):
    a hyperedge circuit (row, split-K row and GEMM kernels, reductions) and a
    split-K GEMM node (partial tiles and their fixed-order sum)."""
    import torch

    from paper_2002_01935_amd.binding import Plan
    circ = circuit_network(4, 5, 12, 5, 0b1011001110100101, open_qubits=(2, 9, 13), decompose="swap_diag")
    ctree = find_tree(circ, seed=0, trials=4, slice_width=16)
    pair = pairwise_network(0, 8, 7, 12, seed=40, dims=(2,))
    pk = [e for e in range(pair.n_idx) if e not in pair.out_idx]
    cases = [(circ, ctree, list(ctree.meta["sliced"])), (pair, TWO, pk[:2])]
    x = torch.randn(512, 512, device="cuda")
    for ci, (net, tree, sl) in enumerate(cases):
        ids = list(range(0, 2 ** len(sl), 3)) if len(sl) > 2 else list(range(2 ** len(sl)))
        ref = oracle_lib.contract(net, tree, sliced=sl, slice_ids=ids)
        monkeypatch.setenv("TN_NO_GRAPH", "1")
        eager = gpu_sliced(net, tree, sliced=sl, slice_ids=ids, precision="c64_4m", max_inflight=2,
                           gemm_all_sizes=True)
        monkeypatch.delenv("TN_NO_GRAPH")
        assert rel(eager, ref) < TOL_C64, ci
        plan = Plan(net, tree, sliced=sl, precision="c64_4m", max_inflight_slices=2, gemm_all_sizes=True)
        for r in range(4):
            note("graph replay", ci, "call", r)
            got = gpu_sliced(net, tree, sliced=sl, slice_ids=ids, plan=plan)
            assert np.array_equal(got, eager), (ci, r)
            y = (x @ x).sum()                      # eager work between the calls
            torch.cuda.synchronize()
            assert torch.isfinite(y)


@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
def test_rank_simplified_tree(oracle_lib, prec):
    """A tree searched on the rank-simplified network (Sec. 3.7: merges that
    do not raise rank, then the finder's tree over the survivors) contracts
    on the GPU to the oracle's value of the original network on its own
    unsimplified tree: a hyperedge circuit (fSim as SWAP . diag) with open
    qubits, sliced."""
    from tn_inputs.simplify import compose, rank_simplify, structure_network
    net = circuit_network(4, 5, 12, 5, 0b1011001110100101, open_qubits=(2, 9, 13), decompose="swap_diag")
    simp = rank_simplify(net)
    st = find_tree(structure_network(net, simp), seed=0, trials=4, slice_width=16)
    tree = compose(simp, st)
    sl = list(st.meta["sliced"])
    plain = find_tree(net, seed=0, trials=4)
    rnet = net if prec == "c128" else c64_leaves(net)
    ref = oracle_lib.contract(rnet, plain)
    note("rank-simplified", prec, "merges", len(simp.pairs), "sliced", len(sl))
    got = gpu_sliced(net, tree, sliced=sl, precision=prec)
    assert got.shape == ref.shape
    assert rel(got, ref) < TOLS[prec]
