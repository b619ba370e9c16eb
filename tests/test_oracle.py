"""Pins of the CPU oracle against things other than itself: statevector
amplitudes, direct nested sums, library routines on special cases, closed
forms, identities of the method (tree invariance, sliced sum = unsliced), and
unitarity.  No GPU."""

import math

import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle import statevector as sv
from tn_inputs.circuits import (FSIM, ONE_QUBIT_GATES, circuit_network, fsim, gate_leaves,
                                random_circuit)
from tn_inputs.graphs import random_network, rrg_network
from tn_inputs.greedy import _Greedy, find_tree, width_cost
from tn_inputs.network import Network, Tree


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def random_tree(net, seed):
    return _Greedy(net).run(float(np.random.default_rng(seed).uniform(0, 1.5)), 1.0,
                            np.random.default_rng(seed))


# ---------------------------------------------------------------- gates


def test_gates_unitary():
    for u in list(ONE_QUBIT_GATES) + [FSIM, fsim(0.3, 1.1)]:
        assert np.allclose(u @ u.conj().T, np.eye(u.shape[0]), atol=1e-14)


def test_fsim_is_swap_times_diagonal():
    phi = np.pi / 6
    swap = np.eye(4)[[0, 2, 1, 3]]
    d = np.diag([1, -1j, -1j, np.exp(-1j * phi)])
    assert np.allclose(FSIM, swap @ d, atol=1e-15)


def test_sqrt_gates_square_to_paulis():
    X = np.array([[0, 1], [1, 0]])
    Y = np.array([[0, -1j], [1j, 0]])
    W = (X + Y) / np.sqrt(2)
    for u, p in zip(ONE_QUBIT_GATES, (X, Y, W)):
        # exp(-i pi/4 P)^2 = exp(-i pi/2 P) = -i P
        assert np.allclose(u @ u, -1j * p, atol=1e-14)


# ---------------------------------------------------------------- circuits vs statevector


def test_cfg1_every_amplitude_matches_statevector(oracle_lib):
    R, C, m, seed = 3, 3, 8, 0
    N = R * C
    net0 = circuit_network(R, C, m, seed, 0)
    tree = find_tree(net0, seed=0, trials=1)
    psi = sv.run(N, net0.meta["gates"])
    total = 0.0
    worst = 0.0
    for b in range(2 ** N):
        net = circuit_network(R, C, m, seed, b)
        c = oracle_lib.contract(net, tree)
        ref = sv.amplitude(N, net0.meta["gates"], b, state=psi)
        worst = max(worst, abs(complex(c) - complex(ref)))
        total += abs(complex(c)) ** 2
    assert worst < 1e-13
    assert abs(total - 1.0) < 1e-12      # sum_b |c_b|^2 = 1 (unitarity)


def test_open_outputs_match_statevector(oracle_lib):
    R, C, m, seed = 3, 4, 6, 3
    N = R * C
    opens = (1, 5, 6, 10)
    b = 0b101101100110
    net = circuit_network(R, C, m, seed, b, open_qubits=opens)
    tree = find_tree(net, seed=2, trials=2)
    got = oracle_lib.contract(net, tree)
    ref = sv.amplitude(N, net.meta["gates"], b, open_qubits=opens)
    assert got.shape == (2,) * len(opens)
    assert rel(got, ref) < 1e-12


def test_norm_over_open_outputs(oracle_lib):
    # all qubits open: the output is the whole state, of unit norm
    R, C, m = 2, 3, 5
    net = circuit_network(R, C, m, 7, 0, open_qubits=tuple(range(R * C)))
    tree = find_tree(net, seed=0, trials=1)
    psi = oracle_lib.contract(net, tree)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12
    assert rel(psi, sv.run(R * C, net.meta["gates"])) < 1e-12


def test_swap_diag_hyperedge_circuit_matches_statevector(oracle_lib):
    """fSim written as SWAP . diag (hyperedge wires, rank-2 diagonal leaves):
    the network changes, the amplitudes do not."""
    R, C, m, seed = 3, 4, 6, 3
    N = R * C
    opens = (1, 5, 6, 10)
    b = 0b011101100110
    net = circuit_network(R, C, m, seed, b, open_qubits=opens, decompose="swap_diag")
    assert any(len(set(t)) == 2 and net.leaves[v].shape == (2, 2) for v, t in enumerate(net.leaf_idx))
    deg = {}
    for t in net.leaf_idx:
        for e in t:
            deg[e] = deg.get(e, 0) + 1
    assert max(deg.values()) == 3            # wires are hyperedges
    tree = find_tree(net, seed=1, trials=2)
    got = oracle_lib.contract(net, tree)
    ref = sv.amplitude(N, net.meta["gates"], b, open_qubits=opens)
    assert rel(got, ref) < 1e-12


# ---------------------------------------------------------------- brute force


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rrg_matches_bruteforce(oracle_lib, seed):
    net = rrg_network(12, 3, seed=seed)
    ref = bf.contract(net)
    for ts in range(3):
        got = oracle_lib.contract(net, random_tree(net, ts))
        assert rel(got, ref) < 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_hyperedges_outputs_nonbinary_match_bruteforce(oracle_lib, seed):
    net = random_network(7, 10, 4, seed=seed, n_out=2, dims=(2, 3), hyper=True)
    ref = bf.contract(net)
    got = oracle_lib.contract(net, random_tree(net, seed))
    assert got.shape == ref.shape
    assert rel(got, ref) < 1e-12


# ---------------------------------------------------------------- library special cases


def _net(leaves, idx, dims, out):
    return Network([np.asarray(t, dtype=np.complex128) for t in leaves], idx, dims, out)


def test_matrix_chain_is_matmul(oracle_lib):
    rng = np.random.default_rng(0)
    A = rng.normal(size=(3, 4)) + 1j * rng.normal(size=(3, 4))
    B = rng.normal(size=(4, 5)) + 1j * rng.normal(size=(4, 5))
    Cm = rng.normal(size=(5, 2)) + 1j * rng.normal(size=(5, 2))
    net = _net([A, B, Cm], [[0, 1], [1, 2], [2, 3]], [3, 4, 5, 2], [0, 3])
    for l, r in ([[0, 3], [1, 2]], [[1, 0], [2, 3]]):
        got = oracle_lib.contract(net, Tree(np.array(l, np.int32), np.array(r, np.int32)))
        assert rel(got, A @ B @ Cm) < 1e-13
    # transposed output order
    net_t = _net([A, B, Cm], [[0, 1], [1, 2], [2, 3]], [3, 4, 5, 2], [3, 0])
    got = oracle_lib.contract(net_t, Tree(np.array([0, 3], np.int32), np.array([1, 2], np.int32)))
    assert rel(got, (A @ B @ Cm).T) < 1e-13


def test_outer_dot_and_batch(oracle_lib):
    rng = np.random.default_rng(1)
    a = rng.normal(size=3) + 1j * rng.normal(size=3)
    b = rng.normal(size=4) + 1j * rng.normal(size=4)
    t = Tree(np.array([0], np.int32), np.array([1], np.int32))
    got = oracle_lib.contract(_net([a, b], [[0], [1]], [3, 4], [1, 0]), t)
    assert rel(got, np.outer(b, a)) < 1e-14                      # outer product
    c = rng.normal(size=3) + 1j * rng.normal(size=3)
    got = oracle_lib.contract(_net([a, c], [[0], [0]], [3], []), t)
    assert abs(complex(got) - np.dot(a, c)) < 1e-13              # dot product (no conj)
    X = rng.normal(size=(2, 3, 4)) + 1j * rng.normal(size=(2, 3, 4))
    Y = rng.normal(size=(2, 4, 5)) + 1j * rng.normal(size=(2, 4, 5))
    got = oracle_lib.contract(_net([X, Y], [[0, 1, 2], [0, 2, 3]], [2, 3, 4, 5], [0, 1, 3]), t)
    assert rel(got, np.matmul(X, Y)) < 1e-13                     # batch (hyper) index


def test_identity_leaves_leave_operand_unchanged(oracle_lib):
    rng = np.random.default_rng(2)
    T = rng.normal(size=(2, 2, 2)) + 1j * rng.normal(size=(2, 2, 2))
    I = np.eye(2)
    net = _net([T, I, I], [[0, 1, 2], [1, 3], [2, 4]], [2] * 5, [0, 3, 4])
    got = oracle_lib.contract(net, Tree(np.array([0, 3], np.int32), np.array([1, 2], np.int32)))
    assert rel(got, T) < 1e-15


def test_closed_forms(oracle_lib):
    # ring of n copies of M: trace(M^n) = sum of eigenvalues^n
    rng = np.random.default_rng(3)
    M = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
    n = 7
    net = _net([M] * n, [[i, (i + 1) % n] for i in range(n)], [3] * n, [])
    got = oracle_lib.contract(net, random_tree(net, 0))
    ev = np.linalg.eigvals(M)
    assert abs(complex(got) - np.sum(ev ** n)) < 1e-10 * np.sum(np.abs(ev) ** n)
    # all-ones tensors: the sum counts assignments, prod_e |D(e)|
    net = random_network(6, 9, 4, seed=4, dims=(2, 3))
    ones = net.with_leaves([np.ones_like(t) for t in net.leaves])
    got = oracle_lib.contract(ones, random_tree(ones, 1))
    assert abs(complex(got) - float(np.prod(net.idx_dim))) < 1e-9


# ---------------------------------------------------------------- method identities


def test_tree_invariance(oracle_lib):
    net = rrg_network(40, 3, seed=5)
    vals = [oracle_lib.contract(net, random_tree(net, s)) for s in range(3)]
    for v in vals[1:]:
        assert rel(v, vals[0]) < 1e-10


@pytest.mark.parametrize("seed", range(4))
def test_sliced_sum_equals_unsliced(oracle_lib, seed):
    net = random_network(8, 12, 4, seed=10 + seed, n_out=1, dims=(2, 3), hyper=True)
    tree = random_tree(net, seed)
    full = oracle_lib.contract(net, tree)
    cand = [e for e in range(net.n_idx) if e not in net.out_idx]
    sliced = list(np.random.default_rng(seed).choice(cand, size=3, replace=False))
    d = int(np.prod([net.idx_dim[e] for e in sliced]))
    assert rel(oracle_lib.contract(net, tree, sliced=sliced), full) < 1e-12
    parts = [oracle_lib.contract(net, tree, sliced=sliced, slice_ids=[s]) for s in range(d)]
    assert rel(np.sum(parts, axis=0), full) < 1e-12


def test_slice_id_radix_matches_projection(oracle_lib):
    # slice id -> values: first sliced index most significant.  Projecting the
    # indices onto those values by hand (appending <x| leaves) gives the slice.
    net = circuit_network(2, 3, 4, 1, 0)
    tree = find_tree(net, seed=0, trials=1)
    sliced = [net.leaf_idx[gate_leaves(net, "2q")[0]][0], net.leaf_idx[gate_leaves(net, "2q")[2]][1]]
    for sid in range(4):
        got = oracle_lib.contract(net, tree, sliced=sliced, slice_ids=[sid])
        x0, x1 = (sid >> 1) & 1, sid & 1
        # split each sliced index into two copies joined by a projector pair
        leaves = list(net.leaves)
        idx = [list(ix) for ix in net.leaf_idx]
        dims = list(net.idx_dim)
        for e, x in ((sliced[0], x0), (sliced[1], x1)):
            holders = [v for v, ix in enumerate(idx) if e in ix]
            e2 = len(dims)
            dims.append(2)
            idx[holders[1]] = [e2 if f == e else f for f in idx[holders[1]]]
            p = np.zeros(2)
            p[x] = 1.0
            leaves += [p, p]
            idx += [[e], [e2]]
        proj = Network(leaves, idx, dims, [])
        ref = oracle_lib.contract(proj, find_tree(proj, seed=0, trials=1))
        assert abs(complex(got) - complex(ref)) < 1e-14


def test_width_cost_by_hand(oracle_lib):
    # ring A(a,b) B(b,c) C(c,d) D(d,a), tree ((A,B),(C,D))
    M = np.ones((2, 2))
    net = _net([M] * 4, [[0, 1], [1, 2], [2, 3], [3, 0]], [2] * 4, [])
    tree = Tree(np.array([0, 2, 4], np.int32), np.array([1, 3, 5], np.int32))
    W, lc = oracle_lib.width_cost(net, tree)
    assert W == 2 and abs(2 ** lc - (8 + 8 + 4)) < 1e-9
    # sequential tree (((A,B),C),D): nodes {a,c}, {a,d}, {} -> C = 8 + 8 + 4
    tree = Tree(np.array([0, 4, 5], np.int32), np.array([1, 2, 3], np.int32))
    W, lc = oracle_lib.width_cost(net, tree)
    assert W == 2 and abs(2 ** lc - 20) < 1e-9
    # slicing index b: widths drop by one wherever b was kept
    W, lc = oracle_lib.width_cost(net, tree, sliced=[1])
    assert W == 2 and abs(2 ** lc - (4 + 8 + 4)) < 1e-9


def test_width_cost_agree_with_finder(oracle_lib):
    for net in (circuit_network(3, 3, 8, 0, 0), rrg_network(30, 3, seed=1)):
        tree = find_tree(net, seed=1, trials=2)
        W1, c1 = width_cost(net, tree)
        W2, c2 = oracle_lib.width_cost(net, tree)
        assert W1 == W2 and abs(c1 - c2) < 1e-9


@pytest.mark.parametrize("case", ["self_loop", "dangling", "bad_tree", "sliced_output"])
def test_validation(oracle_lib, case):
    M = np.ones((2, 2))
    t = Tree(np.array([0], np.int32), np.array([1], np.int32))
    if case == "self_loop":
        net, tree, sl = _net([np.ones((2, 2)), np.ones(2)], [[0, 0], [0]], [2], []), t, []
        net.leaves[0] = np.ones((2, 2))
    elif case == "dangling":
        net, tree, sl = _net([M, np.ones(2)], [[0, 1], [0]], [2, 2], []), t, []
    elif case == "bad_tree":
        net, tree, sl = _net([M, M], [[0, 1], [1, 0]], [2, 2], []), Tree(np.array([0], np.int32), np.array([0], np.int32)), []
    else:
        net, tree, sl = _net([M, M], [[0, 1], [1, 2]], [2, 2, 2], [0, 2]), t, [0]
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.contract(net, tree, sliced=sl)


# ---------------------------------------------------------------- reverse mode


def _env_bruteforce(net, v):
    """dR/dT_v[k] for a leaf appearing once: R with T_v replaced by unit e_k."""
    shape = net.leaves[v].shape
    out = []
    for k in range(int(np.prod(shape))):
        e = np.zeros(int(np.prod(shape)), dtype=np.complex128)
        e[k] = 1.0
        leaves = list(net.leaves)
        leaves[v] = e.reshape(shape)
        out.append(bf.contract(net.with_leaves(leaves)))
    return np.array(out)                         # (k, *out_shape)


@pytest.mark.parametrize("seed", range(3))
def test_grad_matches_bruteforce_environments(oracle_lib, seed):
    net = random_network(6, 8, 4, seed=20 + seed, n_out=2, dims=(2, 3), hyper=True)
    tree = random_tree(net, seed)
    rng = np.random.default_rng(seed)
    out_shape = tuple(net.idx_dim[e] for e in net.out_idx)
    go = rng.normal(size=out_shape) + 1j * rng.normal(size=out_shape)
    wrt = list(range(net.n_leaves))
    grads = oracle_lib.grad(net, tree, go, wrt)
    for v, g in zip(wrt, grads):
        J = _env_bruteforce(net, v).reshape(g.size, -1)          # dR_o / dT[k]
        ref = (J.conj() @ go.ravel()).reshape(g.shape)
        assert rel(g, ref) < 1e-11


def test_grad_circuit_statevector_environments(oracle_lib):
    # 2x3 grid, every 2q gate: E_g[k] = amplitude with gate g replaced by unit
    # matrix k (statevector); for L = |c|^2, grad_g = 2 c conj(E_g)
    R, C, m, seed, b = 2, 3, 4, 2, 0b101100
    N = R * C
    net = circuit_network(R, C, m, seed, b)
    tree = find_tree(net, seed=0, trials=1)
    c = complex(oracle_lib.contract(net, tree))
    g2 = gate_leaves(net, "2q")
    grads = oracle_lib.grad(net, tree, np.array(2 * c), g2)
    gates = net.meta["gates"]
    gpos = [k for k, gt in enumerate(gates) if gt[0] == "2q"]
    for leaf, pos, g in zip(g2, gpos, grads):
        E = np.zeros(16, dtype=np.complex128)
        for k in range(16):
            unit = np.zeros(16, dtype=np.complex128)
            unit[k] = 1.0
            psi = sv.run(N, gates, replace={pos: unit.reshape(4, 4)})
            E[k] = sv.amplitude(N, gates, b, state=psi)
        assert rel(g.ravel(), 2 * c * E.conj()) < 1e-11
        # homogeneity: c is linear in each gate
        G = net.leaves[leaf].ravel()
        assert abs(np.sum(G * E) - c) < 1e-13
        assert abs(np.sum(G * g.ravel().conj()) - 2 * abs(c) ** 2) < 1e-13


def test_grad_finite_differences(oracle_lib):
    net = circuit_network(2, 2, 4, 5, 0b0110)
    tree = find_tree(net, seed=0, trials=1)
    c = complex(oracle_lib.contract(net, tree))
    leaf = gate_leaves(net, "2q")[1]
    (g,) = oracle_lib.grad(net, tree, np.array(2 * c), [leaf])
    h = 1e-4
    flat = net.leaves[leaf].ravel()
    for k in (0, 5, 10, 15):
        fd = []
        for step in (h, 1j * h):
            vals = []
            for s in (+1, -1):
                T = flat.copy()
                T[k] += s * step
                leaves = list(net.leaves)
                leaves[leaf] = T.reshape(net.leaves[leaf].shape)
                vals.append(abs(complex(oracle_lib.contract(net.with_leaves(leaves), tree))) ** 2)
            fd.append((vals[0] - vals[1]) / (2 * h))
        # torch convention: dL/dRe + i dL/dIm; L is quadratic so FD is exact
        assert abs((fd[0] + 1j * fd[1]) - g.ravel()[k]) < 1e-9


def test_grad_sliced_equals_unsliced(oracle_lib):
    net = random_network(8, 12, 4, seed=33, n_out=1, hyper=True)
    tree = random_tree(net, 3)
    go = np.array([1.0 + 2.0j, -0.5j])
    cand = [e for e in range(net.n_idx) if e not in net.out_idx]
    sliced = cand[:3]
    wrt = list(range(net.n_leaves))
    full = oracle_lib.grad(net, tree, go, wrt)
    sl = oracle_lib.grad(net, tree, go, wrt, sliced=sliced)
    for a, b in zip(sl, full):
        assert rel(a, b) < 1e-12


# ---------------------------------------------------------------- paper table


def test_paper_table_flop_convention():
    """The FLOPs-efficiency column of the benchmark table equals
    8 C_s / time / 3.031e12 (complex FLOPs = 8 C, Sec. 2) to within 0.2 points
    on every row; bench.py reports throughput with the same convention."""
    import csv
    import os

    from paper_2002_01935_amd.metrics import complex_flops, efficiency

    path = os.path.join(os.path.dirname(__file__), "golden", "benchmark_table.csv")
    rows = [r for r in csv.DictReader(line for line in open(path) if not line.startswith("#"))]
    assert len(rows) == 16
    for r in rows:
        flops = complex_flops(math.log2(float(r["C_s"])))
        eff = 100.0 * efficiency(flops, float(r["time_s"]), 3.031e12)
        assert abs(eff - float(r["efficiency_pct"])) < 0.2, r["circuit"]


def test_subtree_values_compose_to_root(oracle_lib):
    """The oracle's subtree evaluator: contracting the root's two children
    (numpy einsum over their shared indices) gives the full result, with and
    without slicing."""
    net = random_network(8, 12, 4, seed=41, n_out=2, dims=(2, 3), hyper=False)
    tree = random_tree(net, 2)
    n = net.n_leaves
    full = oracle_lib.contract(net, tree)
    a, ia = oracle_lib.subtree_value(net, tree, int(tree.left[-1]))
    b, ib = oracle_lib.subtree_value(net, tree, int(tree.right[-1]))
    letters = {e: chr(97 + i) for i, e in enumerate(sorted(set(ia) | set(ib)))}
    spec = "".join(letters[e] for e in ia) + "," + "".join(letters[e] for e in ib) + "->" + \
        "".join(letters[e] for e in net.out_idx)
    assert rel(np.einsum(spec, a, b), full) < 1e-12
    cand = [e for e in range(net.n_idx) if e not in net.out_idx]
    sl = cand[:2]
    d = int(np.prod([net.idx_dim[e] for e in sl]))
    tot = 0
    for s in range(d):
        a, ia = oracle_lib.subtree_value(net, tree, int(tree.left[-1]), sl, s)
        b, ib = oracle_lib.subtree_value(net, tree, int(tree.right[-1]), sl, s)
        letters = {e: chr(97 + i) for i, e in enumerate(sorted(set(ia) | set(ib)))}
        spec = "".join(letters[e] for e in ia) + "," + "".join(letters[e] for e in ib) + "->" + \
            "".join(letters[e] for e in net.out_idx)
        tot = tot + np.einsum(spec, a, b)
    assert rel(tot, full) < 1e-12
    assert n == net.n_leaves


def _kappa_cases():
    """(network, tree, sliced, kappa in closed form) with the root's children
    known by construction: two leaves whose product is the root."""
    rng = np.random.default_rng(12)
    two = Tree(np.array([0], np.int32), np.array([1], np.int32))
    u = rng.normal(size=8) + 1j * rng.normal(size=8)
    v = rng.normal(size=8) + 1j * rng.normal(size=8)
    dot = Network([u, v], [[0], [0]], [8], [])
    k_dot = np.linalg.norm(u) * np.linalg.norm(v) / abs(np.dot(u, v))
    # index 1 (dimension 4) sliced: per slice b the children are u[:, b], v[:, b]
    U = rng.normal(size=(8, 4)) + 1j * rng.normal(size=(8, 4))
    V = rng.normal(size=(8, 4)) + 1j * rng.normal(size=(8, 4))
    sliced = Network([U, V], [[0, 1], [0, 1]], [8, 4], [])
    k_sl = sum(np.linalg.norm(U[:, b]) * np.linalg.norm(V[:, b]) for b in range(4)) / abs(np.sum(U * V))
    # open output o: R[o] = sum_a U[a, o] v[a], kappa = ||U|| ||v|| / ||R||
    opened = Network([U, v], [[0, 1], [0]], [8, 4], [1])
    k_open = np.linalg.norm(U) * np.linalg.norm(v) / np.linalg.norm(v @ U)
    # nearly orthogonal vectors: a large kappa (heavy cancellation)
    w = v - np.vdot(u.conj(), v) / np.vdot(u.conj(), u.conj()) * u.conj() + 1e-3 * u.conj()
    ortho = Network([u, w], [[0], [0]], [8], [])
    k_ortho = np.linalg.norm(u) * np.linalg.norm(w) / abs(np.dot(u, w))
    return [(dot, two, [], k_dot), (sliced, two, [1], k_sl), (opened, two, [], k_open), (ortho, two, [], k_ortho)]


def test_root_condition_closed_forms(oracle_lib):
    """kappa = sum over slices of ||T_l|| ||T_r|| / ||R|| for the root's
    children: a dot product, the same with an index sliced (sum of per-slice
    norm products), an open output, and a nearly orthogonal pair (kappa in
    the hundreds)."""
    for i, (net, tree, sl, k) in enumerate(_kappa_cases()):
        got = oracle_lib.root_condition(net, tree, sl)
        assert abs(got - k) <= 1e-12 * k, (i, got, k)
    assert _kappa_cases()[3][3] > 100


@pytest.mark.parametrize("mistake", ["left_twice", "slice_ignored", "abs_of_sum"])
def test_root_condition_catches_planted_mistakes(oracle_lib, monkeypatch, mistake):
    """A plausible mistake planted in the evaluator behind kappa fails the
    closed-form pins: both children read from the left subtree, the slice id
    ignored (every slice's children taken from slice 0), or the result norm
    taken over the absolute values (no cancellation)."""
    from oracle import contract as oc
    real_sub, real_contract = oc.subtree_value, oc.contract
    if mistake == "left_twice":
        def sub(net, tree, node, sliced=(), slice_id=None):
            return real_sub(net, tree, int(tree.left[-1]), sliced, slice_id)
        monkeypatch.setattr(oc, "subtree_value", sub)
    elif mistake == "slice_ignored":
        def sub(net, tree, node, sliced=(), slice_id=None):
            return real_sub(net, tree, node, sliced, 0 if sliced else slice_id)
        monkeypatch.setattr(oc, "subtree_value", sub)
    else:
        def con(net, tree, **kw):
            return np.abs(real_contract(net.with_leaves([np.abs(t) for t in net.leaves]), tree, **kw))
        monkeypatch.setattr(oc, "contract", con)
    caught = 0
    for net, tree, sl, k in _kappa_cases():
        if abs(oc.root_condition(net, tree, sl) - k) > 1e-6 * k:
            caught += 1
    assert caught >= 1, mistake
