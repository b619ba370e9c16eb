"""GPU reverse mode (tn_contract_backward through the autograd wrapper)
against the oracle's complex128 gradient, finite differences, and the
homogeneity identity of a network that is linear in every leaf."""

import numpy as np
import pytest

from tests.gpu_util import TOL_C128, TOL_C64, c64_leaves, note, rel, rel_inf, to_dev
from tn_inputs import configs
from tn_inputs.circuits import circuit_network, gate_leaves
from tn_inputs.graphs import random_network
from tn_inputs.greedy import find_tree
from tn_inputs.slicing import extend_slices

pytestmark = pytest.mark.gpu


def _plan(net, tree, sliced=(), precision="c64_4m", nb=0, gemm_all_sizes=False):
    from paper_2002_01935_amd.binding import Plan
    return Plan(net, tree, sliced=sliced, precision=precision, max_inflight_slices=nb, gemm_all_sizes=gemm_all_sizes)


@pytest.mark.parametrize("prec", ["c128", "c64_4m"])
def test_autograd_amplitude_norm(oracle_lib, prec):
    import torch

    from paper_2002_01935_amd.autograd import contract
    net = circuit_network(3, 4, 6, 1, 0b101101001110)
    tree = find_tree(net, seed=0, trials=2)
    wrt = gate_leaves(net, "2q")
    plan = _plan(net, tree, precision=prec)
    leaves = to_dev(net, prec)
    for v in wrt:
        leaves[v].requires_grad_(True)
    note("autograd", prec)
    c = contract(plan, leaves)
    L = (c.abs() ** 2).sum()
    L.backward()
    rnet = net if prec == "c128" else c64_leaves(net)
    c_ref = complex(oracle_lib.contract(rnet, tree))
    refs = oracle_lib.grad(rnet, tree, np.array(2 * c_ref), wrt)
    tol = TOL_C128 if prec == "c128" else TOL_C64
    _per_leaf([leaves[v].grad.cpu().numpy() for v in wrt], refs, tol, "autograd " + prec)
    for v in range(net.n_leaves):
        if v not in wrt:
            assert leaves[v].grad is None


@pytest.mark.parametrize("seed", range(3))
def test_backward_sliced_hyper_outputs(oracle_lib, seed):
    net = random_network(10, 15, 4, seed=200 + seed, n_out=2, dims=(2, 4), hyper=True)
    tree = find_tree(net, seed=seed, trials=2)
    cand = [e for e in range(net.n_idx) if e not in net.out_idx]
    sliced = cand[:3]
    rng = np.random.default_rng(seed)
    shape = tuple(net.idx_dim[e] for e in net.out_idx)
    go = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    wrt = list(range(net.n_leaves))
    d = int(np.prod([net.idx_dim[e] for e in sliced]))
    ids = [s for s in range(d) if s % 3 != 1]
    import torch
    for prec, tol in (("c128", TOL_C128), ("c64_4m", TOL_C64)):
        refs = oracle_lib.grad(net if prec == "c128" else c64_leaves(net), tree, go, wrt, sliced=sliced,
                               slice_ids=ids)
        note("backward sliced", seed, prec)
        plan = _plan(net, tree, sliced, prec, nb=2)
        grads = plan.backward(to_dev(net, prec), torch.from_numpy(go), wrt, slice_ids=ids)
        torch.cuda.synchronize()
        _per_leaf([g.cpu().numpy() for g in grads], refs, tol, "backward sliced %d %s" % (seed, prec))


def test_backward_bitwise_independent_of_batch():
    import torch
    net = random_network(10, 15, 4, seed=300, n_out=1, dims=(2,), hyper=False)
    tree = find_tree(net, seed=1, trials=2)
    cand = [e for e in range(net.n_idx) if e not in net.out_idx]
    sliced = cand[:4]
    go = torch.tensor([0.7 - 0.1j, -0.2 + 0.9j], dtype=torch.complex128)
    outs = []
    for nb in (1, 4, 16):
        plan = _plan(net, tree, sliced, "c64_4m", nb=nb)
        grads = plan.backward(to_dev(net, "c64_4m"), go, list(range(net.n_leaves)))
        torch.cuda.synchronize()
        outs.append(np.concatenate([g.cpu().numpy().ravel() for g in grads]))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def _per_leaf(got, ref, tol, what):
    """Each leaf's gradient on its own: normwise and max-componentwise
    relative errors within tol; returns the worst of each."""
    w2 = wi = 0.0
    for v, (g, r) in enumerate(zip(got, ref)):
        e2, ei = rel(g, r), rel_inf(g, r)
        w2, wi = max(w2, e2), max(wi, ei)
        assert e2 < tol and ei < tol, (what, v, e2, ei)
    note(what, "per-leaf worst rel %.3e, max-componentwise %.3e" % (w2, wi))
    return w2, wi


def test_cfg4_gradient_full_size(oracle_lib):
    """6x6 grid, 12 cycles, width 28: d|amp|^2 / d(every fSim leaf) in
    complex64 through tn_contract_backward (recomputation from checkpoints).
    Checks, each leaf on its own: (i) homogeneity, (ii) central differences
    on the GPU complex128 path (h = 1e-4; |amp|^2 is quadratic in each entry,
    so exact up to rounding), (iii) the oracle's complex128 gradient on two
    sub-slices of the same tree (more indices sliced on both sides).  The
    references use the same complex64-rounded leaves the complex64 plan
    receives."""
    import torch
    net, tree, sliced = configs.load("cfg4")
    net64 = c64_leaves(net)
    wrt = gate_leaves(net, "2q")
    assert len(wrt) == 180
    plan64 = _plan(net, tree, sliced, "c64_4m")
    leaves = to_dev(net, "c64_4m")
    note("cfg4 forward")
    c = complex(plan64.contract_sliced(leaves).cpu().numpy())
    L = abs(c) ** 2
    note("cfg4 backward, workspace", plan64.backward_info(wrt)["workspace_bytes"] / 2 ** 30, "GiB")
    grads = plan64.backward(leaves, torch.tensor(2 * c, dtype=torch.complex128), wrt)
    torch.cuda.synchronize()
    grads = [g.cpu().numpy() for g in grads]
    # (i) homogeneity: c is linear in each gate, so sum_k G_k conj(grad_k) = 2 L.
    # The sum over a gate's 16 entries cancels (its terms have random phases),
    # so a relative error d of the gradient entries moves it by up to
    # d * sum_k |G_k| |grad_k|: that is the scale the identity is held to.  Its
    # two sides are two complex64 computations of c (the forward value, and
    # sum_k G_k E_k from the reverse pass), each within TOL_C64 of the oracle,
    # so they may differ by twice that.
    worst = worst_rel = 0.0
    for v, g in zip(wrt, grads):
        terms = net64.leaves[v].ravel() * g.ravel().conj()
        h = np.sum(terms)
        worst = max(worst, abs(h - 2 * L) / np.abs(terms).sum())
        worst_rel = max(worst_rel, abs(h - 2 * L) / (2 * L))
    note("cfg4 homogeneity worst error %.3e relative to sum |G||grad| (%.3e relative to 2L)" % (worst, worst_rel))
    assert worst < 2 * TOL_C64
    # (ii) finite differences with the complex128 GPU path on the same leaves
    plan128 = _plan(net, tree, sliced, "c128")
    leaves128 = to_dev(net64, "c128")
    hstep = 1e-4
    fd_err = 0.0
    for v, k in ((wrt[0], 5), (wrt[90], 10), (wrt[179], 15), (wrt[45], 0), (wrt[135], 6)):
        g = grads[wrt.index(v)].ravel()[k]
        parts = []
        for step in (hstep, 1j * hstep):
            vals = []
            for sgn in (1, -1):
                x = leaves128[v].clone().reshape(-1)
                x[k] += sgn * step
                ls = list(leaves128)
                ls[v] = x.reshape(leaves128[v].shape)
                vals.append(abs(complex(plan128.contract_sliced(ls).cpu().numpy())) ** 2)
            parts.append((vals[0] - vals[1]) / (2 * hstep))
        fd = parts[0] + 1j * parts[1]
        scale = np.abs(grads[wrt.index(v)]).max()
        fd_err = max(fd_err, abs(fd - g) / scale)
    note("cfg4 finite-difference worst error relative to the leaf's largest entry", fd_err)
    assert fd_err < TOL_C64
    # (iii) oracle gradient on sub-slices of the same tree, leaf by leaf
    ext = extend_slices(net, tree, sliced, 30.0)
    ids = [0, 5]
    go = np.array(2 * c)
    sub = _plan(net, tree, ext, "c64_4m")
    g_sub = sub.backward(leaves, torch.from_numpy(go), wrt, slice_ids=ids)
    torch.cuda.synchronize()
    ref = oracle_lib.grad(net64, tree, go, wrt, sliced=ext, slice_ids=ids)
    got = [x.cpu().numpy() for x in g_sub]
    note("cfg4 sub-slice gradient rel err (all leaves)",
         rel(np.concatenate([x.ravel() for x in got]), np.concatenate([r.ravel() for r in ref])))
    _per_leaf(got, ref, TOL_C64, "cfg4 sub-slice gradient")


@pytest.mark.parametrize("prec", ["c64_4m", "c64_3m"])
def test_backward_direct_to_lds(oracle_lib, prec):
    """Gradient contractions on the direct-to-LDS matrix-core variants: with
    A(M, K) or A(K, M) and B(K, N) the gradient of A sums N, the lowest axes
    of both the cotangent and B, and reads B conjugated."""
    import torch

    from tests.gpu_util import TOL_3M
    from tn_inputs.network import Network, Tree
    two = Tree(np.array([0], np.int32), np.array([1], np.int32))
    tol = TOL_3M if prec == "c64_3m" else TOL_C64
    m, n, k = 8, 9, 7
    M, K, N = list(range(m)), list(range(m, m + k)), list(range(m + k, m + k + n))
    for case, ia in (("MK,KN", M + K), ("KM,KN", K + M)):
        rng = np.random.default_rng(len(case) + len(ia))
        a = rng.normal(size=(2,) * (m + k)) + 1j * rng.normal(size=(2,) * (m + k))
        b = rng.normal(size=(2,) * (k + n)) + 1j * rng.normal(size=(2,) * (k + n))
        net = Network([a, b], [ia, K + N], [2] * (m + n + k), M + N)
        go = rng.normal(size=(2,) * (m + n)) + 1j * rng.normal(size=(2,) * (m + n))
        refs = oracle_lib.grad(net, two, go, [0, 1])
        ref = np.concatenate([r.ravel() for r in refs])
        for t in (7, 8, 9):
            plan = _plan(net, two, precision=prec, gemm_all_sizes=True)
            plan.backward_info([0, 1])
            plan.set_tile(0)           # off the direct-to-LDS default, so that pinning t changes the op
            changed = plan.set_tile(t)
            note("backward dl", prec, case, "tile", t, "changed", changed)
            assert changed >= 1
            grads = plan.backward(to_dev(net, prec), torch.from_numpy(go), [0, 1])
            torch.cuda.synchronize()
            got = np.concatenate([g.cpu().numpy().ravel() for g in grads])
            assert rel(got, ref) < tol, (case, t)


@pytest.mark.parametrize("prec", ["c128", "c64_4m", "c64_3m"])
def test_backward_split_k(oracle_lib, prec):
    """A(M, K) x B(K, N) with a small A and a long free side of B: the
    gradient of A sums 2^14 values into 2^12 outputs, a split-K GEMM whose
    partial tiles are summed in a fixed order (twice: bitwise repeatable)."""
    import torch

    from tests.gpu_util import TOL_3M
    from tn_inputs.network import Network, Tree
    two = Tree(np.array([0], np.int32), np.array([1], np.int32))
    tol = {"c128": TOL_C128, "c64_4m": TOL_C64, "c64_3m": TOL_3M}[prec]
    m, k, n = 6, 6, 14
    M, K, N = list(range(m)), list(range(m, m + k)), list(range(m + k, m + k + n))
    rng = np.random.default_rng(7)
    a = rng.normal(size=(2,) * (m + k)) + 1j * rng.normal(size=(2,) * (m + k))
    b = rng.normal(size=(2,) * (k + n)) + 1j * rng.normal(size=(2,) * (k + n))
    net = Network([a, b], [M + K, K + N], [2] * (m + n + k), M + N)
    go = rng.normal(size=(2,) * (m + n)) + 1j * rng.normal(size=(2,) * (m + n))
    ref = oracle_lib.grad(net, two, go, [0])[0]
    plan = _plan(net, two, precision=prec, gemm_all_sizes=True)
    note("backward split-k", prec)
    g1 = plan.backward(to_dev(net, prec), torch.from_numpy(go), [0])[0].cpu().numpy()
    g2 = plan.backward(to_dev(net, prec), torch.from_numpy(go), [0])[0].cpu().numpy()
    torch.cuda.synchronize()
    assert rel(g1, ref) < tol
    assert np.array_equal(g1, g2)


@pytest.mark.parametrize("prec", ["c128", "c64_4m"])
@pytest.mark.parametrize("shape", [(13, 2, 13), (14, 2, 12), (13, 1, 13)])
def test_backward_one_shot_smallk(oracle_lib, shape, prec):
    """A(M, K) x B(N, K) with a short free side N: the gradient of A sums only
    N (two or four values) into 2^(m + k) = 2^26 outputs, which the one-shot
    few-summed-values kernel writes from B read conjugated (its only
    conjugated use: forward programs never conjugate)."""
    import torch

    from tn_inputs.network import Network, Tree
    two = Tree(np.array([0], np.int32), np.array([1], np.int32))
    m, n, k = shape
    M, K, N = list(range(m)), list(range(m, m + k)), list(range(m + k, m + k + n))
    rng = np.random.default_rng(sum(shape) + 5)
    a = rng.normal(size=(2,) * (m + k)) + 1j * rng.normal(size=(2,) * (m + k))
    b = rng.normal(size=(2,) * (n + k)) + 1j * rng.normal(size=(2,) * (n + k))
    net = Network([a, b], [M + K, N + K], [2] * (m + n + k), M + N)
    plan = _plan(net, two, precision=prec)
    kernels = plan.backward_kernels([0])
    note("backward one-shot smallk", prec, shape, kernels)
    assert "gemm_smallk_wide" in kernels
    go = rng.normal(size=(2,) * (m + n)) + 1j * rng.normal(size=(2,) * (m + n))
    rnet = net if prec == "c128" else c64_leaves(net)
    ref = oracle_lib.grad(rnet, two, go, [0])
    got = plan.backward(to_dev(net, prec), torch.from_numpy(go), [0])
    torch.cuda.synchronize()
    _per_leaf([g.cpu().numpy() for g in got], ref, TOL_C128 if prec == "c128" else TOL_C64,
              "backward one-shot smallk " + prec)
