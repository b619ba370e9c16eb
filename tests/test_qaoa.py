"""QAOA MAX-CUT energy terms (Sec. 4.4): light-cone term networks against the
brute-force statevector, and the GPU path against the oracle per term."""

import numpy as np
import pytest

from oracle import statevector as sv
from tn_inputs.greedy import find_tree
from tn_inputs.qaoa import instance, light_cone, mixer_gate, term_network, zz_gate

CASES = [(10, 2, 0), (16, 1, 3)]        # (N, p, seed): full light cones; pruned light cones


def _sv_terms(n, edges, gammas, betas):
    """<psi| Z_j Z_k |psi> for every edge from the full 2^N state."""
    h = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2)
    gates = [("1q", (q,), h) for q in range(n)]
    for g, b in zip(gammas, betas):
        gates += [("2q", e, zz_gate(g).reshape(4, 4)) for e in edges]
        gates += [("1q", (q,), mixer_gate(b)) for q in range(n)]
    prob = np.abs(sv.run(n, gates)) ** 2
    out = []
    for j, k in edges:
        z = np.ones((2,) * n)
        zj = np.array([1.0, -1.0]).reshape([2 if a == j else 1 for a in range(n)])
        zk = np.array([1.0, -1.0]).reshape([2 if a == k else 1 for a in range(n)])
        out.append(float(np.sum(prob * z * zj * zk)))
    return np.array(out)


def test_light_cone_prunes():
    edges, g, b = instance(16, 1, 3)
    _, _, cone = light_cone(edges, 1, *edges[0])
    assert 4 <= len(cone) <= 6          # the edge, its four other neighbours at most
    _, _, cone2 = light_cone(edges, 2, *edges[0])
    assert len(cone2) > len(cone)


@pytest.mark.parametrize("n,p,seed", CASES)
def test_terms_oracle_vs_statevector(oracle_lib, n, p, seed):
    edges, gammas, betas = instance(n, p, seed)
    ref = _sv_terms(n, edges, gammas, betas)
    got = []
    for j, k in edges:
        net = term_network(edges, gammas, betas, j, k)
        tree = find_tree(net, seed=0, trials=2)
        val = complex(oracle_lib.contract(net, tree))
        assert abs(val.imag) < 1e-10
        got.append(val.real)
    assert np.max(np.abs(np.array(got) - ref)) < 1e-10


@pytest.mark.gpu
@pytest.mark.parametrize("n,p,seed", CASES)
def test_terms_gpu_vs_oracle(oracle_lib, n, p, seed):
    """Every term through its own plan (complex128 within 1e-10 and complex64
    4M within 1e-5 absolute, the terms being real numbers of magnitude at
    most 1), and the energy sum against the statevector."""
    from tests.gpu_util import gpu_contract, note
    edges, gammas, betas = instance(n, p, seed)
    ref_sv = _sv_terms(n, edges, gammas, betas)
    e128, e64 = [], []
    for i, (j, k) in enumerate(edges):
        net = term_network(edges, gammas, betas, j, k)
        tree = find_tree(net, seed=0, trials=2)
        ref = complex(oracle_lib.contract(net, tree))
        note("qaoa term", n, p, i)
        g128 = complex(gpu_contract(net, tree, precision="c128"))
        g64 = complex(gpu_contract(net, tree, precision="c64_4m"))
        assert abs(g128 - ref) < 1e-10
        assert abs(g64 - ref) < 1e-5
        e128.append(g128.real)
        e64.append(g64.real)
    assert abs(sum(e128) - ref_sv.sum()) < 1e-9
    assert abs(sum(e64) - ref_sv.sum()) < 1e-4


@pytest.mark.gpu
def test_full_size_instance_vs_oracle(oracle_lib):
    """The measured instance (N = 54, p = 3, 81 terms): every term's complex64
    value against the oracle's complex128 contraction of the same network
    and tree, and the energy sum."""
    from tests.gpu_util import gpu_contract, note
    edges, gammas, betas = instance(54, 3, 0)
    ref, got = [], []
    for i, (j, k) in enumerate(edges):
        net = term_network(edges, gammas, betas, j, k)
        tree = find_tree(net, seed=0, trials=4)
        if i % 20 == 0:
            note("qaoa full size term", i)
        ref.append(complex(oracle_lib.contract(net, tree)).real)
        got.append(complex(gpu_contract(net, tree, precision="c64_4m")).real)
    assert np.max(np.abs(np.array(got) - np.array(ref))) < 1e-5
    assert abs(sum(got) - sum(ref)) < 1e-4
