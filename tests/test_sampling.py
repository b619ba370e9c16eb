"""Sampling driver (Sec. 4.7.3): bit composition, the fidelity mixture and the
conditional distributions, pinned against the brute-force statevector."""

import numpy as np
import pytest

from oracle import statevector as sv
from paper_2002_01935_amd.sampling import compose, draw
from tn_inputs.circuits import circuit_network, gate_leaves, random_circuit

R, C, M_CYC, SEED = 3, 3, 8, 4
N = R * C
OPEN = (3, 4, 5)
CLOSED = tuple(q for q in range(N) if q not in OPEN)


def _psi():
    return sv.run(N, random_circuit(R, C, M_CYC, SEED))


def _sv_conditional(psi):
    def cond(x_u):
        b = compose(N, CLOSED, OPEN, x_u, 0)
        p = np.abs(sv.amplitude(N, None, b, OPEN, state=psi).ravel()) ** 2
        return p / p.sum()
    return cond


def test_compose_bit_order():
    # N = 4, closed qubits 0 and 2 carry x_u = 0b10, open qubits 1 and 3 carry x_f = 0b01
    assert compose(4, [0, 2], [1, 3], 0b10, 0b01) == 0b1001
    assert compose(4, [0, 2], [1, 3], 0b01, 0b10) == 0b0110
    # every (x_u, x_f) maps to a distinct bitstring
    got = {compose(N, CLOSED, OPEN, u, f) for u in range(1 << len(CLOSED)) for f in range(1 << len(OPEN))}
    assert got == set(range(1 << N))


def _tv(samples, expected):
    hist = np.bincount(np.asarray(samples), minlength=len(expected)) / len(samples)
    return 0.5 * np.abs(hist - expected).sum()


@pytest.mark.parametrize("fidelity,g", [(1.0, 1.0), (0.0, 1.0), (0.3, 0.6)])
def test_mixture_distribution(fidelity, g):
    """Empirical distribution of 200k seeded samples vs the exact mixture
    (1 - f~) / 2^N + f~ 2^-N_u p(x_f | x_u), f~ = f / g, with the statevector's
    conditional distributions; the number of contractions is f~ M."""
    psi = _psi()
    cond = _sv_conditional(psi)
    n = 200_000
    samples, contractions = draw(n, fidelity, np.random.default_rng(1), N, CLOSED, OPEN, cond, g)
    f_eff = min(1.0, fidelity / g)
    prob = np.abs(psi.ravel()) ** 2
    # P(b) from psi: x_u uniform, then p(x_f | x_u)
    from_psi = np.zeros(1 << N)
    for u in range(1 << len(CLOSED)):
        p = cond(u)
        for f in range(1 << len(OPEN)):
            from_psi[compose(N, CLOSED, OPEN, u, f)] = p[f] / (1 << len(CLOSED))
    expected = (1 - f_eff) / (1 << N) + f_eff * from_psi
    assert abs(expected.sum() - 1) < 1e-12
    assert _tv(samples, expected) < 0.03
    assert abs(contractions - f_eff * n) < 5 * np.sqrt(n * f_eff * (1 - f_eff) + 1)
    if fidelity == 1.0:
        # samples from psi are not the Porter-Thomas distribution itself
        # (x_u is uniform), but they favour the heavy outputs of each x_u
        assert np.mean(prob[np.asarray(samples)]) > 1.5 / (1 << N)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["c64_4m", "c128"])
def test_sampler_on_gpu_plan(prec):
    """CircuitSampler on a compiled plan: p(x_f | x_u) from the GPU contraction
    equals the statevector's; with complex128 the seeded sample sequence is
    the one the same draw gives with the statevector's conditionals."""
    import torch

    from paper_2002_01935_amd.binding import Plan
    from paper_2002_01935_amd.sampling import CircuitSampler
    from tests.gpu_util import note, to_dev
    from tn_inputs.greedy import find_tree
    net = circuit_network(R, C, M_CYC, SEED, 0, open_qubits=OPEN)
    tree = find_tree(net, seed=0, trials=2)
    plan = Plan(net, tree, precision=prec)
    leaves = to_dev(net, prec)
    sampler = CircuitSampler(plan, leaves, N, CLOSED, OPEN, gate_leaves(net, "out"))
    psi = _psi()
    cond = _sv_conditional(psi)
    tol = 1e-10 if prec == "c128" else 1e-5
    for x_u in (0, 5, 37, 63):
        note("sampler conditional", prec, x_u)
        got = sampler.conditional(x_u)
        ref = cond(x_u)
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < tol
    if prec == "c128":
        a, na = sampler.sample(200, 0.5, np.random.default_rng(7))
        b, nb = draw(200, 0.5, np.random.default_rng(7), N, CLOSED, OPEN, cond)
        torch.cuda.synchronize()
        assert a == b and na == nb
