"""Random grid circuits as tensor networks (Sec. 4.6; transition amplitude eq. trans-amp).

Conventions (the paper fixes only the gate families, not these details):
  * qubit q = r * C + c on an R x C grid;
  * bit of qubit q in bitstring b is (b >> (N - 1 - q)) & 1;
  * a cycle is a layer of single-qubit gates on every qubit, drawn iid and
    uniformly from {sqrtX, sqrtY, sqrtW}, followed by fSim(pi/2, pi/6) on every
    coupler of that cycle's pattern; one more single-qubit layer follows the
    last cycle;
  * coupler patterns cycle A, B, C, D: A = horizontal (r,c)-(r,c+1) with c
    even, B = the same with c odd, C = vertical (r,c)-(r+1,c) with r even,
    D = the same with r odd;
  * leaves: rank-1 input states |0>, rank-2 single-qubit gates with axes
    (out, in), rank-4 two-qubit gates with axes (o_a, o_b, i_a, i_b) holding
    U[(o_a o_b), (i_a i_b)], a the lower-numbered qubit of the coupler, and
    rank-1 output projectors <b_q| (Sec. 4.6.1: rank-1 states, rank-2
    single-qubit gates, rank-4 two-qubit gates);
  * qubits listed in `open_qubits` get no output projector: their last wire
    index is an open output index, in ascending q order (Sec. 4.7.3: N_f
    output indices left open).

By default no gate decomposition and no simplification is applied, so every
fSim stays a rank-4 leaf, as in the Sycamore-53 rows of the benchmark table.
With decompose="swap_diag" every fSim(pi/2, phi) is written exactly as a SWAP
after the diagonal gate diag(1, -i, -i, e^{-i phi}) (Sec. 3.5 / 4.6.2: gates
that are diagonal in the computational basis act on hyperedges): its leaf is
the rank-2 tensor D[x_a, x_b] on the two incoming wire indices, which then
continue on the swapped qubits.  Wire indices become hyperedges (the gate that
produced the wire, the diagonal tensor, the next gate), as in the paper's
hyperedge rows of the benchmark table.
"""

from __future__ import annotations

import numpy as np

from .network import Network

_S2 = np.sqrt(0.5)


def _rot(pauli: np.ndarray) -> np.ndarray:
    """exp(-i pi/4 P) for a Pauli-like P with P @ P = I."""
    return np.cos(np.pi / 4) * np.eye(2, dtype=np.complex128) - 1j * np.sin(np.pi / 4) * pauli


PAULI_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PAULI_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PAULI_W = (PAULI_X + PAULI_Y) * _S2

SQRT_X = _rot(PAULI_X)
SQRT_Y = _rot(PAULI_Y)
SQRT_W = _rot(PAULI_W)
ONE_QUBIT_GATES = (SQRT_X, SQRT_Y, SQRT_W)


def fsim(theta: float, phi: float) -> np.ndarray:
    """fSim(theta, phi) in the basis |00>,|01>,|10>,|11> of (a, b)."""
    c, s = np.cos(theta), np.sin(theta)
    u = np.zeros((4, 4), dtype=np.complex128)
    u[0, 0] = 1.0
    u[1, 1] = c
    u[1, 2] = -1j * s
    u[2, 1] = -1j * s
    u[2, 2] = c
    u[3, 3] = np.exp(-1j * phi)
    return u


FSIM = fsim(np.pi / 2, np.pi / 6)


def coupler_patterns(R: int, C: int):
    """The four coupler patterns A, B, C, D as lists of (qa, qb), qa < qb."""
    A = [(r * C + c, r * C + c + 1) for r in range(R) for c in range(0, C - 1, 2)]
    B = [(r * C + c, r * C + c + 1) for r in range(R) for c in range(1, C - 1, 2)]
    Cv = [(r * C + c, (r + 1) * C + c) for r in range(0, R - 1, 2) for c in range(C)]
    D = [(r * C + c, (r + 1) * C + c) for r in range(1, R - 1, 2) for c in range(C)]
    return [A, B, Cv, D]


def random_circuit(R: int, C: int, m: int, seed: int):
    """Gate list [(kind, qubits, matrix)] in time order; kind in {'1q', '2q'}."""
    rng = np.random.default_rng(seed)
    pats = coupler_patterns(R, C)
    N = R * C
    gates = []
    for cyc in range(m + 1):
        choice = rng.integers(0, 3, size=N)
        for q in range(N):
            gates.append(("1q", (q,), ONE_QUBIT_GATES[int(choice[q])]))
        if cyc == m:
            break
        for (qa, qb) in pats[cyc % 4]:
            gates.append(("2q", (qa, qb), FSIM))
    return gates


def bit_of(b: int, q: int, N: int) -> int:
    return (b >> (N - 1 - q)) & 1


def swap_diag_factor(u: np.ndarray):
    """(d, ok): U = SWAP . diag(d) for a 4x4 U (basis |00>,|01>,|10>,|11>)?"""
    swap = np.eye(4, dtype=np.complex128)[[0, 2, 1, 3]]
    d = np.diag(swap @ u).copy()
    return d, bool(np.allclose(swap @ np.diag(d), u, atol=1e-14))


def circuit_network(R: int, C: int, m: int, seed: int, bitstring: int,
                    open_qubits=(), decompose: str = "none") -> Network:
    """Network for <b| U |0^N> with `open_qubits` left open (ascending q);
    decompose in {"none", "swap_diag"} (see the module docstring)."""
    if decompose not in ("none", "swap_diag"):
        raise ValueError(f"unknown decomposition {decompose!r}")
    N = R * C
    gates = random_circuit(R, C, m, seed)
    open_set = set(open_qubits)
    leaves, leaf_idx, kinds = [], [], []
    n_idx = 0
    wire = [0] * N
    zero = np.array([1.0, 0.0], dtype=np.complex128)
    for q in range(N):
        wire[q] = n_idx
        n_idx += 1
        leaves.append(zero.copy())
        leaf_idx.append([wire[q]])
        kinds.append("in")
    for kind, qs, u in gates:
        if kind == "1q":
            (q,) = qs
            o = n_idx
            n_idx += 1
            leaves.append(u.copy())
            leaf_idx.append([o, wire[q]])
            kinds.append("1q")
            wire[q] = o
        elif decompose == "swap_diag":
            qa, qb = qs
            d, ok = swap_diag_factor(u)
            if not ok:
                raise ValueError("two-qubit gate is not SWAP times a diagonal gate")
            leaves.append(d.reshape(2, 2).copy())          # D[x_a, x_b] = d[2 x_a + x_b]
            leaf_idx.append([wire[qa], wire[qb]])
            kinds.append("2q")
            wire[qa], wire[qb] = wire[qb], wire[qa]
        else:
            qa, qb = qs
            oa, ob = n_idx, n_idx + 1
            n_idx += 2
            leaves.append(u.reshape(2, 2, 2, 2).copy())
            leaf_idx.append([oa, ob, wire[qa], wire[qb]])
            kinds.append("2q")
            wire[qa], wire[qb] = oa, ob
    for q in range(N):
        if q in open_set:
            continue
        proj = np.zeros(2, dtype=np.complex128)
        proj[bit_of(bitstring, q, N)] = 1.0
        leaves.append(proj)
        leaf_idx.append([wire[q]])
        kinds.append("out")
    out_idx = [wire[q] for q in sorted(open_set)]
    net = Network(leaves, leaf_idx, [2] * n_idx, out_idx,
                  meta=dict(kind="circuit", R=R, C=C, m=m, seed=seed, bitstring=bitstring,
                            open_qubits=tuple(sorted(open_set)), leaf_kinds=kinds, gates=gates,
                            decompose=decompose))
    net.check()
    return net


def gate_leaves(net: Network, kind: str = "2q"):
    """Leaf ids of the given kind ('in', '1q', '2q', 'out')."""
    return [v for v, k in enumerate(net.meta["leaf_kinds"]) if k == kind]
