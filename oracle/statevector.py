"""Brute-force statevector amplitudes (tree-free reference for circuits).

TEST INFRASTRUCTURE ONLY.  Applies the gates of a circuit, in time order, to a
2^N complex128 vector starting from |0^N>, and reads the transition amplitude
c_x = <x| U_d ... U_1 |0^N> of eq. (trans-amp).  Qubit q is axis q of the
(2,)*N state array, so the bit of qubit q in an integer bitstring b is
(b >> (N - 1 - q)) & 1.  Two-qubit gates act on (a, b) with
U[(o_a o_b), (i_a i_b)].
"""

from __future__ import annotations

import numpy as np


def run(N: int, gates, replace=None) -> np.ndarray:
    """Final state, shape (2,)*N.  `replace` maps a gate position in `gates`
    to a substitute matrix (used for brute-force environments)."""
    psi = np.zeros((2,) * N, dtype=np.complex128)
    psi[(0,) * N] = 1.0
    for k, (kind, qs, u) in enumerate(gates):
        if replace is not None and k in replace:
            u = replace[k]
        if kind == "1q":
            (q,) = qs
            psi = np.tensordot(u, psi, axes=([1], [q]))
            psi = np.moveaxis(psi, 0, q)
        else:
            a, b = qs
            g = np.asarray(u).reshape(2, 2, 2, 2)
            psi = np.tensordot(g, psi, axes=([2, 3], [a, b]))
            psi = np.moveaxis(psi, [0, 1], [a, b])
    return psi


def amplitude(N: int, gates, bitstring: int, open_qubits=(), state=None) -> np.ndarray:
    """Amplitudes with the closed qubits fixed to `bitstring`; open qubits stay
    as axes in ascending q order."""
    psi = run(N, gates) if state is None else state
    idx = []
    open_set = set(open_qubits)
    for q in range(N):
        if q in open_set:
            idx.append(slice(None))
        else:
            idx.append((bitstring >> (N - 1 - q)) & 1)
    return np.asarray(psi[tuple(idx)])
