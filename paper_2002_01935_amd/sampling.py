"""Approximately unbiased sampling of a chaotic circuit at fidelity f from
contractions with N_f output qubits left open (Sec. 4.7.3, estimated runtime of
sampling Sycamore).

For a chaotic circuit the marginal on N_u = N - N_f qubits is taken as
uniform, so a sample is drawn as follows: x_u uniform over the closed qubits;
the 2^N_f amplitudes <x_u x_f|psi> from one sliced contraction whose output
bras on the closed qubits are set to x_u; x_f drawn from
p(x_f | x_u) = |<x_u x_f|psi>|^2 / Z.  Fidelity f is simulated by sampling
rho = (1 - f) 1 / 2^N + f |psi><psi|: with probability f / g (g the fidelity of
psi itself, e.g. below 1 after a lossy gate decomposition) the sample comes
from psi, otherwise it is a uniform N-bit string.  One contraction per sample
from psi: M samples cost about M f / g contractions.

Bitstrings follow the circuit convention: the bit of qubit q is
(b >> (N - 1 - q)) & 1.  Random numbers come from the caller's
numpy Generator in a fixed order per sample (one uniform draw for the
mixture, then either x_u and x_f or the uniform string), so a seed fixes the
samples.
"""

from __future__ import annotations

import numpy as np


def compose(n_qubits, closed, opened, x_u, x_f):
    """N-bit string from the closed-qubit bits x_u (first closed qubit most
    significant) and the open-qubit bits x_f (first open qubit most
    significant)."""
    b = 0
    for i, q in enumerate(closed):
        b |= ((x_u >> (len(closed) - 1 - i)) & 1) << (n_qubits - 1 - q)
    for i, q in enumerate(opened):
        b |= ((x_f >> (len(opened) - 1 - i)) & 1) << (n_qubits - 1 - q)
    return b


def draw(n_samples, fidelity, rng, n_qubits, closed, opened, conditional, g=1.0):
    """Samples and the number of contractions spent.  `conditional(x_u)`
    returns p(x_f | x_u) as a length-2^N_f vector (first open qubit most
    significant)."""
    if not 0.0 <= fidelity <= 1.0 or g <= 0.0:
        raise ValueError("need 0 <= fidelity <= 1 and g > 0")
    f_eff = min(1.0, fidelity / g)
    out, contractions = [], 0
    for _ in range(n_samples):
        if rng.random() < f_eff:
            x_u = int(rng.integers(0, 1 << len(closed)))
            p = conditional(x_u)
            contractions += 1
            x_f = int(rng.choice(len(p), p=p))
            out.append(compose(n_qubits, closed, opened, x_u, x_f))
        else:
            out.append(int(rng.integers(0, 1 << n_qubits)))
    return out, contractions


class CircuitSampler:
    """Sampler over a compiled plan of a circuit network with open qubits.

    `leaves` are the plan's device tensors (complex64 or complex128);
    `out_leaves[i]` is the leaf id of the output bra on closed qubit
    `closed[i]` (ascending qubits); the plan's output axes are the open
    qubits in ascending order.  The bras are overwritten in place for every
    x_u; the plan is reused (a plan depends on the network's structure only).
    """

    def __init__(self, plan, leaves, n_qubits, closed, opened, out_leaves, slice_ids=None, workspace=None):
        import torch
        if len(out_leaves) != len(closed):
            raise ValueError("one output bra per closed qubit")
        if plan.out_shape != (2,) * len(opened):
            raise ValueError("the plan's outputs must be the open qubits")
        self.plan, self.leaves = plan, leaves
        self.n_qubits, self.closed, self.opened = n_qubits, list(closed), list(opened)
        self.out_leaves = list(out_leaves)
        self.slice_ids = slice_ids
        self.workspace = workspace if workspace is not None else plan.workspace()
        dt = plan.storage_dtype
        self._bra = [torch.tensor([1.0, 0.0], dtype=dt, device="cuda"),
                     torch.tensor([0.0, 1.0], dtype=dt, device="cuda")]

    def amplitudes(self, x_u):
        """<x_u x_f|psi> for every x_f (complex128 array, one axis per open qubit)."""
        for i, v in enumerate(self.out_leaves):
            bit = (x_u >> (len(self.closed) - 1 - i)) & 1
            self.leaves[v].copy_(self._bra[bit].reshape(self.leaves[v].shape))
        amp = self.plan.contract_sliced(self.leaves, slice_ids=self.slice_ids, workspace=self.workspace)
        return amp.cpu().numpy()

    def conditional(self, x_u):
        p = np.abs(self.amplitudes(x_u).ravel()) ** 2
        z = p.sum()
        if not z > 0:
            raise ValueError("all amplitudes of this x_u vanish")
        return p / z

    def sample(self, n_samples, fidelity, rng, g=1.0):
        return draw(n_samples, fidelity, rng, self.n_qubits, self.closed, self.opened, self.conditional, g)
