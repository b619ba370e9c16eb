"""torch.autograd.Function over libtn's sliced contraction and its adjoint.

Forward: tn_contract_sliced (FP64 sum over the slice ids, complex128 result).
Backward: tn_contract_backward, which recomputes forward intermediates from
checkpoints along the same tree and contracts each parent cotangent with the
conjugate of the sibling (Sec. 2 pairwise products, reversed).  The incoming
gradient is PyTorch's for a complex output (for L = |R|^2 it is 2 R); leaf
gradients follow the same convention: grad[k] = sum_o conj(dR_o/dT[k]) g[o].
"""

from __future__ import annotations

import torch


class TNContract(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, slice_ids, *leaves):
        leaves = [t.contiguous() for t in leaves]
        out = plan.contract_sliced(leaves, slice_ids=slice_ids)
        ctx.plan = plan
        ctx.slice_ids = slice_ids
        ctx.save_for_backward(*leaves)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        leaves = list(ctx.saved_tensors)
        need = [i for i, n in enumerate(ctx.needs_input_grad[2:]) if n]
        result = [None] * len(leaves)
        if need:
            grads = ctx.plan.backward(leaves, grad_out.contiguous(), wrt=need, slice_ids=ctx.slice_ids)
            for i, g in zip(need, grads):
                result[i] = g
        return (None, None, *result)


def contract(plan, leaves, slice_ids=None):
    """Differentiable sliced contraction of `leaves` with a compiled plan."""
    return TNContract.apply(plan, slice_ids, *leaves)
