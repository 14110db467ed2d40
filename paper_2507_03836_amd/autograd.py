"""torch.autograd.Function over the fused encoding + decoder kernels.

forward:  y = MLP(encode(pos))            -> fhash_fused_fwd
backward: d_table, d_params from dL/dy    -> fhash_fused_bwd
Only the inputs are saved: the backward recomputes the corner weights, the
encoding and the decoder activations inside the kernel instead of storing them.
"""
from __future__ import annotations

import torch

from . import _lib as fl


class FHashFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, table, mlp_params, index, mlp):
        n = pos.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=pos.device)
        fl.fhash_fused_fwd(index, mlp, pos, n, table, mlp_params, y)
        ctx.save_for_backward(pos, table, mlp_params)
        ctx.index, ctx.mlp = index, mlp
        return y

    @staticmethod
    def backward(ctx, dy):
        pos, table, mlp_params = ctx.saved_tensors
        dy = dy.contiguous().float()
        d_table = torch.zeros(table.shape, dtype=torch.float32, device=table.device)
        d_params = torch.zeros_like(mlp_params)
        fl.fhash_fused_bwd(ctx.index, ctx.mlp, pos, pos.shape[0], table, mlp_params, dy,
                           d_table, d_params)
        return None, d_table, d_params, None, None


def fhash_apply(pos, table, mlp_params, index, mlp):
    """Differentiable F-Hash decoder output y[n] for positions pos[n][4]."""
    return FHashFunction.apply(pos, table, mlp_params, index, mlp)
