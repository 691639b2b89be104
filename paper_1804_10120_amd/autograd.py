"""Differentiable fused chain: forward tl_dtg_chain, backward tl_dtg_chain_bwd.

Only the inputs are saved; the backward kernel recomputes g^ij and b^l = g^lk
beta_k instead of storing them.  Gradients are taken with respect to the
stored components (a [6, n] symmetric field gets the sum of the (i,j) and (j,i)
partials in an off-diagonal slot), which is what torch's autograd and finite
differences on the [6, n] storage both measure.  The backward is not itself
differentiable (second derivatives raise).
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from .ops import tl_dtg_chain, tl_dtg_chain_bwd


class DtgChainFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g, dg, beta, dbeta, K, alpha, tune=None):
        out = tl_dtg_chain(g, dg, beta, dbeta, K, alpha, tune=tune)
        ctx.save_for_backward(g, dg, beta, K, alpha)
        ctx.tune = tune
        return out

    @staticmethod
    @once_differentiable
    def backward(ctx, w):
        g, dg, beta, K, alpha = ctx.saved_tensors
        want = ctx.needs_input_grad[:6]
        if not any(want):
            return (None,) * 7
        grads = tl_dtg_chain_bwd(g, dg, beta, K, alpha, w.contiguous(), want=want,
                                 tune=ctx.tune)
        return (*grads, None)


def dtg_chain(g, dg, beta, dbeta, K, alpha, tune=None):
    """d_t g_ij of the fused chain, differentiable with respect to every input."""
    return DtgChainFn.apply(g, dg, beta, dbeta, K, alpha, tune)
