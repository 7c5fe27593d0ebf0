"""torch.autograd wrappers of the filter, the Gaussian-kernel weights and the
row-normalised loss (gradients by the hand-written adjoint kernels of libasc).

    w    = GaussWeights.apply(d2, sigma)          # sigma: 0-d float64 tensor
    Y    = ChebFilter.apply(w, coeffs, graph, lmax, R, ckpt_stride)
    loss = RowNormLoss.apply(Y, target)
    loss.backward()   # -> d2.grad is not produced; sigma.grad, coeffs.grad, w.grad

lambda_max is a constant of the differentiation (detached), as is R.
"""
from __future__ import annotations

import math

import torch

from . import (cheb_filter, cheb_filter_bwd, gauss_weights, gauss_weights_bwd, graph_prepare,
               rownorm_loss_bwd)


def default_ckpt_stride(p: int) -> int:
    return max(2, int(math.ceil(math.sqrt(max(p, 1)))))


def _aligned_copy(t: torch.Tensor) -> torch.Tensor:
    n, r = t.shape
    buf = torch.empty(n, (r + 3) // 4 * 4, dtype=torch.float32, device=t.device)[:, :r]
    buf.copy_(t)
    return buf


class GaussWeights(torch.autograd.Function):
    @staticmethod
    def forward(ctx, d2: torch.Tensor, sigma: torch.Tensor):
        s = float(sigma.detach().cpu())
        w = gauss_weights(d2, s)
        ctx.save_for_backward(d2, w)
        ctx.sigma = s
        ctx.sigma_meta = (sigma.dtype, sigma.device, sigma.shape)
        return w

    @staticmethod
    def backward(ctx, dW: torch.Tensor):
        d2, w = ctx.saved_tensors
        ds = None
        if ctx.needs_input_grad[1]:
            dtype, device, shape = ctx.sigma_meta
            ds = gauss_weights_bwd(d2, w, dW.contiguous(), ctx.sigma).to(device=device, dtype=dtype).reshape(shape)
        return None, ds


class ChebFilter(torch.autograd.Function):
    """Y = sum_j a_j T_j(Lt) R for the graph (row_ptr, col_idx) with weights w."""

    @staticmethod
    def forward(ctx, w, coeffs, row_ptr, col_idx, lmax, R, ckpt_stride=None):
        p = coeffs.numel() - 1
        c = ckpt_stride or default_ckpt_stride(p)
        g = graph_prepare(row_ptr, col_idx, w.detach())
        a = coeffs.detach().to(torch.float64).contiguous()
        Y, ck = cheb_filter(g, lmax, a, R, ckpt_stride=c)
        ctx.g, ctx.ck, ctx.c = g, ck, c
        ctx.save_for_backward(a, lmax, R)
        ctx.coeffs_dtype = coeffs.dtype
        return Y

    @staticmethod
    def backward(ctx, gY):
        a, lmax, R = ctx.saved_tensors
        G = gY if (gY.stride(1) == 1 and gY.stride(0) % 4 == 0 and gY.data_ptr() % 16 == 0) else _aligned_copy(gY)
        want_w, want_a = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        dW, dc = cheb_filter_bwd(ctx.g, lmax, a, R, ctx.ck, ctx.c, G, want_dw=want_w, want_dcoeffs=want_a)
        return dW, (dc.to(ctx.coeffs_dtype) if dc is not None else None), None, None, None, None, None


class RowNormLoss(torch.autograd.Function):
    """loss = sum_i |y_i / |y_i| - t_i|^2 (float64 scalar)."""

    @staticmethod
    def forward(ctx, Y, target):
        loss, G = rownorm_loss_bwd(Y, target)
        ctx.save_for_backward(G)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, gl):
        (G,) = ctx.saved_tensors
        return G * gl.to(G.dtype), None
