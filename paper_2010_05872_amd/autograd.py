"""torch.autograd Functions over the library's forward and adjoint kernels.

Not part of the paper: decomposition D and recomposition R are linear maps,
and the library provides their transposes (mgx_decompose_adjoint,
mgx_recompose_adjoint), so losses on reconstructed fields can backpropagate
to coefficients and inputs.  Level-wise quantization is treated as
straight-through (its gradient is taken as the identity).
"""
from __future__ import annotations

import torch

from . import decompose, decompose_adjoint, dequantize, quantize, recompose, recompose_adjoint


class Decompose(torch.autograd.Function):
    """u -> u_mc (level-centric).  Backward: D^T."""

    @staticmethod
    def forward(ctx, u, coords=None, stop_level=0):
        ctx.coords, ctx.stop = coords, stop_level
        return decompose(u.contiguous(), coords, stop_level)

    @staticmethod
    def backward(ctx, g):
        return decompose_adjoint(g.contiguous(), ctx.coords, ctx.stop), None, None


class Recompose(torch.autograd.Function):
    """u_mc (level-centric) -> u.  Backward: R^T."""

    @staticmethod
    def forward(ctx, u_mc, coords=None, stop_level=0):
        ctx.coords, ctx.stop = coords, stop_level
        return recompose(u_mc.contiguous(), coords, stop_level)

    @staticmethod
    def backward(ctx, g):
        return recompose_adjoint(g.contiguous(), ctx.coords, ctx.stop), None, None


class QuantizeSTE(torch.autograd.Function):
    """Level-wise quantize then dequantize; identity gradient (straight-through)."""

    @staticmethod
    def forward(ctx, u_mc, tol, coords=None, stop_level=0, c_linf=0.0):
        labels = quantize(u_mc.contiguous(), tol, coords, stop_level, c_linf)
        return dequantize(labels, tol, u_mc.dtype, coords, stop_level, c_linf)

    @staticmethod
    def backward(ctx, g):
        return g, None, None, None, None


class MGXRoundTrip(torch.autograd.Function):
    """y = R(Q(D x) + delta), Q the level-wise quantizer at tolerance `tol`
    (skipped when tol is None).  Backward: g_delta = R^T g and
    g_x = D^T R^T g (straight-through over Q)."""

    @staticmethod
    def forward(ctx, x, delta, coords=None, stop_level=0, tol=None):
        ctx.coords, ctx.stop = coords, stop_level
        c = decompose(x.contiguous(), coords, stop_level)
        if tol is not None:
            c = dequantize(quantize(c, tol, coords, stop_level), tol, x.dtype, coords, stop_level)
        return recompose(c + delta, coords, stop_level)

    @staticmethod
    def backward(ctx, g):
        gc = recompose_adjoint(g.contiguous(), ctx.coords, ctx.stop)
        gx = decompose_adjoint(gc, ctx.coords, ctx.stop)
        return gx, gc, None, None, None
