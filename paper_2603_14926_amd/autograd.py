"""torch.autograd.Function wrappers over the libmpx kernels.

GEMM: C = A B with component-plane tensors (K, m, k) x (K, k, n).  The
backward is two more GEMMs through the same kernel with transpose flags:
  dA = dC B^T   (mpx_gemm, transB = 1),   dB = A^T dC   (mpx_gemm, transA = 1).
Horner: y_b = p_b(x_b) for coefficient tensors (K, batch, deg+1); the
backward calls mpx_polyval_backward (coefficient gradient by the adjoint of
the Horner recurrence, x gradient by the derivative recurrence).

Gradients are multicomponent tensors of the same layout; autograd only routes
them (no torch arithmetic touches the components).
"""
from __future__ import annotations

import torch

from . import mpx


class MpGemm(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, prec):
        ctx.prec = prec
        ctx.save_for_backward(A, B)
        return mpx.gemm(prec, A, B)

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        dC = dC.contiguous()
        dA = dB = None
        if ctx.needs_input_grad[0]:
            dA = mpx.gemm(ctx.prec, dC, B, transB=True)
        if ctx.needs_input_grad[1]:
            dB = mpx.gemm(ctx.prec, A, dC, transA=True)
        return dA, dB, None


class MpPolyval(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coef, x, prec):
        ctx.prec = prec
        ctx.save_for_backward(coef, x)
        return mpx.polyval(prec, coef, x)

    @staticmethod
    def backward(ctx, gy):
        coef, x = ctx.saved_tensors
        gc, gx = mpx.polyval_backward(ctx.prec, coef, x, gy.contiguous(),
                                      want_coef=ctx.needs_input_grad[0],
                                      want_x=ctx.needs_input_grad[1])
        return gc, gx, None


def gemm(A, B, prec="qd"):
    return MpGemm.apply(A, B, prec)


def polyval(coef, x, prec="qd"):
    return MpPolyval.apply(coef, x, prec)
