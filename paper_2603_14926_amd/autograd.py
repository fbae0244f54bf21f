"""torch.autograd.Function wrappers over the libmpx kernels.

GEMM: C = A B with component-plane tensors (K, m, k) x (K, k, n).  The
backward is two more GEMMs through the same kernel with transpose flags:
  dA = dC B^T   (mpx_gemm, transB = 1),   dB = A^T dC   (mpx_gemm, transA = 1).
Horner: y_b = p_b(x_b) for coefficient tensors (K, batch, deg+1); the
backward calls mpx_polyval_backward (coefficient gradient by the adjoint of
the Horner recurrence, x gradient by the derivative recurrence).

Gradients are multicomponent tensors of the same layout; autograd only routes
them (no torch arithmetic touches the components).

Cotangent convention: the gradient arriving at a multicomponent output is
read as ONE multicomponent number per entry, the unevaluated sum of its K
planes, and the gradients returned for the inputs have the same form.
Torch's own operations do not follow it: composing a multicomponent output
with a plain torch reduction, e.g. gemm(A, B).sum(), hands every plane a
gradient of 1, i.e. the number K, so the input gradients come out K times
too large in plane 0.  Route such losses through to_value(), whose backward
hands the incoming binary64 gradient on as (g, 0, ..., 0):
    to_value(gemm(A, B)).sum().backward()
gives the gradients of the sum of the entries' values.
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


class MpValue(torch.autograd.Function):
    """Multicomponent planes (K, ...) -> their leading components (...), the
    values to binary64 precision (no arithmetic: a copy of plane 0).  Its
    backward turns a plain gradient g into the multicomponent cotangent
    (g, 0, ..., 0)."""

    @staticmethod
    def forward(ctx, x):
        ctx.K = x.shape[0]
        return x[0].clone()

    @staticmethod
    def backward(ctx, g):
        out = torch.zeros((ctx.K,) + tuple(g.shape), dtype=g.dtype, device=g.device)
        out[0] = g
        return out


def to_value(x):
    return MpValue.apply(x)

