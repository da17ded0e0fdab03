"""torch.autograd wrapper of the wkern generator.

``WKernFunction.apply(taper, w, plan)`` returns the flat complex64 kernel
cache; its backward calls the library's hand-written adjoint (``wkern_grad``)
and returns dL/dtaper (float32) and dL/dw (float64).  torch's convention for
the gradient of a real loss with respect to a complex tensor,
dL/dRe + j dL/dIm, is the one ``wkern_grad`` takes.
"""
from __future__ import annotations

import torch


class WKernFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, taper, w, plan):
        out = plan.generate(taper, w)
        ctx.plan = plan
        ctx.save_for_backward(taper, w)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        taper, w = ctx.saved_tensors
        g_taper, g_w = ctx.plan.grad(taper, w, grad_out.contiguous())
        return g_taper, g_w, None


def wkernels(taper, w, plan):
    """Differentiable kernel generation (see WKernFunction)."""
    return WKernFunction.apply(taper, w, plan)
