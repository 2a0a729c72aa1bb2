"""Differentiation through the PFB: a torch.autograd.Function whose forward is
the HIP forward PFB (y = F S W x, Section 2.3) and whose backward is the
hand-written HIP adjoint ((F S W)^T, needed by the maximum-likelihood form of
Section 4.2).

Gradient convention (torch's, for a real input and complex output): for a
real loss l, grad_x = Re[(F S W)^H grad_y] on the half spectrum, which is
exactly what pfb_adjoint computes (real inner product on x, Re<.,.> on y).
"""
from __future__ import annotations

import torch

from . import ipfb


class PfbFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return ipfb.pfb_forward(plan, x.contiguous())

    @staticmethod
    def backward(ctx, grad_y):
        plan = ctx.plan
        g = grad_y.contiguous()
        if g.dtype != plan.complex_dtype:
            g = g.to(plan.complex_dtype)
        return ipfb.pfb_adjoint(plan, g), None


def pfb(x, plan):
    """Differentiable forward PFB: x [nblock*lblock] real -> [nblock, lblock/2+1] complex."""
    return PfbFunction.apply(x, plan)
