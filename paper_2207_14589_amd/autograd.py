"""PolyApply: Y = p_theta(L) X = sum_j theta_j Lt^j X as a torch.autograd.Function.

Learnable dilation coefficients are the paper's stated next step (meta-learning
the polynomial, Sec. 6).  Forward is Horner's rule in the HIP library
(sped_apply_poly).  Backward is hand written:
  dX      = p_theta(L) dY              (L symmetric, so p(L)^T = p(L))
  dtheta_j = <dY, Lt^j X>_F            (sped_poly_backward recomputes the powers
                                        step by step with a fused inner product,
                                        never storing them)
Lt = (L - shift I) / scale.  theta lives on the host side of the call (the
library takes host coefficients), so a device theta is copied once per call.
"""
from __future__ import annotations

import torch

from . import sped


class PolyApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, X: torch.Tensor, L: "sped.Laplacian", shift: float = 0.0,
                scale: float = 1.0):
        th = theta.detach().to("cpu", torch.float64).numpy().copy()
        if th.shape[0] < 2:
            raise ValueError("PolyApply needs degree >= 1 (theta of length >= 2)")
        Xc = X.detach().contiguous()
        if Xc.dtype != torch.float32:
            raise TypeError("PolyApply takes a float32 block")
        p = sped.monomial(th, shift, scale)
        Y = sped.apply_poly(L, p, Xc)
        ctx.save_for_backward(theta, Xc)
        ctx.L, ctx.p, ctx.shift, ctx.scale = L, p, shift, scale
        return Y

    @staticmethod
    def backward(ctx, dY: torch.Tensor):
        theta, X = ctx.saved_tensors
        dY = dY.contiguous().to(torch.float32)
        dX = dtheta = None
        if ctx.needs_input_grad[1]:
            dX = sped.apply_poly(ctx.L, ctx.p, dY)
        if ctx.needs_input_grad[0]:
            dth = sped.poly_backward(ctx.L, ctx.p.degree, X, dY, ctx.shift, ctx.scale)
            dtheta = dth.to(device=theta.device, dtype=theta.dtype)
        return dtheta, dX, None, None, None


def poly_apply(theta, X, L, shift=0.0, scale=1.0):
    return PolyApply.apply(theta, X, L, shift, scale)
