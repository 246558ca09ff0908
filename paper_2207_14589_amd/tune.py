"""Tuning the dilation coefficients theta by gradient descent (the
meta-learning direction named in Sec. 6), on top of PolyApply.

The operator is M_theta = sum_i theta_i Lt^i with Lt = (L - shift I)/scale
(shift 1 maps the normalised spectrum [0, 2] to [-1, 1], where monomials are
well conditioned).  The loss unrolls `unroll` steps of block subspace
iteration from a fixed start block, Q_t = qr(M_theta Q_{t-1}), and returns the
mean Rayleigh quotient tr(Q^T L Q)/k of the first k columns, which the
bottom-k subspace minimises.  The loss is invariant to the scale of theta, so
theta is normalised inside it.  All sparse work runs in the HIP library
(PolyApply forward, X gradient and recomputed-power coefficient gradient);
torch supplies the QR and the optimiser.
"""
from __future__ import annotations

import numpy as np
import torch

from . import sped
from .autograd import poly_apply


def limit_in_shifted(ell: int, shift: float = 1.0, scale: float = 1.0) -> np.ndarray:
    """Coefficients of (I - L/ell)^ell in the variable Lt = (L - shift I)/scale
    (computed by the library)."""
    return sped.transform("limit", ell).rebase(shift, scale)


def rayleigh_loss(theta, L, V0, k, unroll, shift, scale):
    th = theta / theta.norm()
    Q, _ = torch.linalg.qr(V0)
    for _ in range(unroll):
        W = poly_apply(th, Q, L, shift, scale)
        Q, _ = torch.linalg.qr(W)
    Qk = Q[:, :k]
    LQ = poly_apply(torch.tensor([shift, scale], dtype=torch.float64), Qk, L, shift, scale)
    return (Qk * LQ).sum() / k


def tune_coefficients(L: "sped.Laplacian", k: int, degree: int, V0: torch.Tensor, steps: int = 60,
                      unroll: int = 3, lr: float = 0.02, shift: float = 1.0, scale: float = 1.0,
                      theta0=None):
    """Adam on theta; returns (theta as numpy float64, loss history)."""
    th0 = limit_in_shifted(degree, shift, scale) if theta0 is None else np.asarray(theta0, dtype=np.float64)
    theta = torch.tensor(th0 / np.linalg.norm(th0), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([theta], lr=lr)
    hist = []
    best, best_th = np.inf, theta.detach().clone()
    for _ in range(steps):
        opt.zero_grad()
        loss = rayleigh_loss(theta, L, V0, k, unroll, shift, scale)
        loss.backward()
        val = float(loss.detach())
        hist.append(val)
        if val < best:
            best, best_th = val, theta.detach().clone()
        opt.step()
    th = best_th / best_th.norm()
    return th.numpy(), hist
