"""Bottom-k solver and convergence metrics (oracle; test infrastructure only).

Sec. 3: the bottom-k eigenvectors of L are the top-k of the reversed operator M
(eq. reveig); Sec. 5 runs iterative top-k solvers (Oja's algorithm, mu-EG) on
the transformed matrix.  The oracle solver is block subspace iteration, the
step-size-to-infinity limit of block Oja, V <- qr(M V), or the Oja step
V <- qr(V + eta M V), with Householder QR (LAPACK geqrf through numpy) and a
Rayleigh-Ritz projection on L itself to read off eigenvalues and residuals.

Sec. 5.2 metrics: subspace error delta = 1 - tr(U* P)/k with U*, P the
orthogonal projectors of the true and estimated subspaces, which equals the
mean squared sine of the principal angles; and the eigenvector streak, the
number of leading estimated vectors each within an angle eps of its true one.
mu-EigenGame (the other solver Sec. 5 cites) recovers the eigenvectors one by
one in order, which is what the streak measures.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def orthonormal(V):
    Q, _ = np.linalg.qr(np.asarray(V, dtype=np.float64))
    return Q


def subspace_error(Vstar, Q) -> float:
    """delta = 1 - tr(U* P)/k = 1 - ||V*^T Q||_F^2 / k for orthonormal bases."""
    Vstar, Q = orthonormal(Vstar), orthonormal(Q)
    k = Vstar.shape[1]
    return float(1.0 - np.linalg.norm(Vstar.T @ Q) ** 2 / k)


def max_principal_angle(Vstar, Q) -> float:
    """Largest principal angle, from its sine: sigma_max((I - V* V*^T) Q)."""
    Vstar, Q = orthonormal(Vstar), orthonormal(Q)
    R = Q - Vstar @ (Vstar.T @ Q)
    s = np.linalg.norm(R, 2) if R.size else 0.0
    return float(np.arcsin(min(1.0, s)))


def vector_angles(Vstar, Q):
    """Angle between each estimated vector and its true one (sign-free)."""
    Vstar = Vstar / np.linalg.norm(Vstar, axis=0)
    Q = Q / np.linalg.norm(Q, axis=0)
    c = np.abs(np.sum(Vstar * Q, axis=0)).clip(0, 1)
    s = np.linalg.norm(Q - Vstar * np.sign(np.sum(Vstar * Q, axis=0)), axis=0)
    # sine from the difference vector keeps small angles accurate
    return np.where(c > 0.5, 2.0 * np.arcsin(np.minimum(1.0, s / 2.0)), np.arccos(c))


def eigenvector_streak(Vstar, Q, eps: float = np.pi / 8) -> int:
    ang = vector_angles(Vstar, Q)
    streak = 0
    for a in ang:
        if a > eps:
            break
        streak += 1
    return streak


def rayleigh_ritz(L, Q, return_block: bool = False):
    """Ritz pairs of L on span(Q): H = Q^T L Q = S Theta S^T (ascending).

    Returns (theta, Q S, residual norms), plus the residual block
    R = L Q S - Q S Theta when return_block is set."""
    Z = L @ Q
    H = Q.T @ Z
    H = 0.5 * (H + H.T)
    theta, S = np.linalg.eigh(H)
    Q = Q @ S
    Z = Z @ S
    R = Z - Q * theta
    if return_block:
        return theta, Q, np.linalg.norm(R, axis=0), R
    return theta, Q, np.linalg.norm(R, axis=0)


def residual_norm_bound(R) -> float:
    """rho = sqrt(min(||R^T R||_inf, ||R||_F^2)), an upper bound on ||R||_2:
    the largest eigenvalue of the Gram matrix G = R^T R is at most any induced
    norm of G (the infinity norm here) and at most its trace."""
    G = R.T @ R
    return float(np.sqrt(min(np.abs(G).sum(axis=1).max(), np.trace(G))))


@dataclass
class SolveResult:
    evals: np.ndarray
    Q: np.ndarray
    iters: int
    residuals: np.ndarray
    history: list = field(default_factory=list)
    converged: bool = False


def subspace_iteration(L, apply_M, k: int, V0, max_iters: int, tol: float = 0.0,
                       eta: float = np.inf, check_every: int = 1, Vstar=None,
                       guard: int = 0):
    """Block subspace iteration (eta = inf) or block Oja (finite eta) on M.

    Iterates with k + guard columns; stops when residual_norm_bound of the
    first k Ritz residual columns (an upper bound on their spectral norm)
    divided by the gap estimate theta_{k+1} - ||r_{k+1}|| - theta_k
    (guard > 0) or by 1 (guard = 0) is <= tol (Davis-Kahan).  With Vstar
    given, records the largest principal angle and the subspace error after
    each check."""
    Q = orthonormal(V0)
    hist = []
    theta = res = None
    for t in range(1, max_iters + 1):
        W = apply_M(Q)
        if np.isfinite(eta):
            W = Q + eta * W
        Q = orthonormal(W)
        if t % check_every == 0 or t == max_iters:
            theta, Q, res, R = rayleigh_ritz(L, Q, return_block=True)
            gap = (theta[k] - res[k] - theta[k - 1]) if guard > 0 else 1.0
            bound = residual_norm_bound(R[:, :k]) / max(gap, 1e-300)
            rec = {"iter": t, "bound": bound, "max_residual": float(np.max(res[:k]))}
            if Vstar is not None:
                rec["angle"] = max_principal_angle(Vstar, Q[:, :k])
                rec["delta"] = subspace_error(Vstar, Q[:, :k])
            hist.append(rec)
            if tol > 0 and bound <= tol:
                return SolveResult(theta[:k], Q[:, :k], t, res[:k], hist, True)
    if theta is None:
        theta, Q, res = rayleigh_ritz(L, Q)
    return SolveResult(theta[:k], Q[:, :k], max_iters, res[:k], hist, False)


def mu_eigengame(apply_M, V0, eta: float, iters: int, Vstar=None, eps: float = np.pi / 8,
                 record_every: int = 1):
    """mu-EigenGame on the top-k eigenvectors of M (the solver family Sec. 5
    runs on the transformed matrix).  Player i holds a unit vector v_i and
    moves along the Riemannian projection of its utility gradient
        grad_i = M v_i - sum_{j<i} <v_i, M v_j> v_j,
        grad_i <- grad_i - <grad_i, v_i> v_i,
        v_i <- (v_i + eta grad_i) / ||v_i + eta grad_i||,
    all players at once.  Only players j < i penalise player i, so player 1
    runs Oja's rule for the top eigenvector and player i the same on the
    deflation by the players above it: the fixed point is the ordered top-k
    eigenbasis.  With Vstar given, records the eigenvector streak (Sec. 5.2)
    every `record_every` iterations.  Returns (V, history)."""
    V = np.asarray(V0, dtype=np.float64)
    V = V / np.linalg.norm(V, axis=0)
    hist = []
    for t in range(1, iters + 1):
        W = apply_M(V)
        G = V.T @ W                       # G[j, i] = <v_j, M v_i> = <v_i, M v_j>
        grad = W - V @ np.triu(G, 1)      # column i subtracts sum_{j<i} G[j, i] v_j
        grad = grad - V * np.sum(grad * V, axis=0)
        V = V + eta * grad
        V = V / np.linalg.norm(V, axis=0)
        if Vstar is not None and t % record_every == 0:
            hist.append({"iter": t, "streak": eigenvector_streak(Vstar, V, eps),
                         "angles": vector_angles(Vstar, V)})
    return V, hist


def dense_bottom_k(L_dense, k: int):
    """Ground truth by full symmetric eigendecomposition (LAPACK syevd)."""
    lam, U = np.linalg.eigh(L_dense)
    return lam[:k], U[:, :k], lam
