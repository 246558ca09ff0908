"""Spectral transforms, reversal and exact p(L)V (oracle; test infrastructure only).

Sec. 4.1: a monotonically increasing polynomial f keeps the eigenvectors of L
and their order; the transformed spectrum is then reversed with eq. (reveig),
M = lambda* I - f(L), lambda* > f(lambda_max), so the bottom-k eigenvectors of
L are the top-k of M.  Sec. 4.2 / Table 2 list the transforms; for -exp(-L)
the reversal constant is lambda* = 0 and the spectral radius is 1.

A polynomial is held as coefficients c_0..c_l in the variable
Lt = (L - shift I) / scale:  M = sum_i c_i Lt^i.

Readings where the paper is silent:
* the plain-L baseline ("identity transformation") is M = lambda_bound I - L;
* Taylor log: eps = 1e-3 and lambda* = f(lambda_bound);
* the limit approximation -(I - L/l)^l is reversed with lambda* = 0, giving
  M = (I - L/l)^l.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction
from math import comb, factorial

import numpy as np


@dataclass
class Poly:
    coeffs: np.ndarray   # c_0 .. c_l
    shift: float = 0.0
    scale: float = 1.0
    name: str = ""

    @property
    def degree(self) -> int:
        return len(self.coeffs) - 1

    def __call__(self, lam):
        """Evaluate sum_i c_i ((lam - shift)/scale)^i term by term."""
        y = (np.asarray(lam, dtype=np.float64) - self.shift) / self.scale
        out = np.zeros_like(y)
        for i, c in enumerate(self.coeffs):
            out = out + c * y ** i
        return out


def plain(lambda_bound: float) -> Poly:
    """Identity transform reversed by eq. (reveig): M = lambda_bound I - L."""
    return Poly(np.array([lambda_bound, -1.0]), name="plain")


def limit_exp(ell: int) -> Poly:
    """Table 2 row 5: f(L) = -(I - L/l)^l; lambda* = 0 gives M = (I - L/l)^l.
    Binomial expansion: c_i = C(l, i) (-1/l)^i."""
    c = np.array([comb(ell, i) * (-1.0 / ell) ** i for i in range(ell + 1)])
    return Poly(c, name=f"limit{ell}")


def taylor_exp(ell: int) -> Poly:
    """Table 2 row 4: f(L) = -sum_{i<=l} (-L)^i / i!;  M = -f(L).  1/i! is
    rounded once from the exact rational (it falls below the double range for
    large i, e.g. the degree 251 of the experiments, and then rounds to 0)."""
    c = np.array([(-1.0) ** i * float(Fraction(1, factorial(i))) for i in range(ell + 1)])
    return Poly(c, name=f"texp{ell}")


def taylor_log(ell: int, lambda_bound: float, eps: float = 1e-3) -> Poly:
    """Table 2 row 2: f(L) = sum_{i=1..l} (-1)^{i+1} (L + eps I - I)^i / i, a
    polynomial in y = L - (1 - eps) I.  M = f(lambda_bound) I - f(L)."""
    y_top = lambda_bound - (1.0 - eps)
    f_top = sum((-1.0) ** (i + 1) * y_top ** i / i for i in range(1, ell + 1))
    c = np.zeros(ell + 1)
    c[0] = f_top
    for i in range(1, ell + 1):
        c[i] = -((-1.0) ** (i + 1)) / i
    return Poly(c, shift=1.0 - eps, scale=1.0, name=f"tlog{ell}")


def monomial_in_L(p: Poly) -> np.ndarray:
    """Coefficients of the same polynomial in L itself (expand the shift)."""
    out = np.zeros(p.degree + 1)
    for i, c in enumerate(p.coeffs):
        # ((L - a)/s)^i = s^-i sum_j C(i,j) L^j (-a)^(i-j)
        for j in range(i + 1):
            out[j] += c * comb(i, j) * (-p.shift) ** (i - j) / p.scale ** i
    return out


def apply_terms(L, p: Poly, V: np.ndarray) -> np.ndarray:
    """p(L) V = sum_i c_i Lt^i V by explicit powers P_i = Lt P_{i-1}."""
    V = np.asarray(V, dtype=np.float64)
    P = V.copy()
    Y = p.coeffs[0] * V
    for i in range(1, p.degree + 1):
        P = (L @ P - p.shift * P) / p.scale
        Y = Y + p.coeffs[i] * P
    return Y


def apply_limit_product(L, ell: int, V: np.ndarray) -> np.ndarray:
    """(I - L/l)^l V as l successive factor applications."""
    Y = np.asarray(V, dtype=np.float64).copy()
    for _ in range(ell):
        Y = Y - (L @ Y) / ell
    return Y


def apply_spectral(L_dense: np.ndarray, f, V: np.ndarray) -> np.ndarray:
    """f(L) V through the full eigendecomposition (Sec. 4.1, e^L = V e^Lambda V^T);
    for the exact rows of Table 2 on tiny graphs only."""
    lam, U = np.linalg.eigh(L_dense)
    return U @ (f(lam)[:, None] * (U.T @ V))


def exact_log(eps: float = 1e-3):
    """Table 2 row 1: log(L + eps)."""
    return lambda lam: np.log(np.maximum(lam, 0.0) + eps)


def exact_negexp():
    """Table 2 row 3: -exp(-L)."""
    return lambda lam: -np.exp(-lam)
