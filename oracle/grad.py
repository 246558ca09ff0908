"""Gradient of Y = p_theta(L) X (oracle; test infrastructure only).

Sec. 6 names meta-learning the polynomial coefficients as future work.  With
Y = sum_j theta_j L^j X and an upstream gradient dY:
  d theta_j = <dY, L^j X>_F          (Y is linear in theta),
  dX        = sum_j theta_j L^j dY   (L is symmetric, so p(L)^T = p(L)).
"""
from __future__ import annotations

import numpy as np


def forward(L, theta, X):
    X = np.asarray(X, dtype=np.float64)
    P = X.copy()
    Y = theta[0] * P
    for j in range(1, len(theta)):
        P = L @ P
        Y = Y + theta[j] * P
    return Y


def backward(L, theta, X, dY):
    X = np.asarray(X, dtype=np.float64)
    dY = np.asarray(dY, dtype=np.float64)
    dtheta = np.zeros(len(theta))
    P = X.copy()
    dtheta[0] = float(np.sum(dY * P))
    for j in range(1, len(theta)):
        P = L @ P
        dtheta[j] = float(np.sum(dY * P))
    dX = forward(L, theta, dY)
    return dtheta, dX
