"""Edge-minibatch products with the Laplacian (oracle; test infrastructure only).

The Laplacian is a sum of rank-one terms, one per edge vector (Sec. 2:
L = X^T X = sum_e x_e x_e^T, weighted X^T W X; Sec. 4.1 normalised form with
x_e scaled by s_i = d_i^{-1/2} at each endpoint).  When the edge list does not
fit in memory, a solver sees batches of edge vectors (the eigengap discussion
of Sec. 3 and the conclusion): a batch B gives sum_{e in B} x_e x_e^T V, and
a uniformly drawn batch of b of the m edges, scaled by m / b, has expectation
L V.

Per edge e = (i, j) with weight w (i != j; a self-loop has x_e = 0):
    x_e = sqrt(w) (s_i e_i - s_j e_j),
    x_e x_e^T V adds  w s_i (s_i V_i - s_j V_j)  to row i
               and   -w s_j (s_i V_i - s_j V_j)  to row j.
The sign of x_e (which endpoint gets +1) does not change x_e x_e^T.
"""
from __future__ import annotations

import numpy as np

from . import rng

COMBINATORIAL = "combinatorial"
SYM_NORMALIZED = "sym"


def node_scales(n, src, dst, w=None, kind=SYM_NORMALIZED):
    """(degree, scale): d_i = sum of the weights of the non-loop edges at i
    (repeats add), s_i = d_i^{-1/2} (0 when d_i = 0) for the normalised
    Laplacian, 1 for the combinatorial one."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    wt = np.ones(len(src)) if w is None else np.asarray(w, dtype=np.float64)
    keep = src != dst
    d = np.zeros(n)
    np.add.at(d, src[keep], wt[keep])
    np.add.at(d, dst[keep], wt[keep])
    if kind == COMBINATORIAL:
        return d, np.ones(n)
    s = np.zeros(n)
    pos = d > 0
    s[pos] = 1.0 / np.sqrt(d[pos])
    return d, s


def edge_batch_apply(n, src, dst, w, scale, V):
    """sum over the batch's edges of x_e x_e^T V (float64), rows as above."""
    V = np.asarray(V, dtype=np.float64)
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    wt = np.ones(len(src)) if w is None else np.asarray(w, dtype=np.float64)
    s = np.asarray(scale, dtype=np.float64)
    keep = src != dst
    i, j, wt = src[keep], dst[keep], wt[keep]
    diff = s[i, None] * V[i] - s[j, None] * V[j]
    Y = np.zeros((n, V.shape[1]))
    np.add.at(Y, i, (wt * s[i])[:, None] * diff)
    np.add.at(Y, j, -(wt * s[j])[:, None] * diff)
    return Y


def _orth(V):
    """Orthonormal basis of span(V) by Householder QR, signs fixed so that R
    has a positive diagonal (the factor a Cholesky QR would give)."""
    Q, R = np.linalg.qr(V)
    return Q * np.where(np.diag(R) < 0, -1.0, 1.0)


def batch_offsets(seed, m, first, count):
    """Start offsets o_J in [0, m) of batches J = first .. first + count - 1:
    Lemire's bounded draw from Philox4x32-10 keyed by seed, counter
    (J mod 2^32, J >> 32, 0, 0)."""
    J = np.arange(first, first + count, dtype=np.uint64)
    return rng.bounded(seed, J & np.uint64(0xFFFFFFFF), J >> np.uint64(32), 0, 0, m)


def drawn_batch(m, offset, batch):
    """Indices of the batch that starts at `offset`: (offset + r) mod m, r < batch."""
    return (int(offset) + np.arange(batch)) % m


def minibatch_oja(n, src, dst, w, scale, degree, lambda_bound, V0, batch, eta, iters, seed=0, batch0=0):
    """Oja steps V <- orth(V + eta M_hat V) (Sec. 5's update) with M_hat from
    edge batches, each scaled by m / batch (Sec. 3: edge vectors fed in
    minibatches).  Batch J (J = batch0, batch0 + 1, ... in order) is the run
    of `batch` edges from a uniform random offset (batch_offsets), so every
    edge is in it with probability batch / m and different batches are
    independent.  degree 0: M_hat V = lambda_bound V - L_B V; degree l:
    (I - L_{B_l} / l) ... (I - L_{B_1} / l) V with its own batch per factor,
    whose independence makes E[M_hat] = (I - L/l)^l."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    wt = None if w is None else np.asarray(w, dtype=np.float64)
    m = len(src)
    V = np.asarray(V0, dtype=np.float64).copy()
    F = 1 if degree == 0 else degree
    offs = batch_offsets(seed, m, batch0, iters * F)
    j = 0
    for _ in range(iters):
        W = V
        for _f in range(F):
            idx = drawn_batch(m, offs[j], batch)
            j += 1
            LB = edge_batch_apply(n, src[idx], dst[idx], None if wt is None else wt[idx], scale,
                                  V if degree == 0 else W) * (m / batch)
            W = lambda_bound * V - LB if degree == 0 else W - LB / degree
        V = _orth(V + eta * W)
    return V
