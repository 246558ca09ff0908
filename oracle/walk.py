"""Edge-chain (random walk) estimator of p(L)V (oracle; test infrastructure only).

Sec. 4.3, eq. (walk_summand): L^l = sum over chains c = (e_1..e_l) in E^l of
alpha_c x_{e_1} x_{e_l}^T with alpha_c = prod_j x_{e_j}^T x_{e_{j+1}}; alpha_c is
non-zero only when consecutive edges are incident, so the chains are walks on
the edge-incidence graph H (nodes = edges of G, adjacent when incident, with a
self-loop on every node).  Table 1 gives the inner products for unweighted
combinatorial graphs: 0 disconnected, -1 serial, +1 converging, +1 diverging,
2 repeated.  For the weighted / normalised rows x~_e = sqrt(w_e)(s_i e_i - s_j e_j)
(i = min) the same products are h(e,u) h(f,u) at the shared node u, with
h(e,u) = sign_e(u) sqrt(w_e) s_u, sign +1 at min(e), and
x~_e^T x~_e = h(e,i)^2 + h(e,j)^2.  With w = s = 1 these reduce to Table 1.

Linearity (Sec. 4.3, last paragraphs): one length-l walk yields an estimate for
every prefix i <= l, so sum_i c_i L^i V is estimated from the same walks.

Two samplers:

``importance`` (row-owned).  For output row r, walk w: e_1 is uniform over the
d_r edges at r; each next edge is uniform over the deg_H(e) = d_a + d_b - 1
neighbours of e = (a, b) in H (the d_a edges at a, which include e itself,
then the edges at b other than e).  The proposal probability of a chain is
q(c) = (1/d_r) prod_t 1/deg_H(e_t), so the weight
omega_i = alpha_c (x~_{e_1})_r / q(c) makes omega_i x~_{e_i}^T V unbiased for
row r of L^i V.  This is the expectation of the rejection sampler's accepted
estimate given the chain (it replaces the accept indicator by its mean).

``reject`` (the literal sampler of Sec. 4.3).  e_1 uniform over E; the walk
moves as above; prefix i is accepted with probability
a_i = prod_{t<i} deg_H(e_t) / deg*_inc, deg*_inc = 2 deg* - 1, deg* the maximum
node degree, so an accepted length-i chain has probability
p_min,i = deg*_inc^{-(i-1)} / |E| for every chain; the estimate of L^i V is
(1/(N p_min,i)) sum_{accepted} alpha_c x~_{e_1} (x~_{e_i}^T V) over N trials.

Readings of the garbled text (also in the design notes): the walker state is a
node of H; a length-i walk has i edges and i-1 transitions, so p and p_min
carry i-1 factors; the paper's "rejected with probability p_min/p" is read as
accepted with that probability; N is fixed instead of the data-dependent stop,
and prefixes with no acceptance are reported.

Random numbers: Philox streams of oracle.rng.
  importance: c0 = row, c1 = walk, c2 = counter, step 0 draws e_1, step t
              draws e_{t+1}.
  reject:     c0 = trial mod 2^32, c1 = (trial >> 32) | 2^31, c2 = counter;
              step 0 draws e_1 among the 2|E| directed CSR entries, step t
              draws e_{t+1}; the accept uniform of prefix i uses step l + i.
"""
from __future__ import annotations

import numpy as np

from . import rng
from .laplacian import Laplacian


class _Walker:
    """Neighbour lists of G sorted by neighbour id, plus per-entry data."""

    def __init__(self, lap: Laplacian):
        self.lap = lap
        self.rowptr, self.col, self.w = lap.adjacency()
        self.n = lap.n
        self.row_of = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        self.deg = np.diff(self.rowptr)
        # position of the reverse entry (b -> a) of each entry (a -> b)
        key_fwd = self.row_of * np.int64(self.n) + self.col
        key_rev = self.col * np.int64(self.n) + self.row_of
        # the graph is symmetric, so both key arrays hold the same set: the
        # j-th smallest reverse key belongs to the entry whose forward key is
        # the j-th smallest
        order = np.argsort(key_fwd, kind="stable")
        self.rev = np.empty_like(order)
        self.rev[np.argsort(key_rev, kind="stable")] = order
        assert np.array_equal(key_fwd[self.rev], key_rev)
        self.s = lap.scale

    def h(self, pos, u):
        """Entry of x~_e at node u for the edge stored at CSR position pos."""
        a = self.row_of[pos]
        b = self.col[pos]
        other = np.where(u == a, b, a)
        sign = np.where(u < other, 1.0, -1.0)
        return sign * np.sqrt(self.w[pos]) * self.s[u]

    def edge_dot_V(self, pos, V):
        a = self.row_of[pos]
        b = self.col[pos]
        return self.h(pos, a)[:, None] * V[a] + self.h(pos, b)[:, None] * V[b]

    def step(self, pos, draw):
        """Move from the edge at `pos` to its H-neighbour number `draw`.
        Returns (new position, inner product x~_e^T x~_f, deg_H(e))."""
        a = self.row_of[pos]
        b = self.col[pos]
        da, db = self.deg[a], self.deg[b]
        from_a = draw < da
        q_a = self.rowptr[a] + draw
        jb = draw - da
        q_b = self.rowptr[b] + jb
        q_b = np.where(q_b >= self.rev[pos], q_b + 1, q_b)
        q = np.where(from_a, q_a, q_b)
        u = np.where(from_a, a, b)
        same = q == pos
        ha, hb = self.h(pos, a), self.h(pos, b)
        dot_same = ha * ha + hb * hb
        dot_inc = self.h(pos, u) * self.h(q, u)
        dot = np.where(same, dot_same, dot_inc)
        return q, dot, da + db - 1


def estimate_importance(lap: Laplacian, coeffs, V, walks_per_row: int, seed: int,
                        counter: int = 0, rows=None):
    """Importance-weighted walk estimate of sum_i c_i L^i V for `rows`
    (default all), averaging `walks_per_row` walks per row.  coeffs are the
    monomial coefficients in L.  Returns float64 (len(rows), k)."""
    W = _Walker(lap)
    V = np.asarray(V, dtype=np.float64)
    c = np.asarray(coeffs, dtype=np.float64)
    ell = c.shape[0] - 1
    rows = np.arange(W.n) if rows is None else np.asarray(rows, dtype=np.int64)
    Y = c[0] * V[rows]
    r = np.repeat(rows, walks_per_row)
    widx = np.tile(np.arange(walks_per_row), rows.shape[0])
    dr = W.deg[r]
    live = dr > 0
    r, widx, dr = r[live], widx[live], dr[live]
    acc = np.zeros((r.shape[0], V.shape[1]))
    if r.size and ell >= 1:
        t0 = rng.bounded(seed, r, widx, counter, 0, dr)
        pos = W.rowptr[r] + t0
        omega = dr.astype(np.float64) * W.h(pos, r)
        for i in range(1, ell + 1):
            if i > 1:
                a = W.row_of[pos]
                bnd = W.deg[a] + W.deg[W.col[pos]] - 1
                t = rng.bounded(seed, r, widx, counter, i - 1, bnd)
                pos, dot, degH = W.step(pos, t)
                omega = omega * dot * degH
            acc += (c[i] * omega)[:, None] * W.edge_dot_V(pos, V)
    out = np.zeros((rows.shape[0] * walks_per_row, V.shape[1]))
    out[np.nonzero(live)[0]] = acc
    Y += out.reshape(rows.shape[0], walks_per_row, -1).sum(axis=1) / walks_per_row
    return Y


def estimate_reject(lap: Laplacian, coeffs, V, n_trials: int, seed: int,
                    counter: int = 0, trial_offset: int = 0):
    """Rejection-sampled walk estimate of sum_i c_i L^i V over `n_trials`
    trials.  Returns (Y float64 (n, k), accept_counts int64 (l,))."""
    W = _Walker(lap)
    V = np.asarray(V, dtype=np.float64)
    c = np.asarray(coeffs, dtype=np.float64)
    ell = c.shape[0] - 1
    n_edges = W.col.shape[0] // 2
    dstar = int(W.deg.max()) if W.n else 0
    d_inc = 2 * dstar - 1
    Y = c[0] * V.copy()
    counts = np.zeros(max(ell, 0), dtype=np.int64)
    if n_edges == 0 or ell < 1:
        return Y, counts
    T = np.arange(n_trials, dtype=np.int64) + trial_offset
    c0 = T & 0xFFFFFFFF
    c1 = (T >> 32) | (1 << 31)
    pos = rng.bounded(seed, c0, c1, counter, 0, 2 * n_edges)
    a1 = W.row_of[pos]
    b1 = W.col[pos]
    h1a, h1b = W.h(pos, a1), W.h(pos, b1)
    rho = np.ones(n_trials)            # prod_t deg*_inc * x_et^T x_et+1
    accept_p = np.ones(n_trials)       # prod_t deg_H(e_t) / deg*_inc
    scale = n_edges / float(n_trials)
    for i in range(1, ell + 1):
        if i > 1:
            a = W.row_of[pos]
            bnd = W.deg[a] + W.deg[W.col[pos]] - 1
            t = rng.bounded(seed, c0, c1, counter, i - 1, bnd)
            pos, dot, degH = W.step(pos, t)
            rho = rho * (dot * d_inc)
            accept_p = (accept_p * degH.astype(np.float64)) / float(d_inc)
            u = rng.uniform53(seed, c0, c1, counter, ell + i)
            ok = u < accept_p
        else:
            ok = np.ones(n_trials, dtype=bool)
        counts[i - 1] = int(ok.sum())
        if not ok.any():
            continue
        val = (c[i] * scale * rho[ok])[:, None] * W.edge_dot_V(pos[ok], V)
        np.add.at(Y, a1[ok], h1a[ok][:, None] * val)
        np.add.at(Y, b1[ok], h1b[ok][:, None] * val)
    return Y, counts


def estimate_hybrid(lap: Laplacian, coeffs, V, exact_terms: int, walks_per_row: int, seed: int,
                    counter: int = 0, sampler: str = "importance", n_trials: int = 0):
    """Exact low-order terms plus a sampled tail (the variance-reduction
    direction Sec. 6 leaves open): with m = exact_terms,
        Y = sum_{i<m} c_i L^i V + L^m T,   T = walk estimate of sum_j c_{m+j} L^j V,
    unbiased because L^m commutes with the tail polynomial.  T uses the
    shifted coefficients (c_m, ..., c_l) and the given sampler and seed; the
    exact part is Horner's rule U <- L U + c_i V for i = m-1 .. 0 from U = T.
    m = 0 is the plain estimate, m = l the exact polynomial (T = c_l V).
    The rejection sampler takes n_trials trials.  Returns float64 (n, k)."""
    c = np.asarray(coeffs, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    m = int(exact_terms)
    if not 0 <= m <= c.shape[0] - 1:
        raise ValueError("exact_terms outside [0, degree]")
    tail = c[m:]
    if sampler == "importance":
        U = estimate_importance(lap, tail, V, walks_per_row, seed, counter)
    else:
        U, _ = estimate_reject(lap, tail, V, n_trials, seed, counter)
    for i in range(m - 1, -1, -1):
        U = lap.L @ U + c[i] * V
    return U


def edge_pair_product(lap: Laplacian, e, f):
    """x~_e^T x~_f for merged edges e, f (indices into lap.eu/ev), computed from
    the two incidence rows; the reference point for Table 1."""
    n = lap.n
    xe = np.zeros(n)
    xf = np.zeros(n)
    for x, idx in ((xe, e), (xf, f)):
        i, j, w = lap.eu[idx], lap.ev[idx], lap.ew[idx]
        x[i] += np.sqrt(w) * lap.scale[i]
        x[j] -= np.sqrt(w) * lap.scale[j]
    return float(xe @ xf)
