"""Lazy node-walk estimator of the limit polynomial (I - L/l)^l V (oracle; test
infrastructure only).

Variance of the edge-chain estimators is left open by the paper (Sec. 6);
their weights grow with the product of H-degrees along a chain.  For the
limit approximation of Table 2 (last row) there is a walk with bounded
weights on the nodes of G:

* normalised L = I - D^{-1/2} A D^{-1/2}: I - L/l = D^{1/2} P D^{-1/2} with
  P = (1 - 1/l) I + (1/l) D^{-1} A, a lazy random walk (stay with probability
  1 - 1/l, else move to neighbour j with probability w_ij / d_i); hence
  ((I - L/l)^l V)_r = E[ s_Z V_Z ] / s_r over the walk's position Z after l
  steps from r, s = d^{-1/2};
* combinatorial L = D - A with l >= max_i d_i: I - L/l is itself stochastic
  (stay with probability 1 - d_i/l, move to j with probability w_ij / l), so
  ((I - L/l)^l V)_r = E[ V_Z ].
Isolated nodes never move (their row of L is zero).

Draws (both sides), key = seed, counter (r, w, c, step << 8 | j) for output row
r, walk w, application counter c:
* the walk stays at z with probability 1 - p_move(z) per step, p_move = 1/l
  (normalised, degree > 0) or d_z / l (combinatorial); the number of stays
  before its m-th move (m = 0, 1, ...) is drawn at once as the geometric
  variable G = floor(log(1 - u) / log1p(-p_move(z))), u = uniform53(step m),
  which has the law of one Bernoulli draw per step; the move happens at step
  t + G + 1 if that is at most l (t the steps taken so far), else the walk
  stops;
* a move proposes neighbour number bounded(step 256 + 1024 t + a, deg z) for
  attempt a = 0..15 and accepts it when its weight ratio x_j / max_row x is
  at least 1 - 2^-20 (weights this close count as equal: unweighted graphs
  never reach the test below) or when uniform53(step 2^20 + 1024 t + a) is
  below the ratio; x_j = w_ij (combinatorial) or S_ij / s_j (normalised,
  proportional to w_ij within a row), in the precision the device stores
  (float32 S and s, ratios in float64);
* after 16 rejections, neighbour j is the first whose running sum of x (row
  order) exceeds uniform53(step 2^21 + t) times the row sum: rejection with a
  cap followed by the exact inverse-CDF draw is still exact.
"""
from __future__ import annotations

import numpy as np

from . import rng
from .laplacian import COMBINATORIAL, SYM_NORMALIZED, Laplacian

_ATTEMPTS = 16
_EQUAL = 1.0 - 2.0 ** -20


def _device_weights(lap: Laplacian):
    """Row-major adjacency (neighbours ascending), per stored entry the move
    weight x in the device's precision, per row the largest x, and the
    float32 scale."""
    rowptr, col, w = lap.adjacency()
    n = lap.n
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    if lap.kind == SYM_NORMALIZED:
        s32 = lap.scale.astype(np.float32)
        val32 = (w * lap.scale[rows] * lap.scale[col]).astype(np.float32)
        x = val32.astype(np.float64) / s32[col].astype(np.float64)
    elif lap.kind == COMBINATORIAL:
        s32 = np.ones(n, dtype=np.float32)
        x = w.astype(np.float32).astype(np.float64)
    else:
        raise ValueError(lap.kind)
    xmax = np.zeros(n)
    nz = np.nonzero(np.diff(rowptr) > 0)[0]
    if nz.size:
        xmax[nz] = np.maximum.reduceat(x, rowptr[nz])
    return rowptr, col, x, xmax, s32


def estimate_lazy(lap: Laplacian, ell: int, V, walks_per_row: int, seed: int, counter: int = 0, rows=None):
    """Unbiased estimate of rows `rows` (default all) of (I - L/l)^l V from
    `walks_per_row` lazy walks per row.  Returns float64 (len(rows), k)."""
    V = np.asarray(V, dtype=np.float64)
    n = lap.n
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    rowptr, col, x, xmax, s32 = _device_weights(lap)
    deg = np.diff(rowptr)
    if lap.kind == SYM_NORMALIZED:
        p_move = np.where(deg > 0, 1.0 / ell, 0.0)
    else:
        d32 = lap.degree.astype(np.float32).astype(np.float64)
        if n and d32.max() > ell:
            raise ValueError("combinatorial lazy walk needs l >= the largest weighted degree")
        p_move = d32 / ell
    r = np.repeat(rows, walks_per_row)
    widx = np.tile(np.arange(walks_per_row), rows.shape[0])
    z = r.copy()
    steps = np.zeros(r.shape[0], dtype=np.int64)
    active = deg[z] > 0
    for m in range(ell):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        u = rng.uniform53(seed, r[idx], widx[idx], counter, m)
        with np.errstate(divide="ignore"):
            gap = np.floor(np.log(1.0 - u) / np.log1p(-p_move[z[idx]]))
        go = gap < (ell - steps[idx])
        active[idx[~go]] = False
        movers = idx[go]
        steps[movers] += gap[go].astype(np.int64) + 1
        t = steps[movers]
        chosen = np.full(movers.shape[0], -1, dtype=np.int64)
        for a in range(_ATTEMPTS):
            todo = np.nonzero(chosen < 0)[0]
            if todo.size == 0:
                break
            mv = movers[todo]
            tt = t[todo]
            cand = rng.bounded(seed, r[mv], widx[mv], counter, 256 + 1024 * tt + a, deg[z[mv]]).astype(np.int64)
            p = rowptr[z[mv]] + cand
            ratio = x[p] / xmax[z[mv]]
            acc = ratio >= _EQUAL
            test = np.nonzero(~acc)[0]
            if test.size:
                u2 = rng.uniform53(seed, r[mv[test]], widx[mv[test]], counter, (1 << 20) + 1024 * tt[test] + a)
                acc[test] = u2 < ratio[test]
            chosen[todo[acc]] = p[acc]
        left = np.nonzero(chosen < 0)[0]
        for i in left:  # inverse CDF over the row: running sum in row order
            mv = movers[i]
            zz = z[mv]
            a, b = rowptr[zz], rowptr[zz + 1]
            run = np.cumsum(x[a:b])
            target = rng.uniform53(seed, r[mv], widx[mv], counter, (1 << 21) + t[i]) * run[-1]
            hit = np.nonzero(run > target)[0]
            chosen[i] = a + (hit[0] if hit.size else b - a - 1)
        z[movers] = col[chosen]
        active[movers] = deg[z[movers]] > 0
    weight = s32[z].astype(np.float64) / np.where(s32[r] > 0, s32[r], 1.0).astype(np.float64)
    weight = np.where(s32[r] > 0, weight, 1.0)
    est = weight[:, None] * V[z]
    return est.reshape(rows.shape[0], walks_per_row, -1).mean(axis=1)


def walk_path(lap: Laplacian, ell: int, r: int, w: int, seed: int, counter: int = 0, flip: int | None = None):
    """One walk, step by step (the same draws as `estimate_lazy`), for
    checking single rows.  Returns (end node, decisions): every decision the
    walk took, in order, as (kind, margin), the margin being how far the
    compared quantities were from the other outcome, relative to their size:
      'gap'    |q - nearest integer| / max(1, |q|), q = log(1 - u) / log1p(-p_move)
               (the floor of q is the number of stays);
      'accept' |u - ratio| / ratio for a proposal tested against a uniform u
               (a ratio that the equality rule accepts is not a decision: the
               other rounding of it would be accepted by the test with
               probability 1 - 2^-20);
      'cdf'    distance of the target to the nearest running-sum boundary,
               relative to the row sum.
    flip = i takes decision i the other way (the floor of q on the other side
    of the nearest integer; the other accept outcome; the entry across the
    nearest boundary): what the walk does when the compared values round the
    other way."""
    rowptr, col, x, xmax, _ = _device_weights(lap)
    deg = np.diff(rowptr)
    norm = lap.kind == SYM_NORMALIZED
    d32 = lap.degree.astype(np.float32).astype(np.float64)
    decisions = []

    def flipped():
        return flip is not None and len(decisions) == flip

    def u53(step):
        return float(rng.uniform53(seed, r, w, counter, step)[()])

    z, t, m = int(r), 0, 0
    while deg[z] > 0:
        pm = 1.0 / ell if norm else d32[z] / ell
        with np.errstate(divide="ignore"):
            q = float(np.log(1.0 - u53(m)) / np.log1p(-pm))
        near = float(np.rint(q))
        g = np.floor(q)
        if flipped():
            g = near - 1.0 if q >= near else near
        decisions.append(("gap", abs(q - near) / max(1.0, abs(q)) if np.isfinite(q) else np.inf))
        m += 1
        if not g < ell - t:
            break
        t += int(g) + 1
        a0 = int(rowptr[z])
        chosen = -1
        for a in range(_ATTEMPTS):
            cand = int(rng.bounded(seed, r, w, counter, 256 + 1024 * t + a, int(deg[z]))[0])
            ratio = x[a0 + cand] / xmax[z]
            if ratio >= _EQUAL:
                ok = True
            else:
                u2 = u53((1 << 20) + 1024 * t + a)
                ok = u2 < ratio
                if flipped():
                    ok = not ok
                decisions.append(("accept", abs(u2 - ratio) / ratio))
            if ok:
                chosen = a0 + cand
                break
        if chosen < 0:
            run = np.cumsum(x[a0:a0 + deg[z]])
            target = u53((1 << 21) + t) * run[-1]
            hit = np.nonzero(run > target)[0]
            i = int(hit[0]) if hit.size else int(deg[z]) - 1
            lo = run[i - 1] if i > 0 else -np.inf
            above = abs(run[i] - target) <= abs(target - lo)
            if flipped():
                i = min(i + 1, int(deg[z]) - 1) if above else max(i - 1, 0)
            decisions.append(("cdf", min(abs(run[i] - target), abs(target - lo)) / run[-1]))
            chosen = a0 + i
        z = int(col[chosen])
    return z, decisions


def row_from_ends(lap: Laplacian, r: int, ends, V):
    """Row r of the estimate from its walks' end nodes (weights s_Z / s_r in
    the stored float32 scales; 1 for the combinatorial Laplacian)."""
    _, _, _, _, s32 = _device_weights(lap)
    V = np.asarray(V, dtype=np.float64)
    ends = np.asarray(ends, dtype=np.int64)
    wgt = s32[ends].astype(np.float64) / float(s32[r]) if s32[r] > 0 else np.ones(len(ends))
    return (wgt[:, None] * V[ends]).mean(axis=0)


def lazy_walk_matrix(lap: Laplacian, ell: int):
    """The dense lazy-walk transition matrix P of the module header (for
    checking the similarity to I - L/l)."""
    n = lap.n
    A = np.zeros((n, n))
    np.add.at(A, (lap.eu, lap.ev), lap.ew)
    np.add.at(A, (lap.ev, lap.eu), lap.ew)
    d = lap.degree
    P = np.zeros((n, n))
    for i in range(n):
        if d[i] == 0:
            P[i, i] = 1.0
        elif lap.kind == SYM_NORMALIZED:
            P[i] = A[i] / d[i] / ell
            P[i, i] += 1.0 - 1.0 / ell
        else:
            P[i] = A[i] / ell
            P[i, i] += 1.0 - d[i] / ell
    return P
