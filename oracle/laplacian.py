"""Graph Laplacian from the incidence matrix (oracle; test infrastructure only).

Sec. 2: L = D - A = X^T X, where row x_e of the incidence matrix holds +1 at
min(i, j) and -1 at max(i, j) for edge e = (i, j); L 1 = 0.  With edge weights
the Laplacian is X^T W X (end of Sec. 2).  Sec. 4.1 names the normalised
Laplacian; its symmetric form is D^{-1/2} L D^{-1/2}, i.e. X is used with each
column i scaled by s_i = d_i^{-1/2}.

Readings where the paper is silent (listed in the design notes as well):
* self-loops contribute x_e = 0 and are dropped;
* repeated edges are separate rows of X, so their weights add;
* an isolated node under normalisation gets s_i = 0 (its row and column of L
  vanish, eigenvalue 0);
* `lcc=True` keeps only the largest connected component (ties: the component
  holding the smallest node id) and relabels its nodes in increasing old id.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

COMBINATORIAL = "combinatorial"
SYM_NORMALIZED = "sym"


@dataclass
class Laplacian:
    n: int
    kind: str
    L: sp.csr_matrix          # full Laplacian, float64, diagonal included
    eu: np.ndarray            # merged undirected edges, eu < ev (int64)
    ev: np.ndarray
    ew: np.ndarray            # merged edge weights (float64)
    degree: np.ndarray        # weighted degree d_i = sum of incident weights
    count_degree: np.ndarray  # number of distinct neighbours
    scale: np.ndarray         # s_i (1, or d_i^{-1/2}, 0 if isolated)
    old_of_new: np.ndarray    # original id of each kept node
    lambda_bound: float       # 2 (normalised) or 2 max_i d_i (combinatorial)

    # neighbour lists sorted by neighbour id: the order the walkers index into
    def adjacency(self):
        u = np.concatenate([self.eu, self.ev])
        v = np.concatenate([self.ev, self.eu])
        w = np.concatenate([self.ew, self.ew])
        order = np.lexsort((v, u))
        u, v, w = u[order], v[order], w[order]
        rowptr = np.zeros(self.n + 1, dtype=np.int64)
        np.add.at(rowptr, u + 1, 1)
        rowptr = np.cumsum(rowptr)
        return rowptr, v, w

    def dense(self) -> np.ndarray:
        return self.L.toarray()


def _largest_component(n, u, v):
    adj = sp.coo_matrix((np.ones(u.shape[0]), (u, v)), shape=(n, n))
    ncomp, lab = connected_components(adj, directed=False)
    sizes = np.bincount(lab, minlength=ncomp)
    best = sizes.max()
    # tie: the component containing the smallest node id
    first_node = np.full(ncomp, n, dtype=np.int64)
    np.minimum.at(first_node, lab, np.arange(n))
    cand = np.where(sizes == best)[0]
    comp = cand[np.argmin(first_node[cand])]
    return np.where(lab == comp)[0]


def laplacian(n, src, dst, w=None, kind: str = SYM_NORMALIZED, lcc: bool = False) -> Laplacian:
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    w = np.ones(src.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    if src.shape != dst.shape or src.shape != w.shape:
        raise ValueError("edge arrays differ in length")
    if src.size and (min(src.min(), dst.min()) < 0 or max(src.max(), dst.max()) >= n):
        raise ValueError("node id out of range")
    if np.any(~np.isfinite(w)) or np.any(w <= 0):
        raise ValueError("edge weights must be finite and positive")
    keep = src != dst                       # a self-loop has x_e = 0
    i = np.minimum(src, dst)[keep]
    j = np.maximum(src, dst)[keep]
    w = w[keep]
    old_of_new = np.arange(n, dtype=np.int64)
    if lcc and n > 0:
        kept = _largest_component(n, i, j)
        new_id = -np.ones(n, dtype=np.int64)
        new_id[kept] = np.arange(kept.shape[0])
        inside = new_id[i] >= 0
        i, j, w = new_id[i[inside]], new_id[j[inside]], w[inside]
        old_of_new = kept
        n = kept.shape[0]
    m = i.shape[0]

    # weighted degree: D_ii = sum of weights of edges touching i
    degree = np.zeros(n)
    np.add.at(degree, i, w)
    np.add.at(degree, j, w)
    if kind == SYM_NORMALIZED:
        scale = np.zeros(n)
        nz = degree > 0
        scale[nz] = 1.0 / np.sqrt(degree[nz])
        lambda_bound = 2.0
    elif kind == COMBINATORIAL:
        scale = np.ones(n)
        lambda_bound = 2.0 * (degree.max() if n else 0.0)
    else:
        raise ValueError(kind)

    # incidence matrix: row e = sqrt(w_e) * (s_i e_i - s_j e_j), i = min, j = max
    rows = np.repeat(np.arange(m), 2)
    cols = np.stack([i, j], axis=1).ravel()
    sw = np.sqrt(w)
    vals = np.stack([sw * scale[i], -sw * scale[j]], axis=1).ravel()
    X = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    L = (X.T @ X).tocsr()
    L.sum_duplicates()
    L.sort_indices()

    # merged undirected edges (repeats summed) for the walk estimator
    key = i * np.int64(n) + j
    uk, inv = np.unique(key, return_inverse=True)
    ew = np.zeros(uk.shape[0])
    np.add.at(ew, inv, w)
    eu, ev = uk // n, uk % n
    cdeg = np.bincount(np.concatenate([eu, ev]), minlength=n).astype(np.int64)
    return Laplacian(n=n, kind=kind, L=L, eu=eu, ev=ev, ew=ew, degree=degree,
                     count_degree=cdeg, scale=scale, old_of_new=old_of_new,
                     lambda_bound=float(lambda_bound))


def rows_times_block(n, src, dst, w, kind: str, rows, V_rows_fn):
    """Rows `rows` of L V straight from the edge list, without forming L.

    (L V)_r = sum over edges e = (r, j) of w_e s_r (s_r V_r - s_j V_j), which is
    row r of X~^T W X~ V (Sec. 2, weighted form; s = D^{-1/2} when normalised).
    Repeated edges contribute once each; self-loops contribute nothing.
    `V_rows_fn(ids)` returns the float64 rows of V for the node ids asked for
    (so V never has to be materialised in full).  Returns (len(rows), k).
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    rows = np.asarray(rows, dtype=np.int64)
    w = np.ones(src.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    keep = src != dst
    src, dst, w = src[keep], dst[keep], w[keep]
    degree = np.bincount(src, weights=w, minlength=n) + np.bincount(dst, weights=w, minlength=n)
    if kind == SYM_NORMALIZED:
        scale = np.zeros(n)
        nz = degree > 0
        scale[nz] = 1.0 / np.sqrt(degree[nz])
    else:
        scale = np.ones(n)
    pos = {int(r): i for i, r in enumerate(rows)}
    sel_a = np.isin(src, rows)
    sel_b = np.isin(dst, rows)
    r_of = np.concatenate([src[sel_a], dst[sel_b]])          # the sampled endpoint
    o_of = np.concatenate([dst[sel_a], src[sel_b]])          # the other endpoint
    w_of = np.concatenate([w[sel_a], w[sel_b]])
    Vr = V_rows_fn(rows)
    Vo = V_rows_fn(o_of)
    out = np.zeros((rows.shape[0], Vr.shape[1]))
    idx = np.array([pos[int(r)] for r in r_of], dtype=np.int64)
    contrib = (w_of * scale[r_of])[:, None] * (scale[r_of][:, None] * Vr[idx] - scale[o_of][:, None] * Vo)
    np.add.at(out, idx, contrib)
    return out
