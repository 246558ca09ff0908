"""k-means on the spectral embedding (oracle; test infrastructure only).

Sec. 1: the bottom-k eigenvectors give each node a k-dimensional embedding (a
soft clustering) and a hard clustering follows with k-means; Sec. 2.1 uses
k-means with k = 2 on the Fiedler vector.  The paper fixes neither the
seeding, the row normalisation nor the stopping rule; the readings used here:
rows are optionally scaled to unit length (Ng-Jordan-Weiss for the normalised
Laplacian), Lloyd iterations run from given centres (or k-means++ centres
drawn with numpy) until no label changes or `max_iters`, and a tie between
centres goes to the lower centre index.
"""
from __future__ import annotations

import numpy as np


def normalize_rows(X):
    X = np.asarray(X, dtype=np.float64)
    nrm = np.linalg.norm(X, axis=1, keepdims=True)
    return np.where(nrm > 0, X / np.where(nrm > 0, nrm, 1.0), 0.0)


def assign(X, C):
    """Label of the nearest centre by squared distance; ties -> lowest index."""
    d2 = ((X[:, None, :] - C[None, :, :]) ** 2).sum(axis=2)
    return np.argmin(d2, axis=1), d2


def lloyd(X, C0, max_iters: int = 300):
    X = np.asarray(X, dtype=np.float64)
    C = np.asarray(C0, dtype=np.float64).copy()
    labels, _ = assign(X, C)
    it = 0
    for it in range(1, max_iters + 1):
        for c in range(C.shape[0]):
            members = X[labels == c]
            if members.shape[0]:
                C[c] = members.mean(axis=0)
        new, _ = assign(X, C)
        if np.array_equal(new, labels):
            labels = new
            break
        labels = new
    _, d2 = assign(X, C)
    inertia = float(d2[np.arange(X.shape[0]), labels].sum())
    return labels, C, inertia, it


def kmeans_pp(X, n_clusters: int, seed: int):
    g = np.random.Generator(np.random.PCG64(seed))
    X = np.asarray(X, dtype=np.float64)
    C = [X[g.integers(0, X.shape[0])]]
    d2 = ((X - C[0]) ** 2).sum(axis=1)
    for _ in range(1, n_clusters):
        p = d2 / d2.sum() if d2.sum() > 0 else np.full(X.shape[0], 1.0 / X.shape[0])
        C.append(X[g.choice(X.shape[0], p=p)])
        d2 = np.minimum(d2, ((X - C[-1]) ** 2).sum(axis=1))
    return np.array(C)


def canonical_labels(labels):
    """Relabel clusters by order of first appearance."""
    labels = np.asarray(labels)
    _, first = np.unique(labels, return_index=True)
    order = labels[np.sort(first)]
    remap = {int(c): i for i, c in enumerate(order)}
    return np.array([remap[int(c)] for c in labels])


def adjusted_rand_index(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    table = np.zeros((ai.max() + 1, bi.max() + 1))
    np.add.at(table, (ai, bi), 1)

    def c2(x):
        return x * (x - 1) / 2.0

    sum_ij = c2(table).sum()
    sa = c2(table.sum(axis=1)).sum()
    sb = c2(table.sum(axis=0)).sum()
    expected = sa * sb / c2(a.shape[0])
    maxi = 0.5 * (sa + sb)
    return float((sum_ij - expected) / (maxi - expected)) if maxi != expected else 1.0
