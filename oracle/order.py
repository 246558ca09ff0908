"""Node orderings for gather locality (oracle; test infrastructure only).

The paper fixes no node order: p(L)V (Sec. 4.2) is the same operator under any
relabelling, with the rows of V permuted alike.  An order that puts the
neighbours of a node at nearby ids makes the neighbour-row gathers of the
sparse products touch fewer distinct cache lines.  Two orders are defined
here, each as plainly as it can be written:

* Cuthill-McKee (Cuthill and McKee, "Reducing the bandwidth of sparse
  symmetric matrices", ACM National Conference 1969): a breadth-first search
  that appends the unvisited neighbours of each dequeued node in increasing
  degree.  Readings: the search starts from the node of largest degree (ties:
  smallest id), neighbours of equal degree are taken in increasing id, and
  nodes the search does not reach (other components) follow in increasing id.
  Degree = number of distinct neighbours.
* Degree order: decreasing degree, ties in increasing id.

Both return `new_of_old`, the position of each node in the order.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def _neighbours(n, rowptr, col):
    return [col[rowptr[v]:rowptr[v + 1]].tolist() for v in range(n)]


def cuthill_mckee(n: int, rowptr, col) -> np.ndarray:
    """Cuthill-McKee order of the graph whose adjacency is the CSR (rowptr, col)
    (off-diagonal entries only, each undirected edge stored in both rows)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    nb = _neighbours(n, rowptr, col)
    deg = [len(x) for x in nb]
    order = []
    seen = [False] * n
    if n > 0:
        root = 0
        for v in range(1, n):
            if deg[v] > deg[root]:
                root = v
        seen[root] = True
        queue = deque([root])
        while queue:
            v = queue.popleft()
            order.append(v)
            fresh = sorted((u for u in nb[v] if not seen[u]), key=lambda u: (deg[u], u))
            for u in fresh:
                seen[u] = True
                queue.append(u)
    order += [v for v in range(n) if not seen[v]]
    new_of_old = np.empty(n, dtype=np.int64)
    for pos, v in enumerate(order):
        new_of_old[v] = pos
    return new_of_old


def degree_order(n: int, rowptr) -> np.ndarray:
    """Decreasing degree, ties in increasing id."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    deg = [int(rowptr[v + 1] - rowptr[v]) for v in range(n)]
    order = sorted(range(n), key=lambda v: (-deg[v], v))
    new_of_old = np.empty(n, dtype=np.int64)
    for pos, v in enumerate(order):
        new_of_old[v] = pos
    return new_of_old


def relabel_edges(src, dst, new_of_old):
    """The edge list with every endpoint replaced by its position."""
    new_of_old = np.asarray(new_of_old)
    return new_of_old[np.asarray(src)], new_of_old[np.asarray(dst)]
