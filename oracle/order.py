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
* Label-propagation order: nodes grouped by the communities that synchronous
  label propagation (Raghavan, Albert and Kumara, "Near linear time algorithm
  to detect community structures in large-scale networks", Phys. Rev. E 76,
  2007) finds, groups in increasing label; inside a group decreasing
  degree, then increasing id (a community's hubs share cache lines).
  Readings: every node starts with its own id as label; in each round every
  node with neighbours takes, from the previous round's labels, the label
  most frequent among its stored neighbours (unweighted counts); ties go to
  the label with the smallest splitmix64 output of (label XOR (round + 1) <<
  32), rounds counted from 0 (the published method breaks ties at random;
  this is a seeded stand-in); nodes without neighbours keep their label; at
  most LP_ROUNDS rounds, stopping early after a round that changes no label.

All return `new_of_old`, the position of each node in the order.
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


LP_ROUNDS = 16
_M64 = (1 << 64) - 1


def mix64(x: int) -> int:
    """The output function of splitmix64 (Steele, Lea and Flood, "Fast
    splittable pseudorandom number generators", OOPSLA 2014; the constants of
    Vigna's reference splitmix64): a bijection of 64-bit words."""
    x &= _M64
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & _M64
    return x ^ (x >> 31)


def mix64_np(x) -> np.ndarray:
    """mix64 on an array of 64-bit words (numpy's uint64 products wrap)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return x ^ (x >> np.uint64(31))


def label_propagation(n: int, rowptr, col, rounds: int = LP_ROUNDS, return_rounds: bool = False):
    """Labels after synchronous label propagation (readings in the module
    docstring); a node's label is the id of some node.  With return_rounds,
    also the number of rounds run (the last one changed nothing when it is
    below `rounds`)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    nb = _neighbours(n, rowptr, col)
    lab = list(range(n))
    ran = 0
    for r in range(rounds):
        ran = r + 1
        salt = (r + 1) << 32
        new = list(lab)
        for v in range(n):
            if not nb[v]:
                continue
            counts = {}
            for u in nb[v]:
                counts[lab[u]] = counts.get(lab[u], 0) + 1
            top = max(counts.values())
            new[v] = min((l for l, c in counts.items() if c == top), key=lambda l: mix64(l ^ salt))
        if new == lab:
            break
        lab = new
    lab = np.array(lab, dtype=np.int64)
    return (lab, ran) if return_rounds else lab


def label_propagation_np(n: int, rowptr, col, rounds: int = LP_ROUNDS) -> np.ndarray:
    """The same rounds as `label_propagation`, with numpy doing the counting
    (for graphs too large for the plain loops): each (node, neighbour label)
    pair is counted with np.unique, and each node keeps the pair of largest
    count, then smallest tie-break key.  Pinned against the loops on small
    graphs."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    lab = np.arange(n, dtype=np.int64)
    for r in range(rounds):
        salt = (r + 1) << 32
        pairs, counts = np.unique(rows * n + lab[col], return_counts=True) if n else (np.zeros(0, np.int64),) * 2
        node, cand = pairs // max(n, 1), pairs % max(n, 1)
        keys = mix64_np(cand.astype(np.uint64) ^ np.uint64(salt))
        # per node: largest count first, then smallest key
        pick = np.lexsort((keys, -counts, node))
        first = np.ones(pick.shape[0], dtype=bool)
        first[1:] = node[pick][1:] != node[pick][:-1]
        new = lab.copy()
        new[node[pick][first]] = cand[pick][first]
        if np.array_equal(new, lab):
            break
        lab = new
    return lab


def label_order(n: int, rowptr, col, rounds: int = LP_ROUNDS, fast: bool = False) -> np.ndarray:
    """Nodes sorted by (label after label propagation, decreasing degree,
    id); fast=True counts with numpy (label_propagation_np)."""
    lab = (label_propagation_np if fast else label_propagation)(n, rowptr, col, rounds)
    rowptr = np.asarray(rowptr, dtype=np.int64)
    deg = [int(rowptr[v + 1] - rowptr[v]) for v in range(n)]
    order = sorted(range(n), key=lambda v: (int(lab[v]), -deg[v], v))
    new_of_old = np.empty(n, dtype=np.int64)
    for pos, v in enumerate(order):
        new_of_old[v] = pos
    return new_of_old


def relabel_edges(src, dst, new_of_old):
    """The edge list with every endpoint replaced by its position."""
    new_of_old = np.asarray(new_of_old)
    return new_of_old[np.asarray(src)], new_of_old[np.asarray(dst)]
