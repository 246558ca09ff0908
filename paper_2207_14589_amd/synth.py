"""Seeded synthetic inputs: graph edge lists and dense Gaussian blocks.

This module draws random graphs and random iterate blocks and nothing else: it
holds no Laplacian, polynomial, estimator or solver arithmetic, so the HIP path
and the FP64 oracle can both be fed from it without sharing any of the method.

Generators (every one is seeded and returns int64 ``src``/``dst`` arrays of
undirected edges, possibly with duplicates or self-loops only where stated):

* ``path_graph``, ``cycle_graph``, ``complete_graph``, ``disjoint_cliques`` --
  graphs whose Laplacian spectra have closed forms.
* ``sbm_bernoulli`` -- stochastic block model, one Bernoulli draw per node pair
  (small n, e.g. 2,000 nodes in 10 blocks with p_in=0.05, p_out=0.0005).
* ``sbm_sparse`` -- the same model for large n: a binomial edge count per block
  pair, then uniform distinct pairs (e.g. 10^6 nodes, 100 blocks, mean degree
  20 with 5% of edges crossing blocks).
* ``chung_lu`` -- degree-corrected power-law graph with planted communities.
* ``rmat`` -- recursive-matrix (R-MAT) graph, seeded vertex permutation.
* ``cliques_short_circuit`` -- cliques joined by 0..25 random cross edges, the
  well-clustered workload of the paper's clique experiments (Sec. 5.4).
* ``three_room_grid`` -- the 3-room grid-world state graph of Sec. 5.3.
* ``gaussian_block`` -- an n x k block with i.i.d. N(0,1) entries.
* ``rmat_device``, ``gaussian_block_device`` -- the same on the GPU with torch's
  seeded generator, for graphs and blocks too large to draw on the host.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "path_graph", "cycle_graph", "complete_graph", "disjoint_cliques",
    "sbm_bernoulli", "sbm_sparse", "sbm_from_degrees", "chung_lu", "rmat",
    "cliques_short_circuit", "three_room_grid", "gaussian_block",
    "random_weights", "rmat_device", "gaussian_block_device",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _canon_unique(u: np.ndarray, v: np.ndarray):
    """Orient pairs as (min, max), drop self-pairs and repeated pairs."""
    a = np.minimum(u, v).astype(np.int64)
    b = np.maximum(u, v).astype(np.int64)
    keep = a != b
    key = np.unique(a[keep] * (np.int64(1) << 32) + b[keep])
    return key >> 32, key & 0xFFFFFFFF


def path_graph(n: int):
    s = np.arange(n - 1, dtype=np.int64)
    return n, s, s + 1


def cycle_graph(n: int):
    s = np.arange(n, dtype=np.int64)
    return n, s, (s + 1) % n


def complete_graph(m: int, offset: int = 0):
    iu, ju = np.triu_indices(m, 1)
    return m + offset, iu.astype(np.int64) + offset, ju.astype(np.int64) + offset


def disjoint_cliques(c: int, m: int):
    src, dst = [], []
    for b in range(c):
        _, s, d = complete_graph(m, b * m)
        src.append(s)
        dst.append(d)
    labels = np.repeat(np.arange(c), m)
    return c * m, np.concatenate(src), np.concatenate(dst), labels


def sbm_bernoulli(block_sizes, p_in: float, p_out: float, seed: int):
    """One Bernoulli(p) draw per unordered node pair; nodes listed block by block."""
    sizes = np.asarray(block_sizes, dtype=np.int64)
    n = int(sizes.sum())
    labels = np.repeat(np.arange(len(sizes)), sizes)
    g = rng(seed)
    iu, ju = np.triu_indices(n, 1)
    p = np.where(labels[iu] == labels[ju], p_in, p_out)
    hit = g.random(iu.shape[0]) < p
    return n, iu[hit].astype(np.int64), ju[hit].astype(np.int64), labels


def _distinct_pairs_in_block(g, lo: int, size: int, count: int):
    """`count` distinct unordered pairs drawn uniformly inside [lo, lo+size)."""
    have = np.zeros(0, dtype=np.int64)
    need = count
    while need > 0:
        draw = int(need * 1.05) + 16
        u = g.integers(0, size, draw) + lo
        v = g.integers(0, size, draw) + lo
        a, b = _canon_unique(u, v)
        have = np.unique(np.concatenate([have, a * (np.int64(1) << 32) + b]))
        need = count - have.shape[0]
    if have.shape[0] > count:
        have = g.choice(have, count, replace=False)
    return have


def sbm_sparse(block_sizes, p_in: float, p_out: float, seed: int):
    """Stochastic block model sampled for large n.

    For each block the number of internal edges is Binomial(C(n_b, 2), p_in)
    and that many distinct pairs are drawn uniformly; the cross-block edge count
    is Binomial(#cross pairs, p_out) with pairs drawn uniformly over node pairs
    in different blocks.  The law equals independent Bernoulli edges.
    Nodes are listed block by block.
    """
    sizes = np.asarray(block_sizes, dtype=np.int64)
    n = int(sizes.sum())
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    labels = np.repeat(np.arange(len(sizes)), sizes)
    g = rng(seed)
    keys = []
    for lo, sz in zip(starts.tolist(), sizes.tolist()):
        pairs = sz * (sz - 1) // 2
        cnt = int(g.binomial(pairs, p_in))
        if cnt:
            keys.append(_distinct_pairs_in_block(g, lo, sz, cnt))
    cross_pairs = (n * n - int((sizes * sizes).sum())) // 2
    cnt = int(g.binomial(cross_pairs, p_out)) if cross_pairs else 0
    have = np.zeros(0, dtype=np.int64)
    need = cnt
    while need > 0:
        draw = int(need * 1.1) + 16
        u = g.integers(0, n, draw)
        v = g.integers(0, n, draw)
        ok = labels[u] != labels[v]
        a, b = _canon_unique(u[ok], v[ok])
        have = np.unique(np.concatenate([have, a * (np.int64(1) << 32) + b]))
        need = cnt - have.shape[0]
    if have.shape[0] > cnt:
        have = g.choice(have, cnt, replace=False)
    keys.append(have)
    key = np.sort(np.concatenate(keys))
    return n, key >> 32, key & 0xFFFFFFFF, labels


def sbm_from_degrees(n: int, blocks: int, d_in: float, d_out: float, seed: int):
    """Equal-block SBM with mean internal degree d_in and cross degree d_out."""
    sz = n // blocks
    sizes = [sz] * blocks
    sizes[-1] += n - sz * blocks
    p_in = d_in / (sz - 1)
    p_out = d_out / (n - sz)
    return sbm_sparse(sizes, p_in, p_out, seed)


def chung_lu(n: int, gamma: float, avg_degree: float, communities: int,
             p_within: float, seed: int):
    """Degree-corrected power-law graph with planted communities.

    Node weight w_i is proportional to (i+1)^(-1/(gamma-1)), capped at
    sqrt(sum w) and scaled so the mean degree is `avg_degree`.  Nodes are
    assigned to `communities` equal random communities.  Each of the n*d/2
    edge draws picks u with probability proportional to w, then v proportional
    to w inside u's community with probability `p_within`, else over all nodes.
    Self-pairs and repeats are dropped.
    """
    g = rng(seed)
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    w *= avg_degree * n / w.sum()
    cap = np.sqrt(w.sum())
    w = np.minimum(w, cap)
    w *= avg_degree * n / w.sum()
    comm = g.permutation(np.arange(n) % communities)
    m = int(round(n * avg_degree / 2))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    # per-community cumulative weights for the in-community endpoint
    order = np.argsort(comm, kind="stable")
    counts = np.bincount(comm, minlength=communities)
    cstart = np.concatenate([[0], np.cumsum(counts)[:-1]])
    w_sorted = w[order]
    ccdf = np.cumsum(w_sorted)
    cbase = np.concatenate([[0.0], ccdf])[cstart]
    ctot = ccdf[cstart + counts - 1] - cbase
    srcs, dsts = [], []
    chunk = 1 << 22
    for lo in range(0, m, chunk):
        cnt = min(chunk, m - lo)
        u = np.searchsorted(cdf, g.random(cnt), side="right")
        u = np.minimum(u, n - 1)
        inside = g.random(cnt) < p_within
        r = g.random(cnt)
        cu = comm[u]
        tgt = cbase[cu] + r * ctot[cu]
        vin = np.searchsorted(ccdf, tgt, side="right")
        vin = np.minimum(vin, cstart[cu] + counts[cu] - 1)
        vin = order[vin]
        vout = np.minimum(np.searchsorted(cdf, g.random(cnt), side="right"), n - 1)
        v = np.where(inside, vin, vout)
        srcs.append(u)
        dsts.append(v)
    a, b = _canon_unique(np.concatenate(srcs), np.concatenate(dsts))
    return n, a, b, comm


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         permute: bool = True, dedupe: bool = True):
    """R-MAT edges: each of edge_factor * 2^scale edges descends `scale` levels,
    choosing quadrant (0,0),(0,1),(1,0),(1,1) with probabilities a, b, c, 1-a-b-c.
    Vertex ids are then relabelled by a seeded random permutation."""
    g = rng(seed)
    n = 1 << scale
    m = edge_factor * n
    perm = g.permutation(n).astype(np.int64) if permute else None
    us, vs = [], []
    chunk = 1 << 22
    ab = a + b
    abc = a + b + c
    for lo in range(0, m, chunk):
        cnt = min(chunk, m - lo)
        u = np.zeros(cnt, dtype=np.int64)
        v = np.zeros(cnt, dtype=np.int64)
        for lev in range(scale):
            r = g.random(cnt)
            bit_u = r >= ab
            bit_v = ((r >= a) & (r < ab)) | (r >= abc)
            u |= bit_u.astype(np.int64) << lev
            v |= bit_v.astype(np.int64) << lev
        if permute:
            u = perm[u]
            v = perm[v]
        us.append(u)
        vs.append(v)
    u = np.concatenate(us)
    v = np.concatenate(vs)
    if dedupe:
        u, v = _canon_unique(u, v)
    return n, u, v


def cliques_short_circuit(n: int, c: int, seed: int, max_cross: int = 25):
    """n nodes in c equal cliques; each pair of cliques gets a uniform random
    number in [0, max_cross] of cross edges between random members."""
    g = rng(seed)
    sz = n // c
    src, dst = [], []
    for blk in range(c):
        _, s, d = complete_graph(sz, blk * sz)
        src.append(s)
        dst.append(d)
    for b1 in range(c):
        for b2 in range(b1 + 1, c):
            cnt = int(g.integers(0, max_cross + 1))
            src.append(g.integers(0, sz, cnt) + b1 * sz)
            dst.append(g.integers(0, sz, cnt) + b2 * sz)
    labels = np.repeat(np.arange(c), sz)
    a, b = _canon_unique(np.concatenate(src), np.concatenate(dst))
    return c * sz, a, b, labels


def link_prediction_cliques(n: int, c: int, seed: int, p_remove: float = 0.2, max_cross: int = 25):
    """The clique graph of `cliques_short_circuit` with each edge removed with
    probability p_remove, then completed by common-neighbours link prediction:
    every removed pair gets the number of neighbours its endpoints share in the
    remaining graph, divided by the largest such score, as its weight (kept
    edges weigh 1; removed pairs with no common neighbour stay absent).
    Returns (n, src, dst, w, labels)."""
    N, a, b, labels = cliques_short_circuit(n, c, seed, max_cross)
    g = rng(seed + 1)
    removed = g.random(a.shape[0]) < p_remove
    ka, kb = a[~removed], b[~removed]
    adj = [set() for _ in range(N)]
    for u, v in zip(ka.tolist(), kb.tolist()):
        adj[u].add(v)
        adj[v].add(u)
    ra, rb = a[removed], b[removed]
    score = np.array([len(adj[u] & adj[v]) for u, v in zip(ra.tolist(), rb.tolist())], dtype=np.float64)
    keep = score > 0
    w_pred = score[keep] / score.max() if keep.any() else score[keep]
    src = np.concatenate([ka, ra[keep]])
    dst = np.concatenate([kb, rb[keep]])
    w = np.concatenate([np.ones(ka.shape[0]), w_pred])
    return N, src, dst, w, labels


def three_room_grid(s: int = 2, h: int = 10):
    """State graph of a grid world (10s+1) tall and (30s+1) wide split into three
    rooms by two internal walls, each with a door (10s+1)//h cells tall; edges
    join 4-neighbour cells that are both free."""
    H, W = 10 * s + 1, 30 * s + 1
    free = np.ones((H, W), dtype=bool)
    door = max(1, (10 * s + 1) // h)
    d0 = (H - door) // 2
    for wc in (W // 3, 2 * W // 3):
        free[:, wc] = False
        free[d0:d0 + door, wc] = True
    ids = -np.ones((H, W), dtype=np.int64)
    ids[free] = np.arange(int(free.sum()))
    src, dst = [], []
    for (dy, dx) in ((0, 1), (1, 0)):
        a = ids[: H - dy, : W - dx]
        b = ids[dy:, dx:]
        ok = (a >= 0) & (b >= 0)
        src.append(a[ok])
        dst.append(b[ok])
    return int(free.sum()), np.concatenate(src), np.concatenate(dst)


def random_weights(m: int, seed: int, lo: float = 0.05, hi: float = 1.0):
    """Edge weights uniform in [lo, hi] (weighted graphs have w_e in (0, 1])."""
    return rng(seed).uniform(lo, hi, m)


def gaussian_block(n: int, k: int, seed: int) -> np.ndarray:
    """An n x k float64 block with i.i.d. N(0, 1) entries (row-major)."""
    return rng(seed).standard_normal((n, k))


def rmat_device(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
                device="cuda", chunk: int = 1 << 27):
    """R-MAT on the GPU with torch's seeded counter-based generator, for graphs
    too large to draw on the host (scale 26 = 1.07e9 edges): each edge descends
    `scale` levels choosing quadrant (0,0),(0,1),(1,0),(1,1) with probabilities
    a, b, c, 1-a-b-c; vertex ids are relabelled by a seeded random permutation;
    self-loops and repeated pairs are removed (the graph is unweighted).
    Returns (n, src, dst) as int32 device tensors with src < dst."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    n = 1 << scale
    m = edge_factor * n
    perm = torch.randperm(n, generator=g, device=device, dtype=torch.int64)
    ab, abc = a + b, a + b + c
    keys = []
    for lo in range(0, m, chunk):
        cnt = min(chunk, m - lo)
        u = torch.zeros(cnt, dtype=torch.int64, device=device)
        v = torch.zeros(cnt, dtype=torch.int64, device=device)
        for lev in range(scale):
            r = torch.rand(cnt, generator=g, device=device)
            u |= (r >= ab).to(torch.int64) << lev
            v |= (((r >= a) & (r < ab)) | (r >= abc)).to(torch.int64) << lev
            del r
        u = perm[u]
        v = perm[v]
        lo_, hi_ = torch.minimum(u, v), torch.maximum(u, v)
        del u, v
        k = (lo_ << 32) | hi_
        keys.append(k[lo_ != hi_])
        del lo_, hi_, k
    key = torch.unique(torch.cat(keys))
    del keys
    src = (key >> 32).to(torch.int32)
    dst = (key & 0xFFFFFFFF).to(torch.int32)
    return n, src, dst


def chung_lu_device(n: int, gamma: float, avg_degree: float, communities: int, p_within: float, seed: int,
                    device="cuda"):
    """The recipe of `chung_lu` drawn on the GPU with torch's seeded generator
    (a different realisation of the same distribution, seconds instead of
    minutes at n = 4e6): power-law weights capped at sqrt(sum w), equal random
    communities, u drawn proportional to w, v proportional to w inside u's
    community with probability p_within, else over all nodes; self-pairs and
    repeats dropped.  Returns (n, src, dst) int32 device tensors, src < dst."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    w = (torch.arange(n, dtype=f64, device=device) + 1.0) ** (-1.0 / (gamma - 1.0))
    w *= avg_degree * n / w.sum()
    w = torch.clamp(w, max=float(torch.sqrt(w.sum())))
    w *= avg_degree * n / w.sum()
    comm = torch.randperm(n, generator=g, device=device) % communities
    m = int(round(n * avg_degree / 2))
    cdf = torch.cumsum(w, 0)
    cdf /= cdf[-1].clone()
    order = torch.argsort(comm, stable=True)
    counts = torch.bincount(comm, minlength=communities)
    cstart = torch.cumsum(counts, 0) - counts
    ccdf = torch.cumsum(w[order], 0)
    cbase = torch.cat([torch.zeros(1, dtype=f64, device=device), ccdf])[cstart]
    ctot = ccdf[cstart + counts - 1] - cbase
    u = torch.searchsorted(cdf, torch.rand(m, generator=g, device=device, dtype=f64)).clamp_(max=n - 1)
    cu = comm[u]
    inside = torch.rand(m, generator=g, device=device, dtype=f64) < p_within
    t = cbase[cu] + torch.rand(m, generator=g, device=device, dtype=f64) * ctot[cu]
    vi = torch.searchsorted(ccdf, t).clamp_(min=0, max=n - 1)
    vi = torch.minimum(torch.maximum(vi, cstart[cu]), cstart[cu] + counts[cu] - 1)
    v_in = order[vi]
    v_out = torch.searchsorted(cdf, torch.rand(m, generator=g, device=device, dtype=f64)).clamp_(max=n - 1)
    v = torch.where(inside, v_in, v_out)
    lo, hi = torch.minimum(u, v), torch.maximum(u, v)
    key = torch.unique(((lo << 32) | hi)[lo != hi])
    return n, (key >> 32).to(torch.int32), (key & 0xFFFFFFFF).to(torch.int32)


def gaussian_block_device(n: int, k: int, seed: int, dtype=None, device="cuda"):
    """An n x k block of i.i.d. N(0, 1) entries drawn on the device (float32
    draws, optionally cast), for blocks too large to draw on the host."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    x = torch.randn(n, k, generator=g, device=device, dtype=torch.float32)
    return x if dtype is None else x.to(dtype)
