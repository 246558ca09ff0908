"""Pins of the oracle's node orderings (oracle/order.py): a hand-worked
Cuthill-McKee order, a declarative characterisation of the order checked on
random graphs, breadth-first levels from scipy's own search, and the
bandwidth bound every breadth-first order obeys; for label propagation the
published splitmix64 outputs, hand-worked oscillations (an edge, a star),
cliques whose final label follows from two rounds of reasoning, the
fixed-point condition counted independently, and the planted blocks of an
SBM."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

from oracle import laplacian as olap
from oracle import order as oorder
from paper_2207_14589_amd import synth


def adjacency(n, src, dst):
    lap = olap.laplacian(n, src, dst, kind=olap.COMBINATORIAL)
    rowptr, col, _ = lap.adjacency()
    return rowptr, col


# Nodes 0-8 form one component, 9-10 a second, 11 is isolated.
SMALL_EDGES = [(0, 1), (0, 2), (1, 3), (2, 3), (3, 4), (4, 5), (4, 6), (4, 7), (5, 8), (6, 8), (9, 10)]


def test_cuthill_mckee_hand_worked():
    # Degrees: 0..8 -> 2 2 2 3 4 2 2 1 2; 9, 10 -> 1; 11 -> 0.  The search
    # starts at node 4 (degree 4) and appends its neighbours by degree, then
    # id: 7 (1), 5 (2), 6 (2), 3 (3).  Dequeuing 7 adds nothing, 5 adds 8,
    # 6 nothing, 3 adds 1 then 2, 8 nothing, 1 adds 0.  Order 4 7 5 6 3 8 1 2 0,
    # then the unreached nodes 9 10 11 in id order.
    src, dst = zip(*SMALL_EDGES)
    rowptr, col = adjacency(12, np.array(src), np.array(dst))
    got = oorder.cuthill_mckee(12, rowptr, col)
    np.testing.assert_array_equal(got, [8, 6, 7, 4, 0, 2, 3, 1, 5, 9, 10, 11])


def test_degree_order_hand_worked():
    src, dst = zip(*SMALL_EDGES)
    rowptr, _ = adjacency(12, np.array(src), np.array(dst))
    # degree 4: node 4; 3: node 3; 2: 0 1 2 5 6 8; 1: 7 9 10; 0: 11
    got = oorder.degree_order(12, rowptr)
    np.testing.assert_array_equal(got, [2, 3, 4, 1, 0, 5, 6, 8, 7, 9, 10, 11])


def test_path_and_star():
    n, s, d = synth.path_graph(6)
    rowptr, col = adjacency(n, s, d)
    # every inner node has degree 2: the search starts at node 1, whose
    # neighbours are 0 (degree 1) and 2 (degree 2)
    order = np.argsort(oorder.cuthill_mckee(n, rowptr, col))
    np.testing.assert_array_equal(order, [1, 0, 2, 3, 4, 5])
    # star: hub 3 first, then the leaves in id order
    src = np.array([3, 3, 3, 3, 3])
    dst = np.array([0, 1, 2, 4, 5])
    rowptr, col = adjacency(6, src, dst)
    order = np.argsort(oorder.cuthill_mckee(6, rowptr, col))
    np.testing.assert_array_equal(order, [3, 0, 1, 2, 4, 5])


def test_empty_and_edgeless():
    assert oorder.cuthill_mckee(0, np.zeros(1, np.int64), np.zeros(0, np.int64)).shape == (0,)
    rowptr = np.zeros(5, np.int64)
    np.testing.assert_array_equal(oorder.cuthill_mckee(4, rowptr, np.zeros(0, np.int64)), np.arange(4))
    np.testing.assert_array_equal(oorder.degree_order(4, rowptr), np.arange(4))


def characterise(n, rowptr, col, new_of_old):
    """What fixes a Cuthill-McKee order, stated without a queue: the root has
    the largest degree (ties: smallest id); every other reached node comes
    after its earliest-placed neighbour, and the reached nodes other than the
    root appear sorted by (position of that neighbour, degree, id); the
    unreached nodes follow in id order."""
    pos = np.asarray(new_of_old)
    assert sorted(pos.tolist()) == list(range(n))
    deg = np.diff(rowptr)
    order = np.argsort(pos)
    if n == 0:
        return
    root = order[0]
    assert deg[root] == deg.max() and root == np.flatnonzero(deg == deg.max())[0]
    adj = sp.csr_matrix((np.ones(col.shape[0]), col, rowptr), shape=(n, n))
    dist = shortest_path(adj, unweighted=True, indices=root)
    reached = np.isfinite(dist)
    nr = int(reached.sum())
    assert reached[order[:nr]].all()
    np.testing.assert_array_equal(order[nr:], np.sort(np.flatnonzero(~reached)))
    keys = []
    for v in order[1:nr]:
        nb = col[rowptr[v]:rowptr[v + 1]]
        parent_pos = pos[nb].min()
        assert parent_pos < pos[v]
        keys.append((int(parent_pos), int(deg[v]), int(v)))
    assert keys == sorted(keys)
    # breadth-first: levels never decrease along the order (scipy's distances)
    assert np.all(np.diff(dist[order[:nr]]) >= 0)
    # and every edge joins equal or adjacent levels, so its span is at most
    # the sizes of two consecutive levels
    lv = dist[order[:nr]].astype(np.int64)
    sizes = np.bincount(lv)
    r = np.repeat(np.arange(n), np.diff(rowptr))
    inside = reached[r]
    span = np.abs(pos[r[inside]] - pos[col[inside]])
    lo = np.minimum(dist[r[inside]], dist[col[inside]]).astype(np.int64)
    assert np.all(np.abs(dist[r[inside]] - dist[col[inside]]) <= 1)
    bound = sizes[lo] + np.append(sizes, 0)[lo + 1] - 1
    assert np.all(span <= bound)


@pytest.mark.parametrize("case", ["sbm", "powerlaw", "grid", "rmat", "forest"])
def test_cuthill_mckee_characterisation(case):
    if case == "sbm":
        n, s, d, _ = synth.sbm_sparse([60, 80, 70], 0.15, 0.01, seed=3)
    elif case == "powerlaw":
        n, s, d, _ = synth.chung_lu(600, 2.1, 6.0, 4, 0.8, seed=5)
    elif case == "grid":
        n, s, d = synth.three_room_grid(2, 6)
    elif case == "rmat":
        n, s, d = synth.rmat(10, 8, 0.57, 0.19, 0.19, seed=7)
    else:  # several trees and isolated nodes
        g = np.random.default_rng(11)
        n = 300
        s = np.arange(1, 250)
        d = g.integers(0, s)
        keep = g.random(s.shape[0]) < 0.8
        s, d = s[keep], d[keep]
    rowptr, col = adjacency(n, s, d)
    characterise(n, rowptr, col, oorder.cuthill_mckee(n, rowptr, col))


def test_characterisation_catches_plausible_mistakes():
    """The check above fails for orders a slip in the search would give."""
    n, s, d, _ = synth.sbm_sparse([40, 50], 0.2, 0.02, seed=1)
    rowptr, col = adjacency(n, s, d)
    good = oorder.cuthill_mckee(n, rowptr, col)
    order = np.argsort(good)
    deg = np.diff(rowptr)
    bad = []
    # neighbours by decreasing degree (a flipped sort)
    flip = order.copy()
    for i in range(1, n - 1):
        if flip[i] != flip[i + 1] and deg[flip[i]] < deg[flip[i + 1]]:
            flip[[i, i + 1]] = flip[[i + 1, i]]
            break
    bad.append(flip)
    # the reversed order (reverse Cuthill-McKee)
    bad.append(order[::-1].copy())
    for b in bad:
        pos = np.empty(n, np.int64)
        pos[b] = np.arange(n)
        with pytest.raises(AssertionError):
            characterise(n, rowptr, col, pos)


def test_degree_order_properties():
    n, s, d, _ = synth.chung_lu(500, 2.1, 6.0, 4, 0.8, seed=2)
    rowptr, _ = adjacency(n, s, d)
    pos = oorder.degree_order(n, rowptr)
    order = np.argsort(pos)
    deg = np.diff(rowptr)
    assert np.all(np.diff(deg[order]) <= 0)
    same = np.diff(deg[order]) == 0
    assert np.all(np.diff(order)[same] > 0)


def test_relabelled_laplacian_is_the_permuted_one():
    n, s, d, _ = synth.sbm_sparse([30, 40], 0.2, 0.03, seed=4)
    rowptr, col = adjacency(n, s, d)
    pos = oorder.cuthill_mckee(n, rowptr, col)
    s2, d2 = oorder.relabel_edges(s, d, pos)
    A = olap.laplacian(n, s, d).dense()
    B = olap.laplacian(n, s2, d2).dense()
    P = np.zeros((n, n))
    P[pos, np.arange(n)] = 1.0
    np.testing.assert_allclose(B, P @ A @ P.T, atol=1e-15)


# ---------------------------------------------------------------- label propagation


def test_mix64_is_splitmix64():
    # splitmix64 started at state 0 adds the golden-ratio increment before
    # each output; its published first outputs pin the constants and shifts
    g = 0x9E3779B97F4A7C15
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    got = [oorder.mix64((g * i) & ((1 << 64) - 1)) for i in (1, 2, 3)]
    assert got == want
    assert oorder.mix64(0) == 0


def _first_round_winner(ids):
    """The member with the smallest round-0 tie-break key."""
    return min(ids, key=lambda l: oorder.mix64(l ^ (1 << 32)))


def test_label_propagation_single_edge_and_star_oscillate():
    # K2: each end takes the other's label every round, so an even number of
    # rounds gives the ids back and an odd number swaps them.
    assert list(oorder.label_propagation(2, [0, 1, 2], [1, 0], rounds=16)) == [0, 1]
    assert list(oorder.label_propagation(2, [0, 1, 2], [1, 0], rounds=15)) == [1, 0]
    # Star, centre 0, leaves 1..5.  Round 0: the leaves see only label 0; the
    # centre sees five labels once each and takes the round-0 winner a.
    # Round 1: the centre sees 0 five times, the leaves see a.  From then on
    # the two label sets swap every round, so after 16 rounds the centre is 0
    # and the leaves are a.
    src = np.zeros(5, np.int64)
    dst = np.arange(1, 6)
    rowptr, col = adjacency(6, src, dst)
    a = _first_round_winner(range(1, 6))
    assert list(oorder.label_propagation(6, rowptr, col)) == [0] + [a] * 5


@pytest.mark.parametrize("sizes", [[4, 5, 6], [7, 4, 9, 5]])
def test_label_propagation_cliques(sizes):
    # In a clique of m >= 4 nodes, round 0 gives every member except the
    # round-0 winner a (it cannot take its own label) the label a.  In round 1
    # a member other than a sees a m - 2 >= 2 times and a's own label once,
    # and a sees only a: every member ends with a, and the next round
    # changes nothing.
    src, dst, base = [], [], 0
    for m in sizes:
        for i in range(m):
            for j in range(i + 1, m):
                src.append(base + i)
                dst.append(base + j)
        base += m
    n = base
    rowptr, col = adjacency(n, np.array(src), np.array(dst))
    lab, ran = oorder.label_propagation(n, rowptr, col, return_rounds=True)
    base = 0
    for m in sizes:
        members = range(base, base + m)
        assert set(lab[base:base + m]) == {_first_round_winner(members)}
        base += m
    assert ran == 3


def test_label_propagation_fixed_point_and_planted_blocks():
    """On the 10-block SBM the search stops before its cap; at that point
    every node's label is one of the most frequent among its neighbours
    (counted here with numpy, independently of the oracle's loops), and the
    labels recover the planted blocks."""
    n, s, d, blocks = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    rowptr, col = adjacency(n, s, d)
    lab, ran = oorder.label_propagation(n, rowptr, col, return_rounds=True)
    assert ran < oorder.LP_ROUNDS
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    key = rows * n + lab[col]
    uk, cnt = np.unique(key, return_counts=True)
    top = np.zeros(n, np.int64)
    np.maximum.at(top, uk // n, cnt)
    mine = dict(zip(uk.tolist(), cnt.tolist()))
    for v in range(n):
        if rowptr[v + 1] > rowptr[v]:
            assert mine.get(v * n + int(lab[v]), 0) == top[v]
    # purity: each label's nodes lie in one planted block
    for l in np.unique(lab):
        assert len(np.unique(blocks[lab == l])) == 1
    assert 10 <= len(np.unique(lab)) <= 14


def test_label_order_properties():
    n, s, d, _ = synth.sbm_bernoulli([60, 80, 50], 0.1, 0.005, seed=4)
    n += 3  # isolated nodes keep their own labels
    rowptr, col = adjacency(n, s, d)
    lab = oorder.label_propagation(n, rowptr, col)
    pos = oorder.label_order(n, rowptr, col)
    assert sorted(pos.tolist()) == list(range(n))
    order = np.argsort(pos)
    deg = np.diff(rowptr)
    keys = list(zip(lab[order].tolist(), (-deg[order]).tolist(), order.tolist()))
    assert keys == sorted(keys)  # grouped by label; decreasing degree, then id inside
    assert all(lab[v] == v for v in range(n - 3, n))


def test_label_propagation_empty_and_edgeless():
    assert oorder.label_order(0, [0], []).shape == (0,)
    np.testing.assert_array_equal(oorder.label_order(4, [0, 0, 0, 0, 0], []), np.arange(4))
    np.testing.assert_array_equal(oorder.label_propagation(4, [0, 0, 0, 0, 0], []), np.arange(4))


def test_label_propagation_pins_catch_plausible_mistakes(monkeypatch):
    """Ties broken by the smallest label instead of the hash (every clique
    would end at its smallest id) fail the clique pin above."""
    sizes = [4, 5, 6]
    src, dst, base = [], [], 0
    for m in sizes:
        for i in range(m):
            for j in range(i + 1, m):
                src.append(base + i)
                dst.append(base + j)
        base += m
    rowptr, col = adjacency(base, np.array(src), np.array(dst))
    want = []
    base = 0
    for m in sizes:
        want += [_first_round_winner(range(base, base + m))] * m
        base += m
    assert list(oorder.label_propagation(base, rowptr, col)) == want
    # smallest-label ties: every clique ends at its smallest id instead
    monkeypatch.setattr(oorder, "mix64", lambda x: x & 0xFFFFFFFF)
    assert list(oorder.label_propagation(base, rowptr, col)) != want


@pytest.mark.parametrize("seed", range(6))
def test_label_propagation_numpy_form_matches_the_loops(seed):
    """Brute force: the numpy-counting form equals the plain loops, round
    for round, on small random graphs (several components, isolated nodes,
    ties, 2-cycles) and for every round cap."""
    g = np.random.default_rng(seed)
    n = int(g.integers(5, 60))
    m = int(g.integers(0, 3 * n))
    src, dst = g.integers(0, n, m), g.integers(0, n, m)
    rowptr, col = adjacency(n, src, dst)
    for rounds in (1, 2, 5, oorder.LP_ROUNDS):
        np.testing.assert_array_equal(oorder.label_propagation_np(n, rowptr, col, rounds),
                                      oorder.label_propagation(n, rowptr, col, rounds))
    np.testing.assert_array_equal(oorder.label_order(n, rowptr, col, fast=True), oorder.label_order(n, rowptr, col))


def test_label_propagation_numpy_form_on_the_planted_graph():
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    rowptr, col = adjacency(n, s, d)
    np.testing.assert_array_equal(oorder.label_propagation_np(n, rowptr, col), oorder.label_propagation(n, rowptr, col))


def test_mix64_array_form():
    g = np.random.default_rng(3)
    x = g.integers(0, 2 ** 63, 1000, dtype=np.int64).astype(np.uint64) * np.uint64(2) + np.uint64(1)
    np.testing.assert_array_equal(oorder.mix64_np(x), np.array([oorder.mix64(int(v)) for v in x], dtype=np.uint64))
