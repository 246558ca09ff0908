"""Pins of the oracle's Laplacian (Sec. 2, Sec. 4.1) against closed forms,
identities and brute force that do not go through its incidence-matrix code."""
import numpy as np
import pytest

from oracle import laplacian as olap
from oracle import walk as owalk
from paper_2207_14589_amd import synth


def spectrum(lap):
    return np.linalg.eigvalsh(lap.dense())


@pytest.mark.parametrize("n", [2, 5, 17, 64])
def test_path_closed_forms(n):
    _, s, d = synth.path_graph(n)
    j = np.arange(n)
    comb = olap.laplacian(n, s, d, kind=olap.COMBINATORIAL)
    np.testing.assert_allclose(spectrum(comb), np.sort(2 - 2 * np.cos(np.pi * j / n)), atol=1e-12)
    norm = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    np.testing.assert_allclose(spectrum(norm), np.sort(1 - np.cos(np.pi * j / (n - 1))), atol=1e-12)


@pytest.mark.parametrize("n", [3, 8, 31])
def test_cycle_closed_forms(n):
    _, s, d = synth.cycle_graph(n)
    j = np.arange(n)
    comb = olap.laplacian(n, s, d, kind=olap.COMBINATORIAL)
    np.testing.assert_allclose(spectrum(comb), np.sort(2 - 2 * np.cos(2 * np.pi * j / n)), atol=1e-12)
    norm = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    np.testing.assert_allclose(spectrum(norm), np.sort(1 - np.cos(2 * np.pi * j / n)), atol=1e-12)


@pytest.mark.parametrize("m", [2, 4, 9])
def test_complete_graph(m):
    _, s, d = synth.complete_graph(m)
    comb = olap.laplacian(m, s, d, kind=olap.COMBINATORIAL)
    np.testing.assert_allclose(spectrum(comb), [0.0] + [m] * (m - 1), atol=1e-12)
    norm = olap.laplacian(m, s, d, kind=olap.SYM_NORMALIZED)
    np.testing.assert_allclose(spectrum(norm), [0.0] + [m / (m - 1)] * (m - 1), atol=1e-12)


def test_disjoint_cliques_nullspace():
    c, m = 4, 6
    n, s, d, labels = synth.disjoint_cliques(c, m)
    lap = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    lam, U = np.linalg.eigh(lap.dense())
    assert np.sum(np.abs(lam) < 1e-12) == c
    # null space = span{D^1/2 1_clique}
    B = np.zeros((n, c))
    deg = np.full(n, m - 1.0)
    for b in range(c):
        B[labels == b, b] = np.sqrt(deg[labels == b])
    Q, _ = np.linalg.qr(B)
    P = U[:, :c]
    assert np.linalg.norm(Q - P @ (P.T @ Q), 2) < 1e-10


def _brute_force_combinatorial(n, src, dst, w):
    """D - A by accumulating a dict of pair weights, one edge at a time."""
    A = {}
    for a, b, x in zip(src, dst, w):
        if a == b:
            continue
        A[(a, b)] = A.get((a, b), 0.0) + x
        A[(b, a)] = A.get((b, a), 0.0) + x
    M = np.zeros((n, n))
    for (a, b), x in A.items():
        M[a, b] -= x
        M[a, a] += x
    return M


def test_d_minus_a_and_quadratic_form():
    g = np.random.default_rng(3)
    n = 12
    src = g.integers(0, n, 40)
    dst = g.integers(0, n, 40)       # includes repeats and self-loops
    w = g.uniform(0.1, 1.0, 40)
    comb = olap.laplacian(n, src, dst, w, kind=olap.COMBINATORIAL)
    np.testing.assert_allclose(comb.dense(), _brute_force_combinatorial(n, src, dst, w), atol=1e-12)
    # v^T L v = sum_e w_e (s_i v_i - s_j v_j)^2 (eq. num_cut with weights and scaling)
    norm = olap.laplacian(n, src, dst, w, kind=olap.SYM_NORMALIZED)
    v = g.standard_normal(n)
    for lap in (comb, norm):
        q = 0.0
        for a, b, x in zip(src, dst, w):
            if a != b:
                q += x * (lap.scale[a] * v[a] - lap.scale[b] * v[b]) ** 2
        assert abs(v @ lap.dense() @ v - q) < 1e-11 * max(1.0, abs(q))


def test_null_vectors_and_bounds():
    n, s, d, _ = synth.sbm_bernoulli([30, 30, 40], 0.3, 0.02, seed=5)
    comb = olap.laplacian(n, s, d, kind=olap.COMBINATORIAL)
    norm = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    assert np.abs(comb.L @ np.ones(n)).max() < 1e-12                      # L 1 = 0
    assert np.abs(norm.L @ np.sqrt(norm.degree)).max() < 1e-12             # L D^1/2 1 = 0
    lam_c = spectrum(comb)
    lam_n = spectrum(norm)
    assert lam_c.min() > -1e-12 and lam_c.max() <= comb.lambda_bound + 1e-12
    assert lam_n.min() > -1e-12 and lam_n.max() <= 2 + 1e-12
    np.testing.assert_allclose(norm.dense(), norm.dense().T, atol=0)


def test_duplicates_sum_and_self_loops_drop():
    n = 5
    base_s, base_d, base_w = [0, 1, 2, 3], [1, 2, 3, 4], [1.0, 0.5, 1.0, 0.25]
    lap_dup = olap.laplacian(n, base_s + [1, 4, 2], base_d + [0, 3, 2], base_w + [1.0, 0.25, 7.0],
                             kind=olap.SYM_NORMALIZED)
    lap_ref = olap.laplacian(n, base_s, base_d, [2.0, 0.5, 1.0, 0.5], kind=olap.SYM_NORMALIZED)
    np.testing.assert_allclose(lap_dup.dense(), lap_ref.dense(), atol=1e-14)
    assert lap_dup.eu.shape[0] == 4


def test_components_and_lcc():
    # path of 5 plus triangle plus isolated node 8
    src = [0, 1, 2, 3, 5, 6, 7]
    dst = [1, 2, 3, 4, 6, 7, 5]
    lap = olap.laplacian(9, src, dst, kind=olap.SYM_NORMALIZED)
    lam = spectrum(lap)
    assert np.sum(np.abs(lam) < 1e-12) == 3          # one zero per component
    assert lap.scale[8] == 0.0
    sub = olap.laplacian(9, src, dst, kind=olap.SYM_NORMALIZED, lcc=True)
    assert sub.n == 5 and list(sub.old_of_new) == [0, 1, 2, 3, 4]
    ref = olap.laplacian(5, src[:4], dst[:4], kind=olap.SYM_NORMALIZED)
    np.testing.assert_allclose(sub.dense(), ref.dense(), atol=0)


def test_table1_edge_pair_products():
    """Table 1 (unweighted, combinatorial): serial -1, converging +1,
    diverging +1, repeated 2, disconnected 0."""
    # edges: 0:(0,1) 1:(1,2) 2:(0,2)... build a graph holding every pattern
    src = [0, 1, 3, 2, 6]
    dst = [1, 2, 1, 4, 7]
    lap = olap.laplacian(8, src, dst, kind=olap.COMBINATORIAL)
    idx = {(int(a), int(b)): e for e, (a, b) in enumerate(zip(lap.eu, lap.ev))}
    e01, e12, e13, e24, e67 = idx[(0, 1)], idx[(1, 2)], idx[(1, 3)], idx[(2, 4)], idx[(6, 7)]
    assert owalk.edge_pair_product(lap, e01, e12) == -1.0    # serial 0 -> 1 -> 2
    assert owalk.edge_pair_product(lap, e12, e24) == -1.0    # serial 1 -> 2 -> 4
    assert owalk.edge_pair_product(lap, e12, e13) == 1.0     # diverging 2 <- 1 -> 3
    src2, dst2 = [0, 1], [2, 2]
    lap2 = olap.laplacian(3, src2, dst2, kind=olap.COMBINATORIAL)
    assert owalk.edge_pair_product(lap2, 0, 1) == 1.0        # converging 0 -> 2 <- 1
    assert owalk.edge_pair_product(lap, e01, e01) == 2.0     # repeated
    assert owalk.edge_pair_product(lap, e01, e67) == 0.0     # disconnected


@pytest.mark.parametrize("kind", [olap.COMBINATORIAL, olap.SYM_NORMALIZED])
def test_rows_times_block_matches_full_operator(kind):
    """Sampled rows of L V from the edge list equal the full incidence-built
    operator applied to V (repeats, self-loops and weights included)."""
    g = np.random.default_rng(8)
    n = 300
    src = g.integers(0, n, 2000)
    dst = g.integers(0, n, 2000)
    w = g.uniform(0.1, 1.0, 2000)
    V = g.standard_normal((n, 5))
    lap = olap.laplacian(n, src, dst, w, kind=kind)
    rows = np.array([0, 7, 7 + 1, 150, n - 1])
    got = olap.rows_times_block(n, src, dst, w, kind, rows, lambda ids: V[ids])
    np.testing.assert_allclose(got, (lap.L @ V)[rows], rtol=1e-12, atol=1e-12)
