"""Pins for the edge-minibatch oracle (oracle/stream.py) -- no GPU.

The sum over all edges of x_e x_e^T V must be L V with L built from the
incidence matrix by its definition (Sec. 2: L = X^T X, weighted X^T W X;
Sec. 4.1: columns scaled by s_i = d_i^{-1/2}); degrees are checked on a
graph small enough to add up by hand."""
import numpy as np
import pytest

from oracle import laplacian as olap
from oracle import stream as ost


def incidence_laplacian(n, src, dst, w, scale):
    """X^T X with one row per edge: +sqrt(w) s_i at min(i, j), -sqrt(w) s_j at
    max(i, j); a self-loop's row is zero."""
    rows = []
    for i, j, wt in zip(src, dst, w):
        x = np.zeros(n)
        if i != j:
            a, b = min(i, j), max(i, j)
            x[a] = np.sqrt(wt) * scale[a]
            x[b] = -np.sqrt(wt) * scale[b]
        rows.append(x)
    X = np.array(rows)
    return X.T @ X


def small_graph():
    # repeats (0, 1) twice and (2, 3) in both directions, a self-loop at 4,
    # node 5 isolated
    src = np.array([0, 1, 0, 2, 3, 4, 1, 3])
    dst = np.array([1, 0, 2, 3, 2, 4, 3, 0])
    w = np.array([1.0, 2.0, 0.5, 3.0, 1.5, 7.0, 0.25, 4.0])
    return 6, src, dst, w


def test_degrees_by_hand():
    n, src, dst, w = small_graph()
    d, s = ost.node_scales(n, src, dst, w, kind=ost.SYM_NORMALIZED)
    # node 0: 1 + 2 + 0.5 + 4; node 1: 1 + 2 + 0.25; node 2: 0.5 + 3 + 1.5;
    # node 3: 3 + 1.5 + 0.25 + 4; node 4: only its self-loop; node 5: none
    np.testing.assert_array_equal(d, [7.5, 3.25, 5.0, 8.75, 0.0, 0.0])
    np.testing.assert_allclose(s[:4], 1.0 / np.sqrt([7.5, 3.25, 5.0, 8.75]), rtol=1e-15)
    assert s[4] == 0.0 and s[5] == 0.0
    d2, s2 = ost.node_scales(n, src, dst, w, kind=ost.COMBINATORIAL)
    np.testing.assert_array_equal(d2, d)
    np.testing.assert_array_equal(s2, np.ones(n))


@pytest.mark.parametrize("kind", [ost.COMBINATORIAL, ost.SYM_NORMALIZED])
def test_full_pass_is_incidence_laplacian(kind):
    n, src, dst, w = small_graph()
    _, s = ost.node_scales(n, src, dst, w, kind=kind)
    V = np.random.default_rng(1).standard_normal((n, 3))
    Y = ost.edge_batch_apply(n, src, dst, w, s, V)
    L = incidence_laplacian(n, src, dst, w, s)
    np.testing.assert_allclose(Y, L @ V, rtol=1e-13, atol=1e-13)
    # L 1 = 0 for the combinatorial form; L D^{1/2} 1 = 0 for the normalised one
    d, _ = ost.node_scales(n, src, dst, w, kind=kind)
    null = np.ones((n, 1)) if kind == ost.COMBINATORIAL else np.sqrt(d)[:, None]
    np.testing.assert_allclose(ost.edge_batch_apply(n, src, dst, w, s, null), 0.0, atol=1e-13)


@pytest.mark.parametrize("kind", [olap.COMBINATORIAL, olap.SYM_NORMALIZED])
def test_full_pass_matches_csr_oracle(kind):
    g = np.random.default_rng(7)
    n, m = 300, 2500
    src = g.integers(0, n, m)
    dst = g.integers(0, n, m)
    w = g.uniform(0.05, 1.0, m)
    ref = olap.laplacian(n, src, dst, w=w, kind=kind)
    _, s = ost.node_scales(n, src, dst, w, kind=kind)
    np.testing.assert_allclose(s, ref.scale, rtol=1e-14)
    V = g.standard_normal((n, 5))
    np.testing.assert_allclose(ost.edge_batch_apply(n, src, dst, w, s, V), ref.L @ V, rtol=1e-12, atol=1e-12)
    # the endpoint order of an edge does not matter
    np.testing.assert_allclose(ost.edge_batch_apply(n, dst, src, w, s, V), ref.L @ V, rtol=1e-12, atol=1e-12)


def test_batches_add_up_and_single_edge_mean_is_unbiased():
    n, src, dst, w = small_graph()
    _, s = ost.node_scales(n, src, dst, w)
    V = np.random.default_rng(3).standard_normal((n, 2))
    full = ost.edge_batch_apply(n, src, dst, w, s, V)
    parts = sum(ost.edge_batch_apply(n, src[a:a + 3], dst[a:a + 3], w[a:a + 3], s, V) for a in range(0, 8, 3))
    np.testing.assert_allclose(parts, full, rtol=1e-14, atol=1e-14)
    # a batch of one uniformly drawn edge, scaled by m: its mean over the m
    # equally likely draws is the full product
    m = len(src)
    mean = sum(m * ost.edge_batch_apply(n, src[e:e + 1], dst[e:e + 1], w[e:e + 1], s, V) for e in range(m)) / m
    np.testing.assert_allclose(mean, full, rtol=1e-13, atol=1e-13)


def test_minibatch_oja_full_batch_limit_step_is_the_limit_product():
    """With one batch holding every edge the limit-polynomial step is
    orth(V + eta (I - L/l)^l V) exactly; (I - L/l)^l V from the product
    oracle, orthonormalised by a textbook QR."""
    from oracle import poly as opoly
    from oracle import solver as osol
    g = np.random.default_rng(2)
    n, m = 80, 400
    src, dst = g.integers(0, n, m), g.integers(0, n, m)
    w = g.uniform(0.1, 1.0, m)
    ref = olap.laplacian(n, src, dst, w=w, kind=olap.SYM_NORMALIZED)
    _, s = ost.node_scales(n, src, dst, w)
    V0 = np.linalg.qr(g.standard_normal((n, 4)))[0]
    V = ost.minibatch_oja(n, src, dst, w, s, 6, 2.0, V0, batch=m, eta=0.7, iters=1)
    Vr = np.linalg.qr(V0 + 0.7 * opoly.apply_limit_product(ref.L, 6, V0))[0]
    assert osol.max_principal_angle(V, Vr) < 1e-10
    np.testing.assert_allclose(V.T @ V, np.eye(4), atol=1e-12)


def test_minibatch_oja_fixed_point_and_drawn_batches():
    """The bottom eigenvectors are a fixed point of the full-batch plain step
    (lambda I - L keeps them, orth keeps their span); a batch that starts near
    the end of the list wraps to its first edges; the solver's steps equal the
    same factors applied by hand with a textbook QR, batch J starting at the
    J-th drawn offset, and a solve split in two calls (batch0 = batches drawn
    before) continues the same stream."""
    from oracle import solver as osol
    n, src, dst, w = small_graph()
    _, s = ost.node_scales(n, src, dst, w)
    L = incidence_laplacian(n, src, dst, w, s)
    _, U = np.linalg.eigh(L)
    U = U[:, :3]
    V = ost.minibatch_oja(n, src, dst, w, s, 0, 2.0, U, batch=len(src), eta=0.5, iters=5)
    assert osol.max_principal_angle(U, V) < 1e-10
    m = len(src)
    np.testing.assert_array_equal(ost.drawn_batch(m, m - 3, 5), [m - 3, m - 2, m - 1, 0, 1])
    offs = ost.batch_offsets(17, m, 0, 400)
    assert offs.min() >= 0 and offs.max() < m and len(np.unique(offs)) == m   # every offset drawn
    V0 = np.linalg.qr(np.random.default_rng(4).standard_normal((n, 2)))[0]
    Va = ost.minibatch_oja(n, src, dst, w, s, 2, 2.0, V0, batch=5, eta=0.3, iters=3, seed=17)
    Vh = V0.copy()
    j = 0
    for _ in range(3):
        W = Vh
        for _f in range(2):
            idx = ost.drawn_batch(m, offs[j], 5)
            j += 1
            W = W - ost.edge_batch_apply(n, src[idx], dst[idx], w[idx], s, W) * (m / 5) / 2
        Vh = np.linalg.qr(Vh + 0.3 * W)[0]
    assert osol.max_principal_angle(Va, Vh) < 1e-10
    V1 = ost.minibatch_oja(n, src, dst, w, s, 2, 2.0, V0, batch=5, eta=0.3, iters=1, seed=17)
    V2 = ost.minibatch_oja(n, src, dst, w, s, 2, 2.0, V1, batch=5, eta=0.3, iters=2, seed=17, batch0=2)
    assert osol.max_principal_angle(Va, V2) < 1e-10


@pytest.mark.parametrize("ell,b", [(2, 1), (2, 3), (3, 2)])
def test_drawn_batch_product_is_unbiased(ell, b):
    """E[(I - (m/b) L_{B_l} / l) ... (I - (m/b) L_{B_1} / l)] = (I - L/l)^l when
    each factor's batch starts at its own uniform offset: enumerate every
    offset tuple (m^l of them) and average the product exactly.  A schedule
    whose factors take disjoint consecutive runs of one list (without
    replacement) fails this on the same graph."""
    g = np.random.default_rng(7)
    n, m = 6, 11
    src = g.integers(0, n, m)
    dst = (src + 1 + g.integers(0, n - 1, m)) % n
    w = g.uniform(0.2, 1.0, m)
    _, s = ost.node_scales(n, src, dst, w)
    I = np.eye(n)
    LB = [ost.edge_batch_apply(n, src[ost.drawn_batch(m, o, b)], dst[ost.drawn_batch(m, o, b)],
                               w[ost.drawn_batch(m, o, b)], s, I) * (m / b) for o in range(m)]
    L = incidence_laplacian(n, src, dst, w, s)
    mean = np.zeros((n, n))
    import itertools
    for offs in itertools.product(range(m), repeat=ell):
        P = I.copy()
        for o in offs:
            P = (I - LB[o] / ell) @ P
        mean += P
    mean /= m ** ell
    exact = np.linalg.matrix_power(I - L / ell, ell)
    np.testing.assert_allclose(mean, exact, atol=1e-12)
    # consecutive disjoint runs of one list (the factors not independent)
    if b * ell <= m:
        bad = np.zeros((n, n))
        for start in range(m):
            P = I.copy()
            for f in range(ell):
                P = (I - LB[(start + f * b) % m] / ell) @ P
            bad += P
        bad /= m
        assert np.abs(bad - exact).max() > 1e-3
