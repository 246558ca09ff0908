"""Pins of the oracle's solver, metrics, k-means and gradient."""
import numpy as np
import pytest

from oracle import grad as ograd
from oracle import kmeans as okm
from oracle import laplacian as olap
from oracle import poly as opoly
from oracle import solver as osol
from paper_2207_14589_amd import synth


def _rotated_pair(n, angles, seed=0):
    """Two k-dim subspaces whose principal angles are exactly `angles`."""
    g = np.random.default_rng(seed)
    k = len(angles)
    Q, _ = np.linalg.qr(g.standard_normal((n, 2 * k)))
    A = Q[:, :k]
    B = np.cos(angles) * Q[:, :k] + np.sin(angles) * Q[:, k:]
    return A, B


def test_metrics_known_angles():
    ang = np.array([1e-9, 3e-7, 0.2, 0.7])
    A, B = _rotated_pair(50, ang)
    assert osol.max_principal_angle(A, B) == pytest.approx(0.7, rel=1e-12)
    assert osol.subspace_error(A, B) == pytest.approx(np.mean(np.sin(ang) ** 2), rel=1e-10)
    A2, B2 = _rotated_pair(50, np.array([2e-8, 1e-9]))
    assert osol.max_principal_angle(A2, B2) == pytest.approx(2e-8, rel=1e-6)
    np.testing.assert_allclose(osol.vector_angles(A, B), ang, rtol=1e-6, atol=1e-15)
    assert osol.eigenvector_streak(A, B, eps=0.5) == 3


def test_residual_norm_bound_cases():
    """rho >= ||R||_2 always, <= ||R||_F, and exact for orthogonal columns
    (||R||_2 is then the largest column norm) and for rank one."""
    g = np.random.default_rng(3)
    for _ in range(20):
        R = g.standard_normal((40, 6)) * g.uniform(0.1, 3.0, 6)
        rho = osol.residual_norm_bound(R)
        assert np.linalg.norm(R, 2) <= rho * (1 + 1e-12)
        assert rho <= np.linalg.norm(R) * (1 + 1e-12)
    Q, _ = np.linalg.qr(g.standard_normal((40, 5)))
    D = Q * np.array([0.5, 2.0, 1.0, 0.1, 1.5])
    assert osol.residual_norm_bound(D) == pytest.approx(2.0, rel=1e-12)
    u, v = g.standard_normal(40), g.standard_normal(5)
    assert osol.residual_norm_bound(np.outer(u, v)) == pytest.approx(
        np.linalg.norm(u) * np.linalg.norm(v), rel=1e-12)


def test_stop_bound_dominates_true_angle(sbm2000):
    """Davis-Kahan: at every check the stopping quantity is at least the sine
    of the largest principal angle to the true bottom-k subspace."""
    lap, labels, lam, U, full = sbm2000
    k = 10
    V0 = synth.gaussian_block(lap.n, k + 4, 4)
    res = osol.subspace_iteration(lap.L, lambda Q: opoly.apply_terms(lap.L, opoly.limit_exp(8), Q), k, V0,
                                  max_iters=120, tol=0.0, guard=4, Vstar=U)
    # above the float64 floor of the dense reference itself (~1e-14)
    checked = [h for h in res.history if 1e-12 < h["bound"] < 1.0]
    assert len(checked) > 10
    for h in checked:
        assert np.sin(h["angle"]) <= h["bound"] * (1 + 1e-9)


def _path_eigvecs(n, k):
    """Closed-form bottom eigenvectors of the combinatorial Laplacian of the
    path P_n: u_j(x) = cos(pi j (x + 1/2) / n), eigenvalue 2 - 2 cos(pi j / n)."""
    x = np.arange(n)
    U = np.stack([np.cos(np.pi * j * (x + 0.5) / n) for j in range(k)], axis=1)
    return U / np.linalg.norm(U, axis=0), 2 - 2 * np.cos(np.pi * np.arange(k) / n)


@pytest.mark.parametrize("op", ["limit", "plain"])
def test_mu_eigengame_recovers_ordered_eigenvectors(op):
    """On P_12 (all eigenvalues distinct) mu-EG converges to each of the bottom
    four eigenvectors of L individually and in order (the closed forms), for
    the dilated operator and for plain L reversed."""
    n, k = 12, 4
    _, s, d = synth.path_graph(n)
    lap = olap.laplacian(n, s, d, kind=olap.COMBINATORIAL)
    U, lam = _path_eigvecs(n, k)
    np.testing.assert_allclose(lap.L @ U, U * lam, atol=1e-12)
    p = opoly.limit_exp(8) if op == "limit" else opoly.plain(lap.lambda_bound)
    V0 = synth.gaussian_block(n, k, 3)
    V, hist = osol.mu_eigengame(lambda X: opoly.apply_terms(lap.L, p, X), V0, eta=0.5, iters=4000,
                                Vstar=U, record_every=500)
    assert np.all(osol.vector_angles(U, V) < 1e-7)
    assert hist[-1]["streak"] == k
    np.testing.assert_allclose(np.linalg.norm(V, axis=0), 1.0, rtol=1e-14)


def test_mu_eigengame_fixed_point_and_first_player_is_oja():
    """The ordered eigenbasis is a fixed point; player 1 alone follows Oja's
    normalised rule for the top eigenvector, whatever the other players do."""
    n, k = 12, 4
    _, s, d = synth.path_graph(n)
    lap = olap.laplacian(n, s, d, kind=olap.COMBINATORIAL)
    U, _ = _path_eigvecs(n, k)
    p = opoly.limit_exp(8)
    apply_M = lambda X: opoly.apply_terms(lap.L, p, X)
    V1, _ = osol.mu_eigengame(apply_M, U, eta=0.5, iters=1)
    np.testing.assert_allclose(np.abs(np.sum(V1 * U, axis=0)), 1.0, atol=1e-13)
    g = np.random.default_rng(5)
    V0 = g.standard_normal((n, k))
    V2, _ = osol.mu_eigengame(apply_M, V0, eta=0.3, iters=1)
    v = V0[:, 0] / np.linalg.norm(V0[:, 0])
    mv = apply_M(v[:, None])[:, 0]
    w = v + 0.3 * (mv - (v @ mv) * v)
    np.testing.assert_allclose(V2[:, 0], w / np.linalg.norm(w), rtol=1e-12)


@pytest.fixture(scope="module")
def sbm2000():
    n, s, d, labels = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    lap = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    lam, U, full = osol.dense_bottom_k(lap.dense(), 10)
    return lap, labels, lam, U, full


def test_solver_matches_dense_eigh(sbm2000):
    lap, labels, lam, U, full = sbm2000
    k = 10
    p = opoly.limit_exp(8)
    V0 = synth.gaussian_block(lap.n, k + 4, 2)
    res = osol.subspace_iteration(lap.L, lambda Q: opoly.apply_terms(lap.L, p, Q), k, V0,
                                  max_iters=400, tol=1e-10, guard=4, Vstar=U)
    assert res.converged
    assert osol.max_principal_angle(U, res.Q) < 1e-8
    np.testing.assert_allclose(res.evals[1:], lam[1:], rtol=1e-9)
    assert abs(res.evals[0]) < 1e-9


def test_sped_fewer_steps_than_plain(sbm2000):
    """Sec. 5: the dilated operator needs fewer solver steps than the identity
    transform (plain L reversed by eq. reveig)."""
    lap, labels, lam, U, full = sbm2000
    k = 10
    V0 = synth.gaussian_block(lap.n, k + 4, 2)
    steps = {}
    for name, p in (("plain", opoly.plain(2.0)), ("sped", opoly.limit_exp(8))):
        r = osol.subspace_iteration(lap.L, lambda Q, p=p: opoly.apply_terms(lap.L, p, Q), k, V0,
                                    max_iters=2000, tol=1e-8, guard=4)
        assert r.converged
        steps[name] = r.iters
    assert steps["sped"] * 1.5 < steps["plain"]


def test_oja_step_converges(sbm2000):
    lap, labels, lam, U, full = sbm2000
    k = 10
    p = opoly.limit_exp(8)
    V0 = synth.gaussian_block(lap.n, k + 4, 5)
    r = osol.subspace_iteration(lap.L, lambda Q: opoly.apply_terms(lap.L, p, Q), k, V0,
                                max_iters=600, tol=1e-8, guard=4, eta=1.0)
    assert r.converged and osol.max_principal_angle(U, r.Q) < 1e-6


def test_kmeans_recovers_cliques_and_sbm(sbm2000):
    n, s, d, labels = synth.disjoint_cliques(5, 8)
    lap = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    _, U, _ = osol.dense_bottom_k(lap.dense(), 5)
    X = okm.normalize_rows(U)
    C0 = okm.kmeans_pp(X, 5, seed=0)
    lab, C, inertia, it = okm.lloyd(X, C0)
    assert okm.adjusted_rand_index(lab, labels) == pytest.approx(1.0)
    assert inertia < 1e-20
    lap2, labels2, lam, U2, full = sbm2000
    X2 = okm.normalize_rows(U2)
    best = min((okm.lloyd(X2, okm.kmeans_pp(X2, 10, seed=s)) for s in range(4)), key=lambda r: r[2])
    assert okm.adjusted_rand_index(best[0], labels2) > 0.99


def test_ari_textbook_values():
    assert okm.adjusted_rand_index([0, 0, 1, 1], [1, 1, 0, 0]) == pytest.approx(1.0)
    # by hand: contingency [[2,1],[1,2]]: sum C(nij,2) = 2, row sums 2*C(3,2) = 6,
    # column sums 6, C(6,2) = 15 -> (2 - 36/15) / (6 - 36/15) = -1/9
    assert okm.adjusted_rand_index([0, 0, 0, 1, 1, 1], [0, 0, 1, 0, 1, 1]) == pytest.approx(-1 / 9)
    assert list(okm.canonical_labels([3, 3, 1, 2, 1])) == [0, 0, 1, 2, 1]


def test_gradient_finite_differences_and_adjoint():
    n, s, d, _ = synth.sbm_bernoulli([15, 20], 0.4, 0.05, seed=3)
    lap = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    g = np.random.default_rng(0)
    theta = g.standard_normal(6)
    X = g.standard_normal((n, 3))
    G = g.standard_normal((n, 3))
    dtheta, dX = ograd.backward(lap.L, theta, X, G)
    Ld = lap.dense()
    # d theta_j = <G, L^j X> from dense matrix powers
    ref = [np.sum(G * (np.linalg.matrix_power(Ld, j) @ X)) for j in range(6)]
    np.testing.assert_allclose(dtheta, ref, rtol=1e-12, atol=1e-12)
    # loss <G, p(L) X> is linear in theta: central differences are exact up to rounding
    for j in range(6):
        e = np.zeros(6)
        e[j] = 0.5
        fd = (np.sum(G * ograd.forward(lap.L, theta + e, X)) - np.sum(G * ograd.forward(lap.L, theta - e, X)))
        assert fd == pytest.approx(dtheta[j], rel=1e-10, abs=1e-10)
    # adjoint: <G, p(L) X> = <p(L) G, X>
    assert np.sum(G * ograd.forward(lap.L, theta, X)) == pytest.approx(np.sum(dX * X), rel=1e-12)
    # dX by finite differences of a nonlinear loss sum(p(L)X)^2/2 in one entry
    Y = ograd.forward(lap.L, theta, X)
    _, dX2 = ograd.backward(lap.L, theta, X, Y)
    h = 1e-6
    Xp, Xm = X.copy(), X.copy()
    Xp[4, 1] += h
    Xm[4, 1] -= h
    fd = (0.5 * np.sum(ograd.forward(lap.L, theta, Xp) ** 2) - 0.5 * np.sum(ograd.forward(lap.L, theta, Xm) ** 2)) / (2 * h)
    assert fd == pytest.approx(dX2[4, 1], rel=1e-6)


def test_limit_degree_must_cover_the_spectrum_on_cliques():
    """Sec. 5 (cliques) and App. A (series accuracy): the limit approximation
    (I - L/l)^l of the combinatorial Laplacian reverses the spectrum only when
    it is accurate up to lambda_max, i.e. 2 l > lambda_max (else |1 - lambda/l|^l
    blows up at the top of the spectrum and the iteration locks onto the top
    eigenvectors of L).  200 nodes in 4 cliques (lambda_max = 54.2): l = 11, 21,
    25 end on a wrong subspace, l = 31, 51 reach the bottom-4 subspace in a few
    iterations, far fewer than plain L reversed."""
    N, s, d, _ = synth.cliques_short_circuit(200, 4, seed=1)
    lap = olap.laplacian(N, s, d, kind=olap.COMBINATORIAL)
    lam, U, full = osol.dense_bottom_k(lap.dense(), 4)
    assert full[-1] == pytest.approx(54.16, abs=0.01)
    V0 = synth.gaussian_block(N, 6, 2)
    plain = osol.subspace_iteration(lap.L, lambda X: opoly.apply_terms(lap.L, opoly.plain(lap.lambda_bound), X), 4,
                                    V0, max_iters=300, tol=1e-8, guard=2)
    assert plain.converged and osol.max_principal_angle(U, plain.Q) < 1e-6
    for ell in (11, 21, 25, 31, 51):
        with np.errstate(all="ignore"):
            r = osol.subspace_iteration(lap.L, lambda X, l=ell: opoly.apply_limit_product(lap.L, l, X), 4, V0,
                                        max_iters=300, tol=1e-8, guard=2)
        ang = osol.max_principal_angle(U, r.Q)
        if 2 * ell > full[-1]:
            assert r.converged and ang < 1e-6 and r.iters * 5 < plain.iters
        else:
            assert ang > 1.0
