"""Pins of the oracle's Table 2 transforms and exact p(L)V."""
from math import factorial

import numpy as np
import pytest

from oracle import laplacian as olap
from oracle import poly as opoly
from paper_2207_14589_amd import synth


LAM = np.linspace(0.0, 2.0, 2001)


@pytest.mark.parametrize("ell", [1, 2, 8, 12, 16, 51])
def test_limit_binomial(ell):
    """Coefficients C(l,i)(-1/l)^i reproduce (1 - lam/l)^l (binomial theorem)."""
    p = opoly.limit_exp(ell)
    np.testing.assert_allclose(p(LAM), (1.0 - LAM / ell) ** ell, rtol=1e-12, atol=1e-13)
    assert p(0.0) == pytest.approx(1.0)             # spectral radius 1 at lambda* = 0


@pytest.mark.parametrize("ell", [3, 8, 15, 16])
def test_taylor_exp_remainder(ell):
    """|p(lam) - exp(-lam)| <= lam^(l+1)/(l+1)!  (Lagrange remainder)."""
    p = opoly.taylor_exp(ell)
    err = np.abs(p(LAM) - np.exp(-LAM))
    assert np.all(err <= LAM ** (ell + 1) / factorial(ell + 1) + 1e-15)


@pytest.mark.parametrize("ell", [5, 11, 31])
def test_taylor_log_series(ell):
    """f = sum (-1)^(i+1) y^i / i approximates log(lam + eps) for |y| < 1 within
    the tail bound sum_{i>l} |y|^i/i <= |y|^(l+1)/((l+1)(1-|y|)); M = f(2) - f."""
    eps = 1e-3
    p = opoly.taylor_log(ell, 2.0, eps)
    lam = np.linspace(0.1, 1.9, 181)
    y = lam + eps - 1.0
    assert abs(p(2.0)) < 1e-12      # M(lambda_bound) = f(lambda_bound) - f(lambda_bound)
    f = p.coeffs[0] - p(lam)        # c_0 = f(lambda_bound), so f(lam) = c_0 - M(lam)
    np.testing.assert_array_less(np.abs(f - np.log(lam + eps)), np.abs(y) ** (ell + 1) / ((ell + 1) * (1 - np.abs(y))) + 1e-14)


@pytest.mark.parametrize("maker", [lambda l: opoly.limit_exp(l), lambda l: opoly.taylor_exp(l),
                                   lambda l: opoly.taylor_log(l, 2.0)])
@pytest.mark.parametrize("ell", [5, 9, 15])
def test_odd_degree_monotone(maker, ell):
    """Sec. 4.1: f increasing keeps the eigenvector order, so M = lam* - f is
    strictly decreasing on [0, lambda_bound] for odd l (Table 2: l odd)."""
    p = maker(ell)
    assert np.all(np.diff(p(LAM)) < 0)


def test_even_log_not_monotone():
    p = opoly.taylor_log(8, 2.0)
    assert not np.all(np.diff(p(LAM)) < 0)


def test_plain_and_shift_expansion():
    p = opoly.plain(2.0)
    np.testing.assert_allclose(p(LAM), 2.0 - LAM)
    q = opoly.taylor_log(7, 2.0)
    c = opoly.monomial_in_L(q)
    lam = np.linspace(0, 2, 17)
    np.testing.assert_allclose(np.polynomial.polynomial.polyval(lam, c), q(lam), rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("kind", [olap.COMBINATORIAL, olap.SYM_NORMALIZED])
def test_path_eigenpairs(kind):
    """p(L) v = p(lambda) v on the closed-form eigenvectors of the path graph:
    combinatorial v_j(x) = cos(pi j (x + 1/2)/n); normalised D^1/2 of the
    Chebyshev nodes' vector u_j(x) = cos(pi j x/(n-1))."""
    n = 40
    _, s, d = synth.path_graph(n)
    lap = olap.laplacian(n, s, d, kind=kind)
    x = np.arange(n)
    V, lam = [], []
    for j in range(0, n, 7):
        if kind == olap.COMBINATORIAL:
            V.append(np.cos(np.pi * j * (x + 0.5) / n))
            lam.append(2 - 2 * np.cos(np.pi * j / n))
        else:
            V.append(np.sqrt(lap.degree) * np.cos(np.pi * j * x / (n - 1)))
            lam.append(1 - np.cos(np.pi * j / (n - 1)))
    V = np.stack(V, 1)
    lam = np.array(lam)
    p = opoly.limit_exp(16) if kind == olap.SYM_NORMALIZED else opoly.taylor_exp(9)
    Y = opoly.apply_terms(lap.L, p, V)
    np.testing.assert_allclose(Y, V * p(lam), atol=1e-11 * np.abs(V).max())


def test_terms_vs_spectral_and_product():
    n, s, d, _ = synth.sbm_bernoulli([20, 25], 0.4, 0.05, seed=11)
    lap = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    V = synth.gaussian_block(n, 6, seed=2)
    for p in (opoly.limit_exp(16), opoly.taylor_exp(12), opoly.taylor_log(9, 2.0), opoly.plain(2.0)):
        Y = opoly.apply_terms(lap.L, p, V)
        Z = opoly.apply_spectral(lap.dense(), p, V)
        np.testing.assert_allclose(Y, Z, atol=1e-11)
    np.testing.assert_allclose(opoly.apply_limit_product(lap.L, 16, V),
                               opoly.apply_terms(lap.L, opoly.limit_exp(16), V), atol=1e-12)


def test_reversal_maps_bottom_k_to_top_k():
    """eq. (reveig): the top-k eigenvectors of M span the bottom-k of L."""
    n, s, d, _ = synth.sbm_bernoulli([15, 15, 15], 0.5, 0.02, seed=4)
    lap = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    Ld = lap.dense()
    lam, U = np.linalg.eigh(Ld)
    k = 3
    for p in (opoly.limit_exp(15), opoly.plain(2.0)):
        M = opoly.apply_terms(lap.L, p, np.eye(n))
        mu, W = np.linalg.eigh(0.5 * (M + M.T))
        top = W[:, -k:]
        assert np.linalg.norm(top - U[:, :k] @ (U[:, :k].T @ top), 2) < 1e-8


# ----------------------------------------------------------- exact transforms (Table 2 rows 1 and 3)
def _closed_form_pairs(kind, n=40):
    """Closed-form eigenpairs of the path and cycle graphs (orthonormal columns)."""
    out = []
    x = np.arange(n)
    _, s, d = synth.path_graph(n)
    lap = olap.laplacian(n, s, d, kind=kind)
    V, lam = [], []
    for j in range(0, n, 5):
        if kind == olap.COMBINATORIAL:
            V.append(np.cos(np.pi * j * (x + 0.5) / n))
            lam.append(2 - 2 * np.cos(np.pi * j / n))
        else:
            V.append(np.sqrt(lap.degree) * np.cos(np.pi * j * x / (n - 1)))
            lam.append(1 - np.cos(np.pi * j / (n - 1)))
    out.append((lap, np.stack(V, 1), np.array(lam)))
    _, s, d = synth.cycle_graph(n)
    lap = olap.laplacian(n, s, d, kind=kind)
    V, lam = [], []
    for j in range(0, n // 2 + 1, 3):  # cos(2 pi j x / n), eigenvalue 2 - 2 cos(2 pi j / n) (halved if normalised)
        V.append(np.cos(2 * np.pi * j * x / n))
        mu = 2 - 2 * np.cos(2 * np.pi * j / n)
        lam.append(mu if kind == olap.COMBINATORIAL else mu / 2)
    out.append((lap, np.stack(V, 1), np.array(lam)))
    return out


@pytest.mark.parametrize("kind", [olap.COMBINATORIAL, olap.SYM_NORMALIZED])
def test_exact_transforms_on_closed_form_spectra(kind):
    """Table 2 rows 1 and 3 applied through the eigendecomposition act on the
    closed-form eigenvectors of the path and cycle graphs as f(lambda):
    log(L + eps) v = log(lambda + eps) v and -exp(-L) v = -exp(-lambda) v.
    The cycle's eigenvalues are double, so this also checks that a repeated
    eigenvalue's whole eigenspace gets the same factor."""
    eps = 1e-3
    for lap, V, lam in _closed_form_pairs(kind):
        Ld = lap.dense()
        np.testing.assert_allclose(Ld @ V, V * lam, atol=1e-12 * max(1.0, np.abs(V).max()))
        Y = opoly.apply_spectral(Ld, opoly.exact_log(eps), V)
        np.testing.assert_allclose(Y, V * np.log(lam + eps), atol=1e-11 * np.abs(V).max())
        Y = opoly.apply_spectral(Ld, opoly.exact_negexp(), V)
        np.testing.assert_allclose(Y, -V * np.exp(-lam), atol=1e-12 * np.abs(V).max())


def test_exact_transforms_match_matrix_functions():
    """The same transforms against scipy's matrix exponential (scaling and
    squaring with Pade approximants) and matrix logarithm (inverse scaling and
    squaring), which never form an eigendecomposition: -exp(-L) = -expm(-L),
    log(L + eps I) = logm(L + eps I)."""
    from scipy.linalg import expm, logm

    n, s, d, _ = synth.sbm_bernoulli([12, 15, 9], 0.5, 0.05, seed=21)
    for kind in (olap.SYM_NORMALIZED, olap.COMBINATORIAL):
        Ld = olap.laplacian(n, s, d, kind=kind).dense()
        V = synth.gaussian_block(n, 4, seed=5)
        np.testing.assert_allclose(opoly.apply_spectral(Ld, opoly.exact_negexp(), V), -expm(-Ld) @ V,
                                   atol=1e-12 * np.abs(V).max())
        eps = 1e-3
        Lg = np.real(logm(Ld + eps * np.eye(n)))
        np.testing.assert_allclose(opoly.apply_spectral(Ld, opoly.exact_log(eps), V), Lg @ V,
                                   atol=1e-9 * np.abs(Lg @ V).max())


def test_series_forms_converge_to_exact_negexp():
    """Table 2's series rows approximate row 3: the degree-30 Taylor series of
    exp(-lam) is within its Lagrange remainder of the exact transform on [0, 2],
    and the limit form (1 - lam/l)^l approaches exp(-lam) from below with
    0 <= exp(-lam) - (1 - lam/l)^l <= lam^2 exp(-lam) / (2 (l - lam)) for lam < l."""
    f = opoly.exact_negexp()
    assert np.abs(opoly.taylor_exp(30)(LAM) + f(LAM)).max() <= 2.0 ** 31 / factorial(31) + 1e-15
    for ell in (16, 64, 251):
        gap = -f(LAM) - opoly.limit_exp(ell)(LAM)
        assert gap.min() >= -1e-15
        assert np.all(gap <= LAM ** 2 * np.exp(-LAM) / (2 * (ell - LAM)) + 1e-15)


def test_exact_transforms_reverse_the_spectrum():
    """Sec. 4.1: both exact transforms are increasing, so the reversed
    operators lambda* - f(L) (lambda* = f(lambda_bound) for the log, 0 for
    -exp(-L)) are decreasing, nonnegative on [0, lambda_bound], and keep the
    bottom-k eigenvectors on top."""
    lam = np.linspace(0.0, 2.0, 2001)
    for f, lam_star in ((opoly.exact_log(1e-3), opoly.exact_log(1e-3)(2.0)), (opoly.exact_negexp(), 0.0)):
        M = lam_star - f(lam)
        assert np.all(np.diff(M) < 0) and M.min() >= -1e-15
    # the log dilates the bottom of the spectrum: ratio of M's gaps near 0 vs near 2
    g = opoly.exact_log(1e-3)
    assert (g(0.02) - g(0.01)) / (g(1.99) - g(1.98)) > 50
