"""The 3-room grid experiment (Sec. 5, proto-value functions, s = 2, h = 10)
with the exact rows of Table 2, on the oracle.

The paper reports that the series forms of -e^{-L} cut the solver's steps by
about an order of magnitude against the identity transform, and the exact
matrix log by over two orders.  The exact transforms need the full
eigendecomposition, which the method exists to avoid, so they run only here,
through the oracle's dense spectral transform (`apply_spectral`), with the
same block subspace iteration, start block and stopping rule as the series
and identity arms.  The qualitative claim is what is checked: the figures
that hold the paper's step counts are not in its text.
"""
import numpy as np
import pytest

from oracle import laplacian as olap
from oracle import poly as opoly
from oracle import solver as osol
from paper_2207_14589_amd import synth

CHECKPOINTS = [10, 40, 160, 640, 2560, 10240]


@pytest.fixture(scope="module")
def grid():
    N, s, d = synth.three_room_grid(2, 10)
    lap = olap.laplacian(N, s, d, kind=olap.COMBINATORIAL)
    lam, U = np.linalg.eigh(lap.dense())
    return lap, lam, U


def _iters_to_target(lap, apply_M, Uk, V0, target=1e-8):
    """First checkpoint at which the paper's subspace error
    1 - ||U*^T Q||_F^2 / k of the first k Ritz vectors is below target."""
    k = Uk.shape[1]
    Q = osol.orthonormal(V0)
    t = 0
    for T in CHECKPOINTS:
        while t < T:
            Q = osol.orthonormal(apply_M(Q))
            t += 1
        _, Qr, _ = osol.rayleigh_ritz(lap.L, Q)
        if osol.subspace_error(Uk, Qr[:, :k]) < target:
            return T
    return None


def test_exact_log_and_series_cut_steps(grid):
    lap, lam, U = grid
    k = 3
    Uk = U[:, :k]
    V0 = synth.gaussian_block(lap.n, k + 2, 2)
    lb, eps = lap.lambda_bound, 1e-3

    def spectral(f, lam_star):
        diag = lam_star - f(lam)  # eq. reveig: M = lambda* I - f(L)
        return lambda Q: U @ (diag[:, None] * (U.T @ Q))

    arms = {
        "identity": lambda Q: lb * Q - lap.L @ Q,
        "limit251": spectral(lambda x: -opoly.limit_exp(251)(x), 0.0),
        "taylor_exp251": spectral(lambda x: -opoly.taylor_exp(251)(x), 0.0),
        "exact_negexp": spectral(opoly.exact_negexp(), 0.0),
        "exact_log": spectral(opoly.exact_log(eps), float(opoly.exact_log(eps)(lb))),
    }
    steps = {name: _iters_to_target(lap, f, Uk, V0) for name, f in arms.items()}
    print(steps)
    assert steps["exact_log"] is not None and steps["identity"] is not None
    # series forms: about an order of magnitude; exact log: over two orders
    for name in ("limit251", "taylor_exp251", "exact_negexp"):
        assert steps[name] is not None and 8 <= steps["identity"] / steps[name] <= 64
    assert steps["identity"] / steps["exact_log"] >= 100
    # the series forms are within float64 rounding of the exact -e^{-L} on [0, 8]
    assert steps["limit251"] == steps["taylor_exp251"] == steps["exact_negexp"]


def test_exact_log_gap_dilation(grid):
    """Why: the log maps the three room modes near 0 far apart
    (log(eps) ... log(3e-3)) while the identity keeps their gaps at about
    1e-3 on a spectrum of width 8."""
    _, lam, _ = grid
    f = opoly.exact_log(1e-3)
    rel_identity = (lam[3] - lam[2]) / lam[-1]
    rel_log = (f(lam[3]) - f(lam[2])) / (f(lam[-1]) - f(lam[0]))
    assert rel_log > 10 * rel_identity
