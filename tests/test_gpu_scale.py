"""Parity at the full sizes of the stated workloads (MI355X; marked gpu).

* Chung-Lu power-law graph, 4e6 nodes, exponent 2.1, mean degree 16, 256
  planted communities, largest component: the device build against the oracle
  (component, relabelling, rows) and the degree-16 limit polynomial on a bf16
  block against the oracle's float64 chain (4 columns).
* SBM, 5e5 nodes, 50 blocks, mean degree 24: PolyApply (degree 12, k = 50)
  forward, X gradient and coefficient gradient against the float64 oracle.
* R-MAT scale 26 (67M nodes, edge factor 16, a = 0.57, b = c = 0.19,
  symmetrised, repeats and self-loops removed): one fused step on a 64-column
  bf16 block checked row by row on 2,000 sampled rows and the 16 largest hubs
  (heavy rows of up to about 10^6 entries, cut into pieces), whose exact values
  the oracle computes straight from the edge list.
* Chung-Lu power-law graph at a tenth of the size (4e5 nodes, the same
  exponent, mean degree and 256 communities, so the 64 wanted vectors are
  still fewer than the communities): three solver iterations of the
  degree-16 limit polynomial on 64 + 8 columns from one start block.  The
  span of M^3 V0 (the library's chain and Cholesky-QR) against the oracle's,
  and the solver's Ritz values after 3 iterations (float32 and bf16 storage)
  against the oracle's subspace iteration.
* R-MAT scale 20 (same parameters, largest component): the importance edge
  walk and the lazy node walk (8 walks per row, degree 16) against the
  oracle's walks on sampled rows that include the 8 largest hubs.
* R-MAT scale 22 (same parameters, largest component): the degree-16 limit
  chain on a 72-column float32 block (the solver's 64 + 8 columns), every row
  of 4 columns against the oracle's float64 chain; hubs of up to about
  1.6 * 10^5 entries go through the heavy pieces.
"""
import gc

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import grad as ograd
from oracle import laplacian as olap
from oracle import poly as opoly
from paper_2207_14589_amd import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sped():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2207_14589_amd import sped as s
    s.lib()
    return s


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_chung_lu_4m_lcc_and_poly(sped):
    _say("Chung-Lu 4e6 nodes, largest component, bf16 block, degree-16 limit polynomial")
    n, s, d, comm = synth.chung_lu(4_000_000, 2.1, 16.0, 256, 0.95, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym", lcc=True)
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED, lcc=True)
    assert L.n == ref.n
    np.testing.assert_array_equal(L.old_of_new.cpu().numpy(), ref.old_of_new)
    assert L.nnz == ref.L.nnz - np.count_nonzero(ref.L.diagonal())
    assert L.max_degree == int(ref.count_degree.max())
    _say(f"  n_lcc={L.n} nnz={L.nnz} max_degree={L.max_degree} medium={L.n_medium} heavy={L.n_heavy}")
    X = synth.gaussian_block_device(L.n, 64, seed=2, dtype=torch.bfloat16)
    Y = sped.apply_poly(L, sped.transform("limit", 16), X, out_dtype=torch.float32)
    cols = [0, 17, 40, 63]
    Xc = X[:, cols].float().cpu().numpy().astype(np.float64)
    Yr = opoly.apply_limit_product(ref.L, 16, Xc)
    Yg = Y[:, cols].cpu().numpy().astype(np.float64)
    assert _rel(Yg, Yr) < 3e-5
    assert np.abs(Yg - Yr).max() < 2e-4 * np.abs(Yr).max()


def test_sbm_500k_polyapply_gradients(sped):
    _say("SBM 5e5 nodes, 50 blocks, degree 24: PolyApply degree 12, k=50")
    from paper_2207_14589_amd.autograd import poly_apply
    n, s, d, _ = synth.sbm_from_degrees(500_000, 50, 22.8, 1.2, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    g = np.random.default_rng(4)
    theta0 = opoly.limit_exp(12).coeffs + 0.01 * g.standard_normal(13)
    X0 = synth.gaussian_block(n, 50, 2).astype(np.float32)
    G0 = synth.gaussian_block(n, 50, 3).astype(np.float32)
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    X = torch.from_numpy(X0).cuda().requires_grad_(True)
    Y = poly_apply(theta, X, L)
    (Y * torch.from_numpy(G0).cuda()).sum().backward()
    Yr = ograd.forward(ref.L, theta0, X0.astype(np.float64))
    dth_r, dX_r = ograd.backward(ref.L, theta0, X0.astype(np.float64), G0.astype(np.float64))
    assert _rel(Y.detach().cpu().numpy(), Yr) < 3e-5
    assert _rel(X.grad.cpu().numpy(), dX_r) < 3e-5
    np.testing.assert_allclose(theta.grad.numpy(), dth_r, rtol=2e-5, atol=2e-5 * np.abs(dth_r).max())


def _threaded(apply, workers=16):
    """Apply a column-separable oracle operator on column slices in threads
    (scipy's sparse products release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    def run(V):
        sl = np.array_split(np.arange(V.shape[1]), min(workers, V.shape[1]))
        with ThreadPoolExecutor(len(sl)) as ex:
            parts = list(ex.map(lambda c: apply(np.ascontiguousarray(V[:, c])), sl))
        return np.concatenate(parts, axis=1)
    return run


def test_power_law_trajectory_parity_k64(sped):
    _say("Chung-Lu 4e5, 256 communities, k=64+8, 3 iterations of the degree-16 limit operator vs the oracle")
    from oracle import solver as osol
    n, s, d, _ = synth.chung_lu(400_000, 2.1, 16.0, 256, 0.95, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym", lcc=True, walk_records=False)
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED, lcc=True)
    assert L.n == ref.n
    k, guard, ell, T = 64, 8, 16, 3
    V0n = synth.gaussian_block(L.n, k + guard, 2).astype(np.float32)
    apply_M = _threaded(lambda V: opoly.apply_limit_product(ref.L, ell, V))
    # the iteration core: span(M^3 V0) from the chain and Cholesky QR2
    p = sped.transform("limit", ell)
    Q = torch.from_numpy(V0n).cuda()
    W = torch.empty_like(Q)
    for _ in range(T):
        sped.apply_poly(L, p, Q, out=W)
        sped.orthonormalize(W, passes=2)
        Q, W = W, Q
    Wo = V0n.astype(np.float64)
    for _ in range(T):
        Wo = osol.orthonormal(apply_M(Wo))
    ang = osol.max_principal_angle(Wo, Q.cpu().numpy().astype(np.float64))
    _say(f"  span of M^3 V0: largest angle {ang:.2e}")
    assert ang < 1e-5
    # the solver: Ritz values of L on span(M^3 V0) (Rayleigh-Ritz rotates the
    # basis but keeps the span), float32 and bf16 storage
    theta = osol.rayleigh_ritz(ref.L, Wo)[0][:k]
    V0 = torch.from_numpy(V0n).cuda()
    r32 = sped.bottomk(L, k, p, V0=V0, guard=guard, tol=0.0, max_iters=T)
    np.testing.assert_allclose(r32.evals, theta, rtol=1e-5, atol=1e-6)
    r16 = sped.bottomk(L, k, p, V0=V0, guard=guard, tol=0.0, max_iters=T, storage="bf16")
    assert r16.stats["coarse_iters"] == T
    # bf16 storage (u = 2^-9) perturbs the iterate, and so the Ritz values
    np.testing.assert_allclose(r16.evals, theta, rtol=0, atol=3e-3)
    _say(f"  Ritz values: float32 max err {np.abs(r32.evals - theta).max():.2e}, "
         f"bf16 {np.abs(r16.evals - theta).max():.2e}")


def test_rmat_scale26_sampled_rows(sped):
    _say("R-MAT scale 26 on the device: build, one fused step on a 64-column bf16 block")
    n, src, dst = synth.rmat_device(26, 16, 0.57, 0.19, 0.19, seed=1)
    m = src.numel()
    _say(f"  n={n} edges={m}")
    L = sped.Laplacian(n, src, dst, kind="sym", walk_records=False)  # exact path only: no walk records
    assert L.nnz == 2 * m
    torch.cuda.empty_cache()
    X = synth.gaussian_block_device(n, 64, seed=2, dtype=torch.bfloat16)
    Y = sped.apply_poly(L, sped.monomial([0.0, 1.0]), X, out_dtype=torch.float32)
    rng = np.random.default_rng(0)
    deg_host = None
    src_h = src.cpu().numpy()
    dst_h = dst.cpu().numpy()
    del src, dst
    gc.collect()
    deg = np.bincount(src_h, minlength=n) + np.bincount(dst_h, minlength=n)
    hubs = np.argsort(deg)[-16:]
    _say(f"  largest degrees {np.sort(deg[hubs])[::-1][:4].tolist()}, heavy rows {L.n_heavy}")
    assert deg[hubs].min() > 8192  # the hubs are heavy rows
    rows = np.unique(np.concatenate([rng.choice(n, 1990, replace=False), np.arange(10), hubs]))
    del deg

    def xrows(ids):
        t = torch.as_tensor(np.asarray(ids, dtype=np.int64), device="cuda")
        return X.index_select(0, t).float().cpu().numpy().astype(np.float64)

    want = olap.rows_times_block(n, src_h, dst_h, None, olap.SYM_NORMALIZED, rows, xrows)
    got = Y.index_select(0, torch.as_tensor(rows, device="cuda")).cpu().numpy().astype(np.float64)
    scale = np.abs(want).max(axis=1, keepdims=True) + 1e-30
    # one fused step: each output is one float32 sum of d products of float32 values
    assert (np.abs(got - want) / scale).max() < 1e-5
    del deg_host


def test_rmat_scale22_chain_with_heavy_pieces(sped):
    _say("R-MAT scale 22, largest component, degree-16 limit chain on 72 float32 columns")
    n, src, dst = synth.rmat_device(22, 16, 0.57, 0.19, 0.19, seed=1)
    src_h, dst_h = src.cpu().numpy(), dst.cpu().numpy()
    L = sped.Laplacian(n, src, dst, kind="sym", lcc=True, walk_records=False)
    del src, dst
    ref = olap.laplacian(n, src_h, dst_h, kind=olap.SYM_NORMALIZED, lcc=True)
    assert L.n == ref.n and L.max_degree == int(ref.count_degree.max())
    _say(f"  n_lcc={L.n} nnz={L.nnz} max_degree={L.max_degree} medium={L.n_medium} heavy={L.n_heavy}")
    assert L.n_heavy >= 10 and L.max_degree > 8 * 8192  # hubs cut into many pieces
    X = synth.gaussian_block_device(L.n, 72, seed=2, dtype=torch.float32)
    Y = sped.apply_poly(L, sped.transform("limit", 16), X)
    cols = [0, 17, 40, 71]
    Yr = opoly.apply_limit_product(ref.L, 16, X[:, cols].cpu().numpy().astype(np.float64))
    Yg = Y[:, cols].cpu().numpy().astype(np.float64)
    assert _rel(Yg, Yr) < 3e-5
    assert np.abs(Yg - Yr).max() < 2e-4 * np.abs(Yr).max()
    # the heavy rows themselves, elementwise
    hr = L.bins[L.n_medium:L.n_medium + L.n_heavy].long().cpu().numpy()
    assert np.abs(Yg[hr] - Yr[hr]).max() < 2e-4 * np.abs(Yr).max()


def test_rmat_scale20_walks_on_hub_rows(sped):
    _say("R-MAT scale 20, largest component: edge walks and lazy walks on sampled rows and the hubs")
    from oracle import lazywalk as olazy
    from oracle import walk as owalk
    n, src, dst = synth.rmat_device(20, 16, 0.57, 0.19, 0.19, seed=3)
    src_h, dst_h = src.cpu().numpy(), dst.cpu().numpy()
    L = sped.Laplacian(n, src, dst, kind="sym", lcc=True)
    del src, dst
    ref = olap.laplacian(n, src_h, dst_h, kind=olap.SYM_NORMALIZED, lcc=True)
    assert L.n == ref.n
    deg = ref.count_degree
    hubs = np.argsort(deg)[-8:]
    med = np.nonzero((deg > 128) & (deg <= 8192))[0][:8]
    rows = np.unique(np.concatenate([np.random.default_rng(1).choice(L.n, 300, replace=False), hubs, med]))
    _say(f"  n_lcc={L.n} nnz={L.nnz} hub degrees {np.sort(deg[hubs])[::-1][:3].tolist()}")
    X = synth.gaussian_block(L.n, 8, 4).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    c = opoly.limit_exp(16).coeffs
    Y = sped.apply_poly_stochastic(L, c, Xd, walks=8, seed=3, counter=1).cpu().numpy()
    Yr = owalk.estimate_importance(ref, c, X.astype(np.float64), 8, seed=3, counter=1, rows=rows)
    scale = np.abs(Yr).max(axis=1, keepdims=True) + 1.0
    assert (np.abs(Y[rows] - Yr) / scale).max() < 1e-4
    Yl = sped.apply_limit_lazy(L, 16, Xd, 8, seed=3).cpu().numpy()
    Ylo = olazy.estimate_lazy(ref, 16, X.astype(np.float64), 8, seed=3, rows=rows)
    assert np.abs(Yl[rows] - Ylo).max() <= 2e-6 * np.abs(Ylo).max()


def test_rmat_scale18_locality_orders(sped):
    """The node orders on an R-MAT scale-18 largest component (hubs of
    thousands of neighbours, ~10 search levels, label runs of every length)
    equal the oracle's exactly (label propagation against its numpy-counting
    form); the ordered build numbers its rows in that order."""
    from oracle import order as oorder
    _say("R-MAT scale 18, largest component: Cuthill-McKee, degree and label-propagation orders, ordered build")
    n, src, dst = synth.rmat_device(18, 16, 0.57, 0.19, 0.19, seed=5)
    src_h, dst_h = src.cpu().numpy(), dst.cpu().numpy()
    L = sped.Laplacian(n, src, dst, kind="sym", lcc=True, walk_records=False)
    ref = olap.laplacian(n, src_h, dst_h, kind=olap.SYM_NORMALIZED, lcc=True)
    rowptr, col, _ = ref.adjacency()
    assert L.n == ref.n
    _say(f"  n_lcc={L.n} nnz={L.nnz} max_degree={L.max_degree}")
    for method, want in (("cuthill_mckee", oorder.cuthill_mckee(ref.n, rowptr, col)),
                         ("degree", oorder.degree_order(ref.n, rowptr)),
                         ("label_propagation", oorder.label_order(ref.n, rowptr, col, fast=True))):
        _say(f"  {method}")
        got = sped.locality_order(L, method).cpu().numpy()
        np.testing.assert_array_equal(got, want)
        Lo = sped.Laplacian(n, src, dst, kind="sym", lcc=True, walk_records=False, order=method)
        placed = np.argsort(want)  # the node at each position
        np.testing.assert_array_equal(Lo.old_of_new.cpu().numpy(), ref.old_of_new[placed])
        np.testing.assert_array_equal(np.diff(Lo.rowptr[: Lo.n + 1].cpu().numpy()), np.diff(rowptr)[placed])
        del Lo
