"""Parity at the full sizes of the stated workloads (MI355X; marked gpu).

* Chung-Lu power-law graph, 4e6 nodes, exponent 2.1, mean degree 16, 256
  planted communities, largest component: the device build against the oracle
  (component, relabelling, rows) and the degree-16 limit polynomial on a bf16
  block against the oracle's float64 chain (4 columns).
* SBM, 5e5 nodes, 50 blocks, mean degree 24: PolyApply (degree 12, k = 50)
  forward, X gradient and coefficient gradient against the float64 oracle.
* R-MAT scale 26 (67M nodes, edge factor 16, a = 0.57, b = c = 0.19,
  symmetrised, repeats and self-loops removed): one fused step on a 64-column
  bf16 block checked row by row on 2,000 sampled rows, whose exact values the
  oracle computes straight from the edge list.
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
    rows = np.unique(np.concatenate([rng.choice(n, 1990, replace=False),
                                     np.arange(10)]))
    src_h = src.cpu().numpy()
    dst_h = dst.cpu().numpy()
    del src, dst
    gc.collect()

    def xrows(ids):
        t = torch.as_tensor(np.asarray(ids, dtype=np.int64), device="cuda")
        return X.index_select(0, t).float().cpu().numpy().astype(np.float64)

    want = olap.rows_times_block(n, src_h, dst_h, None, olap.SYM_NORMALIZED, rows, xrows)
    got = Y.index_select(0, torch.as_tensor(rows, device="cuda")).cpu().numpy().astype(np.float64)
    scale = np.abs(want).max(axis=1, keepdims=True) + 1e-30
    # one fused step: each output is one float32 sum of d products of float32 values
    assert (np.abs(got - want) / scale).max() < 1e-5
    del deg_host
