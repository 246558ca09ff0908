"""GPU parity: every libsped entry point against the FP64 oracle on the same
seeded inputs (run on an MI355X; marked gpu).

Tolerances (float32 storage and accumulation, unit roundoff u = 2^-24):
* Laplacian values: each entry is one float64 product rounded once to float32,
  so |rel err| <= u; we allow 2u.
* p(L)X, degree l: every fused step rounds once per output and accumulates
  d_i float32 products; the polynomial's coefficient mass sum |c_i| ||L||^i
  (<= 7.4 for the Table 2 rows on [0, 2]) amplifies it, so the relative
  Frobenius error stays below l * 8 * 4u ~ 3e-5 for l = 16; we check 3e-5
  relative Frobenius and 2e-4 relative to the max entry elementwise.
* Gram in float64 of float32 data: products are exact, sums float64: 1e-13.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import grad as ograd
from oracle import kmeans as okm
from oracle import laplacian as olap
from oracle import poly as opoly
from oracle import solver as osol
from oracle import walk as owalk
from paper_2207_14589_amd import synth

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sped():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2207_14589_amd import sped as s
    s.lib()
    return s


def mixed_degree_graph(seed=5):
    """SBM rows plus a hub of degree 9000 (heavy bin) and hubs of degree 300
    (medium bin), weighted, with repeated edges and self-loops."""
    n, s, d, _ = synth.sbm_bernoulli([700, 900, 1400], 0.01, 0.0008, seed=seed)
    n = 12000
    g = np.random.default_rng(seed)
    hub_s = np.zeros(9000, dtype=np.int64)
    hub_d = g.choice(np.arange(1, n), 9000, replace=False)
    med_s = np.repeat([17, 1200], 300)
    med_d = g.integers(3000, n, 600)
    extra_s = g.integers(3000, n, 20000)
    extra_d = g.integers(3000, n, 20000)
    src = np.concatenate([s, hub_s, med_s, extra_s, [5, 5, 8]])
    dst = np.concatenate([d, hub_d, med_d, extra_d, [5, 9, 9]])
    w = synth.random_weights(src.shape[0], seed + 1).astype(np.float32).astype(np.float64)
    return n, src, dst, w


def dense_from_gpu(L):
    rowptr, col, val, diag, scale = L.host_csr()
    import scipy.sparse as sp
    n = L.n
    S = sp.csr_matrix((val.astype(np.float64), col, rowptr), shape=(n, n))
    return sp.diags(diag.astype(np.float64)) - S


@pytest.mark.parametrize("kind", ["sym", "combinatorial"])
@pytest.mark.parametrize("lcc", [False, True])
def test_laplacian_build(sped, kind, lcc):
    n, src, dst, w = mixed_degree_graph()
    # add a separate small component so that lcc matters
    src = np.concatenate([src, [n - 3, n - 2]])
    dst = np.concatenate([dst, [n - 2, n - 1]])
    w = np.concatenate([w, [0.5, 0.25]])
    _say(f"laplacian kind={kind} lcc={lcc} n={n} m={src.shape[0]}")
    L = sped.Laplacian(n, src, dst, w, kind=kind, lcc=lcc)
    ref = olap.laplacian(n, src, dst, w, kind=olap.SYM_NORMALIZED if kind == "sym" else olap.COMBINATORIAL, lcc=lcc)
    assert L.n == ref.n
    rowptr, col, val, diag, scale = L.host_csr()
    r_rowptr, r_col, r_w = ref.adjacency()
    np.testing.assert_array_equal(rowptr, r_rowptr)
    np.testing.assert_array_equal(col, r_col)
    np.testing.assert_array_equal(L.old_of_new.cpu().numpy(), ref.old_of_new)
    Lg = dense_from_gpu(L).tocsr()
    diff = abs(Lg - ref.L)
    assert diff.max() <= 2 * U32 * abs(ref.L).max()
    np.testing.assert_allclose(scale, ref.scale, rtol=2 * U32)
    assert L.max_degree == int(ref.count_degree.max())
    assert L.lambda_bound == pytest.approx(ref.lambda_bound, rel=1e-12)
    rev = L.rev[: L.nnz].cpu().numpy()
    row_of = np.repeat(np.arange(L.n), np.diff(rowptr))
    np.testing.assert_array_equal(col[rev], row_of)
    np.testing.assert_array_equal(rev[rev], np.arange(L.nnz))
    # packed walk records agree with the CSR arrays and the oracle's adjacency
    we = L.wentry[: 8 * L.nnz].view(L.nnz, 8).cpu().numpy()
    np.testing.assert_array_equal(we[:, 0], r_col)
    np.testing.assert_array_equal(we[:, 1].view(np.float32), val)
    np.testing.assert_array_equal(we[:, 2], rev - rowptr[r_col])
    np.testing.assert_array_equal(we[:, 3], np.diff(r_rowptr)[r_col])
    np.testing.assert_array_equal(we[:, 4:6].copy().view(np.int64)[:, 0], rowptr[r_col])
    np.testing.assert_allclose(we[:, 6].view(np.float32), np.sqrt(ref.scale)[r_col], rtol=3 * U32)
    wn = L.wnode[: 2 * L.n].view(L.n, 2).cpu().numpy()
    np.testing.assert_array_equal(wn[:, 0], rowptr[:-1])
    np.testing.assert_array_equal((wn[:, 1] & 0xFFFFFFFF).astype(np.int64), np.diff(r_rowptr))
    root = (wn[:, 1] >> 32).astype(np.uint32).view(np.float32)
    np.testing.assert_allclose(root, np.sqrt(ref.scale), rtol=3 * U32)
    d = np.diff(rowptr)
    bins = L.bins[: L.n_medium + L.n_heavy].cpu().numpy()
    np.testing.assert_array_equal(bins[: L.n_medium], np.nonzero((d > sped.LIGHT_MAX) & (d <= sped.MEDIUM_MAX))[0])
    np.testing.assert_array_equal(bins[L.n_medium:], np.nonzero(d > sped.MEDIUM_MAX)[0])
    assert L.n_heavy >= 1 and L.n_medium >= 2


def test_laplacian_edge_cases(sped):
    _say("laplacian empty / self-loops only")
    L = sped.Laplacian(7, [], [], kind="sym")
    assert L.n == 7 and L.nnz == 0
    assert np.all(L.host_csr()[3] == 0) and np.all(L.host_csr()[4] == 0)
    L2 = sped.Laplacian(4, [1, 2], [1, 2], kind="combinatorial")
    assert L2.nnz == 0
    with pytest.raises(sped.SpedError):
        sped.Laplacian(4, [0, 5], [1, 2])
    with pytest.raises(sped.SpedError):
        sped.Laplacian(4, [0, 1], [1, 2], w=[1.0, -1.0])


def test_limit_chain_at_the_largest_degree(sped):
    """The limit product at the largest degree the chain takes (l = 1024):
    every factor I - L/1024 has its spectrum in [1 - 2/1024, 1], so float32
    rounding adds up over the 1024 steps to about 1024 u; checked against
    the oracle's float64 product at 3e-4 relative."""
    _say("limit chain, degree 1024")
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    X = synth.gaussian_block(n, 8, 4).astype(np.float32)
    Y = sped.apply_poly(L, sped.transform("limit", 1024), torch.from_numpy(X).cuda()).cpu().numpy()
    Yr = opoly.apply_limit_product(ref.L, 1024, X.astype(np.float64))
    assert _rel(Y.astype(np.float64), Yr) < 3e-4


def test_empty_graph_products(sped):
    """A 0-node Laplacian and its 0-row blocks: the polynomial chain, the
    walk estimate and the Gram return empty results without error; on the
    7-node edgeless graph p(L) X = p(0) X for the combinatorial L."""
    _say("products on an empty graph")
    L = sped.Laplacian(0, [], [], kind="sym")
    X = torch.zeros(0, 8, dtype=torch.float32, device="cuda")
    assert sped.apply_poly(L, sped.transform("limit", 4), X).shape == (0, 8)
    assert sped.apply_poly_stochastic(L, sped.transform("limit", 4).monomial(), X, walks=4, seed=1).shape == (0, 8)
    assert sped.gram(X).shape == (8, 8) and float(sped.gram(X).abs().max()) == 0.0
    L7 = sped.Laplacian(7, [], [], kind="combinatorial")
    X7 = torch.from_numpy(synth.gaussian_block(7, 8, 1).astype(np.float32)).cuda()
    p = sped.transform("taylor_exp", 5)
    Y = sped.apply_poly(L7, p, X7).cpu().numpy()
    np.testing.assert_allclose(Y, p.monomial()[0] * X7.cpu().numpy(), rtol=1e-6, atol=1e-6)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


POLYS = [
    ("limit16-product", lambda s, lam: s.transform("limit", 16, lam), lambda lam: opoly.limit_exp(16)),
    ("limit16-horner", lambda s, lam: s.transform("limit", 16, lam, product_form=False), lambda lam: opoly.limit_exp(16)),
    ("taylor_exp9", lambda s, lam: s.transform("taylor_exp", 9, lam), lambda lam: opoly.taylor_exp(9)),
    ("taylor_log9", lambda s, lam: s.transform("taylor_log", 9, lam), lambda lam: opoly.taylor_log(9, lam)),
    ("plain", lambda s, lam: s.transform("plain", 1, lam), lambda lam: opoly.plain(lam)),
]


@pytest.mark.parametrize("pname,mk,mkref", POLYS, ids=[p[0] for p in POLYS])
@pytest.mark.parametrize("k", [32, 7, 64])
def test_apply_poly_parity(sped, pname, mk, mkref, k):
    n, src, dst, w = mixed_degree_graph()
    _say(f"apply_poly {pname} k={k}")
    L = sped.Laplacian(n, src, dst, w, kind="sym")
    ref = olap.laplacian(n, src, dst, w, kind=olap.SYM_NORMALIZED)
    X = synth.gaussian_block(n, k, 3).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    Y = sped.apply_poly(L, mk(sped, L.lambda_bound), Xd).cpu().numpy().astype(np.float64)
    Yr = opoly.apply_terms(ref.L, mkref(ref.lambda_bound), X.astype(np.float64))
    assert _rel(Y, Yr) < 3e-5
    assert np.abs(Y - Yr).max() < 2e-4 * np.abs(Yr).max()


@pytest.mark.parametrize("xdt,ydt", [("bf16", "f32"), ("f32", "bf16"), ("bf16", "bf16")])
def test_apply_poly_bf16(sped, xdt, ydt):
    n, src, dst, w = mixed_degree_graph()
    _say(f"apply_poly bf16 x={xdt} y={ydt}")
    L = sped.Laplacian(n, src, dst, w, kind="sym")
    ref = olap.laplacian(n, src, dst, w, kind=olap.SYM_NORMALIZED)
    k = 64
    X = torch.from_numpy(synth.gaussian_block(n, k, 4).astype(np.float32))
    tx = {"bf16": torch.bfloat16, "f32": torch.float32}
    Xd = X.to(tx[xdt]).cuda()
    Y = sped.apply_poly(L, sped.transform("limit", 16), Xd, out_dtype=tx[ydt]).float().cpu().numpy()
    Yr = opoly.apply_terms(ref.L, opoly.limit_exp(16), Xd.float().cpu().numpy().astype(np.float64))
    tol = 3e-5 + (2.0 ** -8 if ydt == "bf16" else 0.0)
    assert _rel(Y, Yr) < tol


@pytest.mark.parametrize("k", [8, 64, 72])
@pytest.mark.parametrize("ydt", ["bf16", "f32"])
def test_bf16_gather_eight_columns_per_lane(sped, k, ydt):
    """A bf16 block whose width is a multiple of 8 is gathered 8 columns per
    lane (one 16-byte load per lane and row): one step L X and the degree-3
    Taylor chain on the hub graph (light, medium and heavy rows), against the
    oracle on the bf16-rounded input."""
    n, src, dst, w = mixed_degree_graph()
    _say(f"bf16 8-column gathers k={k} y={ydt}")
    L = sped.Laplacian(n, src, dst, w, kind="sym")
    ref = olap.laplacian(n, src, dst, w, kind=olap.SYM_NORMALIZED)
    Xb = torch.from_numpy(synth.gaussian_block(n, k, 6).astype(np.float32)).cuda().to(torch.bfloat16)
    X64 = Xb.float().cpu().numpy().astype(np.float64)
    out_dt = torch.bfloat16 if ydt == "bf16" else torch.float32
    Y = sped.apply_poly(L, sped.monomial([0.0, 1.0]), Xb, out_dtype=out_dt).float().cpu().numpy()
    Yr = ref.L @ X64
    # one float32 sum per entry, then (bf16 output) one rounding of 2^-9
    rel = 2.0 ** -8 if ydt == "bf16" else 1e-5
    assert np.all(np.abs(Y - Yr) <= rel * np.abs(Yr) + 1e-5 * np.abs(Yr).max())
    Y3 = sped.apply_poly(L, sped.transform("taylor_exp", 3), Xb, out_dtype=out_dt).float().cpu().numpy()
    Y3r = opoly.apply_terms(ref.L, opoly.taylor_exp(3), X64)
    assert _rel(Y3, Y3r) < (3e-5 + (2.0 ** -8 if ydt == "bf16" else 0.0))


def test_apply_poly_padded_ld_and_tiny(sped):
    """leading dimension > k, k = 1, and n smaller than one block."""
    _say("apply_poly padded ld / k=1 / tiny n")
    n, s, d = synth.path_graph(5)
    L = sped.Laplacian(n, s, d, kind="combinatorial")
    ref = olap.laplacian(n, s, d, kind=olap.COMBINATORIAL)
    big = torch.from_numpy(synth.gaussian_block(n, 12, 1).astype(np.float32)).cuda()
    X = big[:, 2:7]   # k = 5, ld = 12, offset 2 floats
    p = sped.transform("taylor_exp", 5, L.lambda_bound)
    Y = sped.apply_poly(L, p, X).cpu().numpy()
    Yr = opoly.apply_terms(ref.L, opoly.taylor_exp(5), X.cpu().numpy().astype(np.float64))
    assert _rel(Y, Yr) < 1e-5
    X1 = big[:, :1].contiguous()
    Y1 = sped.apply_poly(L, p, X1).cpu().numpy()
    assert _rel(Y1, opoly.apply_terms(ref.L, opoly.taylor_exp(5), X1.cpu().numpy().astype(np.float64))) < 1e-5


@pytest.mark.parametrize("k", [97, 300])
def test_wide_blocks_span_column_tiles(sped, k):
    """Blocks wider than one column tile (64 lanes x VEC columns: k = 97 has
    VEC = 1, two tiles; k = 300 has VEC = 4, two tiles) on the mixed-degree
    graph: the exact product, the inner-product path of the backward and the
    walk estimate against the oracle."""
    n, src, dst, w = mixed_degree_graph()
    _say(f"wide block k={k}")
    L = sped.Laplacian(n, src, dst, w, kind="sym")
    ref = olap.laplacian(n, src, dst, w, kind=olap.SYM_NORMALIZED)
    X = synth.gaussian_block(n, k, 12).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    Y = sped.apply_poly(L, sped.transform("limit", 6), Xd).cpu().numpy()
    Yr = opoly.apply_terms(ref.L, opoly.limit_exp(6), X.astype(np.float64))
    assert _rel(Y, Yr) < 3e-5
    G = synth.gaussian_block(n, k, 13).astype(np.float32)
    dth = sped.poly_backward(L, 4, Xd, torch.from_numpy(G).cuda()).cpu().numpy()
    dth_r, _ = ograd.backward(ref.L, np.zeros(5), X.astype(np.float64), G.astype(np.float64))
    np.testing.assert_allclose(dth, dth_r, rtol=5e-5, atol=5e-5 * np.abs(dth_r).max())
    c = np.array([0.9, -0.5, 0.25])
    Ys = sped.apply_poly_stochastic(L, c, Xd, walks=3, seed=2, counter=1).cpu().numpy()
    rows = np.concatenate([np.arange(30), [0, 17, 1200], np.arange(n - 30, n)])
    Ysr = owalk.estimate_importance(ref, c, X.astype(np.float64), 3, seed=2, counter=1, rows=rows)
    assert (np.abs(Ys[rows] - Ysr) / (np.abs(Ysr).max(axis=1, keepdims=True) + 1.0)).max() < 1e-4


def test_apply_poly_isolated_nodes(sped):
    _say("apply_poly with isolated nodes")
    src, dst = [0, 1, 2, 5], [1, 2, 3, 6]
    L = sped.Laplacian(9, src, dst, kind="sym")
    ref = olap.laplacian(9, src, dst, kind=olap.SYM_NORMALIZED)
    X = synth.gaussian_block(9, 4, 2).astype(np.float32)
    Y = sped.apply_poly(L, sped.transform("limit", 8), torch.from_numpy(X).cuda()).cpu().numpy()
    np.testing.assert_allclose(Y, opoly.apply_terms(ref.L, opoly.limit_exp(8), X.astype(np.float64)), atol=1e-5)
    np.testing.assert_allclose(Y[[4, 7, 8]], X[[4, 7, 8]], rtol=1e-6)   # zero rows: M = I there


def test_xcd_row_split_power_law(sped):
    """Degree-sorted power-law graph: the builder's 8 XCD row ranges carry
    equal light-row work (recomputed here from the row pointers, exactly), and
    the light SpMM gives the same rows bit for bit under that split, the even
    split and a caller-built (zeroed or invalid) split; all match the oracle."""
    n, src, dst, _ = synth.chung_lu(30000, 2.1, 12.0, 8, 0.7, seed=4)
    _say(f"xcd split power-law n={n} m={src.shape[0]}")
    L = sped.Laplacian(n, src, dst, kind="sym")
    ref = olap.laplacian(n, src, dst, None, kind=olap.SYM_NORMALIZED)
    d = np.diff(L.host_csr()[0])
    work = np.where(d <= sped.LIGHT_MAX, d + 2, 1)
    pre = np.concatenate([[0], np.cumsum(work)])
    tot = int(pre[-1])
    x = np.arange(9)
    expect = np.searchsorted(pre, tot // 8 * x + tot % 8 * x // 8, side="left")
    assert L.xcd_rows == expect.tolist()
    assert L.xcd_rows[0] == 0 and L.xcd_rows[8] == n
    per = np.diff(pre[expect])
    assert per.max() - per.min() <= 2 * (sped.LIGHT_MAX + 2)
    assert pre[n // 8] > 2 * tot / 8  # the even split would load the first die with > 2x
    poly = sped.transform("limit", 16, L.lambda_bound)
    for k in (32, 7):
        X = synth.gaussian_block(n, k, 8).astype(np.float32)
        Xd = torch.from_numpy(X).cuda()
        Y = sped.apply_poly(L, poly, Xd).cpu().numpy()
        Yr = opoly.apply_terms(ref.L, opoly.limit_exp(16), X.astype(np.float64))
        assert _rel(Y.astype(np.float64), Yr) < 3e-5
        saved = list(L.c.xcd_rows)
        try:
            for other in ([0] * 9, [0, 5, 4, 9, 9, 9, 9, 9, n], [0, n, n, n, n, n, n, n, n]):
                L.c.xcd_rows[:] = other
                Y2 = sped.apply_poly(L, poly, Xd).cpu().numpy()
                np.testing.assert_array_equal(Y2, Y)
        finally:
            L.c.xcd_rows[:] = saved
    # the inner-product path (partials per block) under both splits
    g = np.random.default_rng(9)
    X = g.standard_normal((n, 10)).astype(np.float32)
    G = g.standard_normal((n, 10)).astype(np.float32)
    Xd, Gd = torch.from_numpy(X).cuda(), torch.from_numpy(G).cuda()
    dth = sped.poly_backward(L, 12, Xd, Gd).cpu().numpy()
    saved = list(L.c.xcd_rows)
    try:
        L.c.xcd_rows[:] = [0] * 9
        dth_even = sped.poly_backward(L, 12, Xd, Gd).cpu().numpy()
    finally:
        L.c.xcd_rows[:] = saved
    theta = np.zeros(13)
    dth_r, _ = ograd.backward(ref.L, theta, X.astype(np.float64), G.astype(np.float64))
    np.testing.assert_allclose(dth, dth_r, rtol=5e-5, atol=5e-5 * np.abs(dth_r).max())
    np.testing.assert_allclose(dth, dth_even, rtol=1e-6, atol=1e-6 * np.abs(dth_r).max())


@pytest.fixture(scope="module")
def c2_case(sped):
    """SBM, 10^6 nodes, 100 blocks, mean degree 20, 5% cross edges (k=32, l=16)."""
    _say("building the 1e6-node SBM")
    n, s, d, labels = synth.sbm_from_degrees(1_000_000, 100, 19.0, 1.0, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    X = synth.gaussian_block(n, 32, 2).astype(np.float32)
    return L, ref, X


def test_apply_poly_full_size(sped, c2_case):
    L, ref, X = c2_case
    _say("apply_poly limit16 at n=1e6, k=32")
    Y = sped.apply_poly(L, sped.transform("limit", 16), torch.from_numpy(X).cuda()).cpu().numpy()
    Yr = opoly.apply_limit_product(ref.L, 16, X.astype(np.float64))
    assert _rel(Y, Yr) < 3e-5
    assert np.abs(Y - Yr).max() < 2e-4 * np.abs(Yr).max()


def test_stochastic_full_size_sampled_rows(sped, c2_case):
    L, ref, X = c2_case
    _say("importance walks at n=1e6, k=32, 8 walks/row, sampled rows")
    c = opoly.limit_exp(16).coeffs
    Y = sped.apply_poly_stochastic(L, c, torch.from_numpy(X).cuda(), walks=8, seed=3, counter=1).cpu().numpy()
    rows = np.random.default_rng(0).choice(L.n, 300, replace=False)
    rows = np.concatenate([rows, [0, L.n - 1]])
    Yr = owalk.estimate_importance(ref, c, X.astype(np.float64), 8, seed=3, counter=1, rows=rows)
    err = np.abs(Y[rows] - Yr)
    assert err.max() <= 1e-4 * max(1.0, np.abs(Yr).max())


@pytest.mark.parametrize("kind", ["sym", "combinatorial"])
def test_stochastic_importance_same_walks(sped, kind):
    n, src, dst, w = mixed_degree_graph()
    _say(f"importance walks parity kind={kind}")
    L = sped.Laplacian(n, src, dst, w, kind=kind)
    ref = olap.laplacian(n, src, dst, w, kind=olap.SYM_NORMALIZED if kind == "sym" else olap.COMBINATORIAL)
    X = synth.gaussian_block(n, 16, 5).astype(np.float32)
    c = np.array([0.9, -0.5, 0.25, -0.1, 0.05]) / (1.0 if kind == "sym" else 100.0)
    Y = sped.apply_poly_stochastic(L, c, torch.from_numpy(X).cuda(), walks=6, seed=11, counter=4).cpu().numpy()
    rows = np.concatenate([np.arange(40), [0, 17, 1200], np.arange(n - 40, n)])
    Yr = owalk.estimate_importance(ref, c, X.astype(np.float64), 6, seed=11, counter=4, rows=rows)
    scale = np.abs(Yr).max(axis=1, keepdims=True) + 1.0
    assert (np.abs(Y[rows] - Yr) / scale).max() < 1e-4


@pytest.mark.parametrize("kind,m,ydt", [("sym", 1, "f32"), ("sym", 3, "bf16"), ("combinatorial", 2, "f32"),
                                         ("sym", 4, "f32")])
def test_hybrid_same_walks(sped, kind, m, ydt):
    """Exact low-order terms plus sampled tail: the same walks as the oracle's
    (m = 4 = degree: no walks, the exact polynomial)."""
    n, src, dst, w = mixed_degree_graph()
    _say(f"hybrid parity kind={kind} m={m} y={ydt}")
    L = sped.Laplacian(n, src, dst, w, kind=kind)
    ref = olap.laplacian(n, src, dst, w, kind=olap.SYM_NORMALIZED if kind == "sym" else olap.COMBINATORIAL)
    X = synth.gaussian_block(n, 16, 5).astype(np.float32)
    c = np.array([0.9, -0.5, 0.25, -0.1, 0.05]) / (1.0 if kind == "sym" else np.array([1, 100, 1e4, 1e6, 1e8]))
    out_dt = torch.bfloat16 if ydt == "bf16" else torch.float32
    Y = sped.apply_poly_hybrid(L, c, torch.from_numpy(X).cuda(), m, walks=6, seed=11, counter=4,
                               out_dtype=out_dt).float().cpu().numpy()
    Yr = owalk.estimate_hybrid(ref, c, X.astype(np.float64), m, 6, seed=11, counter=4)
    scale = np.abs(Yr).max(axis=1, keepdims=True) + 1.0
    tol = 8e-3 if ydt == "bf16" else 1e-4
    assert (np.abs(Y - Yr) / scale).max() < tol


def test_hybrid_reject_sampler_same_trials(sped):
    _say("hybrid with the rejection sampler, m=2")
    n, s, d, _ = synth.sbm_bernoulli([60, 80], 0.2, 0.02, seed=2)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    X = synth.gaussian_block(n, 8, 6).astype(np.float32)
    c = np.array([0.9, -0.5, 0.25, -0.1, 0.05])
    trials = 200000
    Y = sped.apply_poly_hybrid(L, c, torch.from_numpy(X).cuda(), 2, walks=trials, seed=5, counter=2,
                               sampler="reject").cpu().numpy()
    Yr = owalk.estimate_hybrid(ref, c, X.astype(np.float64), 2, 0, seed=5, counter=2, sampler="reject",
                               n_trials=trials)
    scale = np.abs(Yr).max(axis=1, keepdims=True) + 1.0
    assert (np.abs(Y - Yr) / scale).max() < 1e-4


def test_hybrid_full_size_sampled_rows(sped, c2_case):
    """n = 1e6, k = 32, degree-16 limit polynomial, 8 walks per row, 2 exact
    terms: sampled rows against the oracle, which needs the tail only on the
    rows' 2-hop neighbourhoods."""
    L, ref, X = c2_case
    _say("hybrid m=2 at n=1e6, k=32, sampled rows")
    c = opoly.limit_exp(16).coeffs
    Y = sped.apply_poly_hybrid(L, c, torch.from_numpy(X).cuda(), 2, walks=8, seed=3, counter=1).cpu().numpy()
    rows = np.concatenate([np.random.default_rng(1).choice(L.n, 48, replace=False), [0, L.n - 1]])
    A = ref.L.tocsr()
    n1 = np.unique(np.concatenate([rows, A[rows].indices]))
    n2 = np.unique(np.concatenate([n1, A[n1].indices]))
    X64 = X.astype(np.float64)
    U = np.zeros_like(X64)
    U[n2] = owalk.estimate_importance(ref, c[2:], X64, 8, seed=3, counter=1, rows=n2)
    U1 = np.zeros_like(X64)
    U1[n1] = A[n1] @ U + c[1] * X64[n1]
    Yr = A[rows] @ U1 + c[0] * X64[rows]
    err = np.abs(Y[rows] - Yr)
    assert err.max() <= 1e-4 * max(1.0, np.abs(Yr).max())


def test_stochastic_reject_same_walks(sped):
    _say("rejection walks parity")
    n, s, d, _ = synth.sbm_bernoulli([60, 80], 0.2, 0.02, seed=2)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    X = synth.gaussian_block(n, 8, 3).astype(np.float32)
    c = np.array([0.5, -0.5, 0.25, -0.125])
    N = 200000
    Y, cnt = sped.apply_poly_stochastic(L, c, torch.from_numpy(X).cuda(), walks=N, seed=9, counter=2,
                                        sampler="reject", accept_counts=True)
    Yr, cr = owalk.estimate_reject(ref, c, X.astype(np.float64), N, seed=9, counter=2)
    np.testing.assert_array_equal(cnt.cpu().numpy(), cr)
    assert _rel(Y.cpu().numpy(), Yr) < 1e-5


def test_stochastic_unbiased(sped):
    """Mean over many seeds of the GPU importance estimate matches p(L)X."""
    _say("importance unbiasedness over 64 seeds")
    n, s, d, _ = synth.sbm_bernoulli([30, 40], 0.3, 0.05, seed=7)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    X = synth.gaussian_block(n, 4, 3).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    c = opoly.limit_exp(8).coeffs
    est = np.stack([sped.apply_poly_stochastic(L, c, Xd, walks=512, seed=100 + t).cpu().numpy() for t in range(64)])
    exact = opoly.apply_terms(ref.L, opoly.limit_exp(8), X.astype(np.float64))
    z = np.abs(est.mean(0) - exact) / (est.std(0, ddof=1) / 8.0 + 1e-12)
    assert z.max() < 5.0


@pytest.mark.parametrize("dt", ["f32", "bf16"])
@pytest.mark.parametrize("ka,kb", [(20, 36), (56, 56), (61, 128), (100, 7), (128, 128), (32, 32), (18, 30),
                                   (31, 32), (14, 24), (72, 72), (65, 80), (40, 48)])
def test_gram_parity(sped, dt, ka, kb):
    """G = A^T B against float64 numpy on the same (rounded) operands: narrow
    (both widths <= 32; column pairs when both are even and above 16, else one
    column per lane), wide with 4 or 8 wavefronts per block, symmetric Grams
    of 33-80 columns on the narrow kernel (3, 4 and 5 tiles a side), odd
    widths and a ragged row count; the symmetric form is exactly symmetric
    and the reduction order is fixed."""
    _say(f"gram {dt} {ka}x{kb}")
    g = np.random.default_rng(ka * 1000 + kb)
    n = 100_003
    A = torch.from_numpy(g.standard_normal((n, ka)).astype(np.float32))
    B = torch.from_numpy(g.standard_normal((n, kb)).astype(np.float32))
    tdt = torch.float32 if dt == "f32" else torch.bfloat16
    Ad, Bd = A.to(tdt).cuda(), B.to(tdt).cuda()
    G = sped.gram(Ad, Bd).cpu().numpy()
    An = Ad.float().cpu().numpy().astype(np.float64)
    Bn = Bd.float().cpu().numpy().astype(np.float64)
    Gr = An.T @ Bn
    assert np.abs(G - Gr).max() <= 1e-12 * np.abs(Gr).max()
    for X, Xn in ((Ad, An), (Bd, Bn)):
        S = sped.gram(X).cpu().numpy()
        np.testing.assert_allclose(S, Xn.T @ Xn, rtol=1e-12, atol=1e-12 * n)
        np.testing.assert_array_equal(S, S.T)
    G2 = sped.gram(Ad, Bd).cpu().numpy()
    np.testing.assert_array_equal(G, G2)   # fixed reduction order


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_gram_symmetric_width_sweep(sped, dt):
    """Symmetric Grams at every width class the planner distinguishes
    (1-32 narrow and column pairs, 33-80 on the narrow kernel with 3-5 tiles
    a side, 81-128 wide) and row counts 0, 1, 17, 1000 and 100,003, against
    float64 numpy; exactly symmetric."""
    g = np.random.default_rng(11)
    tdt = torch.float32 if dt == "f32" else torch.bfloat16
    _say(f"gram symmetric width sweep {dt}")
    for k in (1, 15, 16, 17, 31, 32, 33, 47, 48, 49, 56, 64, 65, 72, 80, 81, 96, 128):
        for n in (0, 1, 17, 1000, 100_003):
            A = torch.from_numpy(g.standard_normal((n, k)).astype(np.float32)).to(tdt).cuda()
            S = sped.gram(A).cpu().numpy()
            An = A.float().cpu().numpy().astype(np.float64)
            R = An.T @ An
            assert np.abs(S - R).max() <= 1e-12 * max(np.abs(R).max(), 1.0) + 1e-300, (k, n)
            np.testing.assert_array_equal(S, S.T)


@pytest.mark.parametrize("ld,k,off", [(40, 30, 2), (40, 30, 1), (33, 30, 2)])
def test_gram_strided_operands(sped, ld, k, off):
    """Operands that are column slices of wider blocks: an even leading
    dimension with pair-aligned starts keeps the column-pair Gram; an odd
    start or an odd leading dimension (rows not aligned to two elements)
    takes the one-column form; all match float64 numpy."""
    _say(f"gram strided ld={ld} k={k} off={off}")
    g = np.random.default_rng(ld * 100 + k + off)
    n = 50_001
    W = torch.from_numpy(g.standard_normal((n, ld)).astype(np.float32)).cuda()
    A, B = W[:, :k], W[:, off:k + off]
    An = A.cpu().numpy().astype(np.float64)
    Bn = B.cpu().numpy().astype(np.float64)
    G = sped.gram(A, B).cpu().numpy()
    Gr = An.T @ Bn
    assert np.abs(G - Gr).max() <= 1e-12 * np.abs(Gr).max()
    S = sped.gram(A).cpu().numpy()
    np.testing.assert_allclose(S, An.T @ An, rtol=1e-12, atol=1e-12 * n)
    np.testing.assert_array_equal(S, S.T)


@pytest.mark.parametrize("k", [1, 2, 3, 8, 14, 15, 16, 17, 18, 56, 57, 70, 72, 90, 96])
def test_orthonormalize_and_rr(sped, k):
    """CholQR2 (fused Cholesky and triangular inverse) and Rayleigh-Ritz
    (Jacobi eigensolver, odd widths padded) against the oracle's Householder
    basis and dense Ritz pairs; widths up to 16 take the one-wavefront
    factorisations, 17 and up the 1024-thread ones; widths 70 and 90 take the
    scalar-load product with 5 and 6 column tiles, 72 and 96 the 4-wide one."""
    _say(f"CholQR2 and Rayleigh-Ritz k={k}")
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    V = synth.gaussian_block(n, k, 2).astype(np.float32)
    Vd = torch.from_numpy(V).cuda()
    Q = sped.orthonormalize(Vd.clone(), passes=2).cpu().numpy().astype(np.float64)
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 2e-6
    assert osol.max_principal_angle(V.astype(np.float64), Q) < 1e-5
    Qd = torch.from_numpy(Q.astype(np.float32)).cuda()
    theta, resid = sped.rayleigh_ritz(L, Qd)
    th_r, Q_r, res_r = osol.rayleigh_ritz(ref.L, Qd.cpu().numpy().astype(np.float64))
    np.testing.assert_allclose(theta.cpu().numpy(), th_r, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(resid.cpu().numpy(), res_r, rtol=1e-3, atol=1e-5)


@pytest.mark.parametrize("k,rows", [(64, 5003), (8, 77), (96, 1000)])
def test_orthonormalize_bf16(sped, k, rows):
    """CholQR2 of a bf16 block (bf16 Gram operands, float64 Gram, bf16 output)
    against the oracle's basis: orthonormal to bf16 rounding, same span; a
    ragged row count and the widest block."""
    _say(f"CholQR2 bf16 k={k} n={rows}")
    V = synth.gaussian_block(rows, k, 4).astype(np.float32)
    Vb = torch.from_numpy(V).cuda().to(torch.bfloat16)
    Q = sped.orthonormalize(Vb.clone(), passes=2).float().cpu().numpy().astype(np.float64)
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 3e-2
    Vr = Vb.float().cpu().numpy().astype(np.float64)
    assert osol.max_principal_angle(Vr, Q) < 2e-2


@pytest.mark.parametrize("poly", ["limit", "plain"])
def test_bottomk_solve_c1(sped, poly):
    """SBM n=2000, 10 blocks, k=10: the bottom-10 span within 1e-6 of dense eigh."""
    _say(f"bottomk solve C1 poly={poly}")
    n, s, d, labels = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    lam, U, _ = osol.dense_bottom_k(ref.dense(), 10)
    k, guard = 10, 4
    V0 = torch.from_numpy(synth.gaussian_block(n, k + guard, 2).astype(np.float32)).cuda()
    p = sped.transform("limit", 8) if poly == "limit" else None
    r = sped.bottomk(L, k, p, V0=V0, guard=guard, tol=1e-6, max_iters=3000)
    assert r.converged, r.stats
    ang = osol.max_principal_angle(U, r.V.cpu().numpy().astype(np.float64))
    assert ang <= 1e-6, (ang, r.stats)
    np.testing.assert_allclose(r.evals[1:], lam[1:], rtol=1e-6)
    assert abs(r.evals[0]) < 1e-6
    _say(f"  iters={r.stats['iters']} spmm={r.stats['spmm_count']} angle={ang:.2e}")


def test_bottomk_solve_c1_tuned_coefficients(sped):
    """Degree-8 coefficients tuned through PolyApply on another 2,000-node SBM
    of the same family (seed 5) solve the C1 graph: the bottom-10 span within
    1e-6 of dense eigh in far fewer iterations than the limit polynomial (43)."""
    from paper_2207_14589_amd import tune
    _say("bottomk solve C1 with tuned degree-8 coefficients")
    k, guard = 10, 4
    n5, s5, d5, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=5)
    Lp = sped.Laplacian(n5, s5, d5, kind="sym")
    Vt = torch.from_numpy(synth.gaussian_block(n5, k + guard, 7).astype(np.float32)).cuda()
    theta, hist = tune.tune_coefficients(Lp, k, 8, Vt, steps=60, unroll=3)
    assert min(hist) < 0.5 * hist[0]
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    lam, U, _ = osol.dense_bottom_k(ref.dense(), 10)
    V0 = torch.from_numpy(synth.gaussian_block(n, k + guard, 2).astype(np.float32)).cuda()
    r = sped.bottomk(L, k, sped.monomial(theta, shift=1.0, scale=1.0), V0=V0, guard=guard, tol=1e-6,
                     max_iters=3000, polish=2)
    assert r.converged, r.stats
    ang = osol.max_principal_angle(U, r.V.cpu().numpy().astype(np.float64))
    assert ang <= 1e-6, (ang, r.stats)
    np.testing.assert_allclose(r.evals[1:], lam[1:], rtol=1e-6)
    assert r.stats["iters"] < 43, r.stats
    _say(f"  iters={r.stats['iters']} spmm={r.stats['spmm_count']} angle={ang:.2e}")


def test_bottomk_combinatorial_limit_cuts_iterations(sped):
    """Combinatorial L of the 2,000-node SBM (lambda_bound = 2 d_max = 56):
    the degree-32 limit operator (2l > lambda_bound) reaches the bottom-10
    span at the 1e-5 bound in a handful of iterations and within 1e-5 of dense
    eigh; the plain operator needs more than ten times as many iterations."""
    _say("bottomk combinatorial C1: limit32 vs plain")
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="combinatorial")
    ref = olap.laplacian(n, s, d, kind=olap.COMBINATORIAL)
    lam, U, _ = osol.dense_bottom_k(ref.dense(), 10)
    V0 = torch.from_numpy(synth.gaussian_block(n, 14, 2).astype(np.float32)).cuda()
    r = sped.bottomk(L, 10, sped.transform("limit", 32, L.lambda_bound), V0=V0, guard=4, tol=1e-5, max_iters=200)
    assert r.converged, r.stats
    assert osol.max_principal_angle(U, r.V.cpu().numpy().astype(np.float64)) <= 1e-5
    np.testing.assert_allclose(r.evals[1:], lam[1:], rtol=1e-5)
    rp = sped.bottomk(L, 10, None, V0=V0, guard=4, tol=1e-5, max_iters=10 * r.stats["iters"])
    assert not rp.converged
    _say(f"  limit32 iters={r.stats['iters']}; plain not converged after {rp.stats['iters']}")


def test_bottomk_oja_and_stochastic_start(sped):
    _say("bottomk with Oja step and stochastic first iterations")
    n, s, d, labels = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    lam, U, _ = osol.dense_bottom_k(ref.dense(), 10)
    V0 = torch.from_numpy(synth.gaussian_block(n, 14, 2).astype(np.float32)).cuda()
    r = sped.bottomk(L, 10, sped.transform("limit", 8), V0=V0, guard=4, tol=1e-6, max_iters=3000, solver="oja",
                     eta=1.0)
    assert r.converged and osol.max_principal_angle(U, r.V.cpu().numpy().astype(np.float64)) <= 1e-6
    r2 = sped.bottomk(L, 10, sped.transform("limit", 8), V0=V0, guard=4, tol=1e-6, max_iters=3000,
                      stochastic_iters=5, walks_per_row=16, seed=5)
    assert r2.converged and osol.max_principal_angle(U, r2.V.cpu().numpy().astype(np.float64)) <= 1e-6


def test_poly_backward_parity(sped):
    _say("poly backward")
    n, src, dst, w = mixed_degree_graph()
    L = sped.Laplacian(n, src, dst, w, kind="sym")
    ref = olap.laplacian(n, src, dst, w, kind=olap.SYM_NORMALIZED)
    g = np.random.default_rng(3)
    theta = g.standard_normal(13) * 0.3
    X = g.standard_normal((n, 10)).astype(np.float32)
    G = g.standard_normal((n, 10)).astype(np.float32)
    dth = sped.poly_backward(L, 12, torch.from_numpy(X).cuda(), torch.from_numpy(G).cuda()).cpu().numpy()
    dth_r, dX_r = ograd.backward(ref.L, theta, X.astype(np.float64), G.astype(np.float64))
    np.testing.assert_allclose(dth, dth_r, rtol=5e-5, atol=5e-5 * np.abs(dth_r).max())


def test_polyapply_autograd(sped):
    _say("PolyApply forward/backward vs float64 reference")
    from paper_2207_14589_amd.autograd import poly_apply
    n, s, d, _ = synth.sbm_bernoulli([150, 150, 200], 0.05, 0.002, seed=4)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    g = np.random.default_rng(2)
    theta0 = g.standard_normal(13) * 0.2
    X0 = g.standard_normal((n, 6)).astype(np.float32)
    G0 = g.standard_normal((n, 6)).astype(np.float32)
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    X = torch.from_numpy(X0).cuda().requires_grad_(True)
    Y = poly_apply(theta, X, L)
    loss = (Y * torch.from_numpy(G0).cuda()).sum()
    loss.backward()
    dth_r, dX_r = ograd.backward(ref.L, theta0, X0.astype(np.float64), G0.astype(np.float64))
    np.testing.assert_allclose(Y.detach().cpu().numpy(), ograd.forward(ref.L, theta0, X0.astype(np.float64)),
                               rtol=1e-4, atol=1e-4)
    np.testing.assert_allclose(theta.grad.numpy(), dth_r, rtol=1e-4, atol=1e-4 * np.abs(dth_r).max())
    np.testing.assert_allclose(X.grad.cpu().numpy(), dX_r, rtol=1e-4, atol=1e-4 * np.abs(dX_r).max())
    # finite differences in theta (the loss is linear in theta: exact up to rounding)
    for j in (0, 5, 12):
        e = np.zeros(13)
        e[j] = 0.1
        lp = float((poly_apply(torch.tensor(theta0 + e), X.detach(), L) * torch.from_numpy(G0).cuda()).sum())
        lm = float((poly_apply(torch.tensor(theta0 - e), X.detach(), L) * torch.from_numpy(G0).cuda()).sum())
        assert (lp - lm) / 0.2 == pytest.approx(dth_r[j], rel=1e-3, abs=1e-3 * np.abs(dth_r).max())


def test_cluster_embed_parity(sped):
    _say("k-means from given centres, and with k-means++ seeding")
    n, s, d, labels = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    _, U, _ = osol.dense_bottom_k(ref.dense(), 10)
    X = okm.normalize_rows(U)
    C0 = okm.kmeans_pp(X, 10, seed=3)
    lab_r, C_r, in_r, it_r = okm.lloyd(X, C0)
    Vd = torch.from_numpy(U.astype(np.float32)).cuda()
    lab, C, inertia, iters = sped.cluster_embed(Vd, 10, row_normalize=True, init=C0)
    Xf = okm.normalize_rows(U.astype(np.float32).astype(np.float64))
    lab_f, C_f, in_f, it_f = okm.lloyd(Xf, C0)
    np.testing.assert_array_equal(lab.cpu().numpy(), lab_f)
    np.testing.assert_allclose(C.cpu().numpy(), C_f, atol=1e-10)
    assert inertia == pytest.approx(in_f, rel=1e-9, abs=1e-12)
    lab2, _, _, _ = sped.cluster_embed(Vd, 10, row_normalize=True, seed=7)
    assert okm.adjusted_rand_index(lab2.cpu().numpy(), labels) > 0.99


def test_stream_copy(sped):
    _say("stream copy")
    a = torch.arange(1 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    sped.stream_copy(a, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_bottomk_bf16_then_f32_refinement(sped):
    """bf16 iterate storage down to its rounding floor (bound ~1e-2 here: bf16's
    u = 2^-9 over a gap of 0.33), then a float32 refinement sweep to 1e-6: the
    bottom-10 span still matches dense eigh within 1e-6, and the bf16 iterate
    itself is within 1e-2 of it."""
    _say("bottomk bf16 storage + float32 refinement")
    n, s, d, labels = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    lam, U, _ = osol.dense_bottom_k(ref.dense(), 10)
    V0 = torch.from_numpy(synth.gaussian_block(n, 14, 2).astype(np.float32)).cuda()
    r = sped.bottomk(L, 10, sped.transform("limit", 8), V0=V0, guard=4, tol=1e-6, max_iters=3000,
                     storage="bf16")
    assert r.converged, r.stats
    assert 0 < r.stats["coarse_iters"] < r.stats["iters"]
    ang = osol.max_principal_angle(U, r.V.cpu().numpy().astype(np.float64))
    assert ang <= 1e-6, (ang, r.stats)
    np.testing.assert_allclose(r.evals[1:], lam[1:], rtol=1e-6)
    _say(f"  bf16 iters={r.stats['coarse_iters']} total={r.stats['iters']} angle={ang:.2e}")


def test_gram_bf16_f32_rayleigh_path(sped):
    """The mixed bf16 x float32 Gram used by the bf16 solver: H = Q^T (L Q)."""
    _say("mixed-dtype Rayleigh-Ritz inside a bf16 solve, 3 iterations vs oracle trajectory")
    n, s, d, _ = synth.sbm_bernoulli([150] * 6, 0.08, 0.002, seed=9)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    V0n = synth.gaussian_block(n, 10, 4).astype(np.float32)
    V0 = torch.from_numpy(V0n).cuda()
    p = opoly.limit_exp(8)
    r32 = sped.bottomk(L, 6, sped.transform("limit", 8), V0=V0, guard=4, tol=0.0, max_iters=3)
    o = osol.subspace_iteration(ref.L, lambda Q: opoly.apply_terms(ref.L, p, Q), 6, V0n.astype(np.float64),
                                max_iters=3, guard=4)
    assert osol.max_principal_angle(o.Q, r32.V.cpu().numpy().astype(np.float64)) < 1e-4
    np.testing.assert_allclose(r32.evals, o.evals, rtol=1e-5, atol=1e-6)


def test_tuned_coefficients_converge_to_true_subspace(sped):
    """Coefficients tuned through PolyApply lower the unrolled Rayleigh loss;
    the solver on the tuned operator needs fewer iterations than on the
    degree-12 limit polynomial (compared at 1e-5, above the float32 iterate's
    noise floor of a few 1e-7 in residual), and still reaches the dense-eigh
    subspace within 1e-6 (eigenvectors come from Rayleigh-Ritz on L itself).
    The reported bound dominates the true sine of the largest angle."""
    _say("theta tuning on a 4,000-node SBM, then a solve with the tuned operator")
    from paper_2207_14589_amd import tune
    n, s, d, _ = synth.sbm_bernoulli([500] * 8, 0.03, 0.0005, seed=3)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    lam, U, _ = osol.dense_bottom_k(ref.dense(), 8)
    Vt = torch.from_numpy(synth.gaussian_block(n, 12, 7).astype(np.float32)).cuda()
    theta, hist = tune.tune_coefficients(L, 8, 12, Vt, steps=40, unroll=3)
    assert min(hist) < hist[0]
    V0 = torch.from_numpy(synth.gaussian_block(n, 12, 2).astype(np.float32)).cuda()
    tuned = sped.monomial(theta, shift=1.0, scale=1.0)
    r = sped.bottomk(L, 8, tuned, V0=V0, guard=4, tol=1e-5, max_iters=3000)
    r0 = sped.bottomk(L, 8, sped.transform("limit", 12), V0=V0, guard=4, tol=1e-5, max_iters=3000)
    assert r.converged and r0.converged
    assert r.stats["iters"] < r0.stats["iters"]
    for res in (r, r0):
        ang = osol.max_principal_angle(U, res.V.cpu().numpy().astype(np.float64))
        assert np.sin(ang) <= res.stats["bound"] <= 1e-5
    r6 = sped.bottomk(L, 8, tuned, V0=V0, guard=4, tol=1e-6, max_iters=3000)
    assert r6.converged
    ang = osol.max_principal_angle(U, r6.V.cpu().numpy().astype(np.float64))
    assert np.sin(ang) <= r6.stats["bound"] <= 1e-6
    _say(f"  loss {hist[0]:.4f} -> {min(hist):.4f}; iters to 1e-5: tuned {r.stats['iters']} "
         f"vs limit {r0.stats['iters']}")


def test_plain_polish_reaches_1e6_past_the_chain_floor(sped):
    """The degree-12 limit polynomial on a 4,000-node SBM settles near its
    float32 rounding floor around 1e-6; with polish_checks the solver hands
    its Ritz vectors to plain iterations on 2I - L once the residual stalls,
    and reaches 1e-6.  The reported bound dominates the true sine of the
    largest angle to the dense-eigh subspace, and the Ritz values match."""
    _say("plain polish after the degree-12 limit operator, 4,000-node SBM, tol 1e-6")
    n, s, d, _ = synth.sbm_bernoulli([500] * 8, 0.03, 0.0005, seed=3)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    lam, U, _ = osol.dense_bottom_k(ref.dense(), 8)
    V0 = torch.from_numpy(synth.gaussian_block(n, 12, 2).astype(np.float32)).cuda()
    p = sped.transform("limit", 12)
    r = sped.bottomk(L, 8, p, V0=V0, guard=4, tol=1e-6, max_iters=600, polish=2)
    r0 = sped.bottomk(L, 8, p, V0=V0, guard=4, tol=1e-6, max_iters=600)
    _say(f"  polish: converged {r.converged} in {r.stats['iters']} iterations ({r.stats['polish_iters']} plain), "
         f"bound {r.stats['bound']:.2e}; without: converged {r0.converged}, bound {r0.stats['bound']:.2e}")
    assert r.converged and r.stats["bound"] <= 1e-6
    ang = osol.max_principal_angle(U, r.V.cpu().numpy().astype(np.float64))
    assert np.sin(ang) <= r.stats["bound"]
    np.testing.assert_allclose(r.evals, lam, rtol=1e-6, atol=1e-7)
    # the polish is refused for the other solvers
    with pytest.raises(sped.SpedError) as e:
        sped.bottomk(L, 8, p, V0=V0, guard=4, tol=1e-6, max_iters=5, polish=2, solver="oja", eta=1.0)
    assert e.value.status == sped.E_UNSUPPORTED


def test_mu_eigengame_trajectory_parity(sped):
    """mu-EigenGame on the GPU follows the oracle's trajectory: same start
    block, same step, 60 iterations of the degree-8 limit operator on the
    2,000-node SBM; every player's vector within 1e-4 rad of the oracle's (the
    guard players do not act on the first k: penalties only come from players
    above)."""
    _say("mu-EigenGame trajectory parity, SBM n=2000, k=10 (+4)")
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    k, guard, eta, iters = 10, 4, 0.5, 60
    V0 = synth.gaussian_block(n, k + guard, 2).astype(np.float32)
    r = sped.bottomk(L, k, sped.transform("limit", 8), V0=torch.from_numpy(V0).cuda(), guard=guard, tol=0.0,
                     max_iters=iters, check_every=iters, solver="mu_eg", eta=eta)
    assert r.stats["iters"] == iters
    p = opoly.limit_exp(8)
    Vo, _ = osol.mu_eigengame(lambda X: opoly.apply_terms(ref.L, p, X), V0[:, :k].astype(np.float64), eta, iters)
    Vg = r.V.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(np.linalg.norm(Vg, axis=0), 1.0, rtol=1e-5)
    assert osol.vector_angles(Vo, Vg).max() < 1e-4


def test_mu_eigengame_recovers_path_eigenvectors(sped):
    """On the path P_40 (distinct eigenvalues, closed-form eigenvectors) the
    GPU game converges to each of the bottom 4 eigenvectors individually, in
    order: full streak, every angle below 1e-3 (float32)."""
    _say("mu-EigenGame on P_40, k=4 (+2)")
    n, k, guard = 40, 4, 2
    _, s, d = synth.path_graph(n)
    L = sped.Laplacian(n, s, d, kind="combinatorial")
    x = np.arange(n)
    U = np.stack([np.cos(np.pi * j * (x + 0.5) / n) for j in range(k)], axis=1)
    U /= np.linalg.norm(U, axis=0)
    V0 = torch.from_numpy(synth.gaussian_block(n, k + guard, 4).astype(np.float32)).cuda()
    r = sped.bottomk(L, k, sped.transform("limit", 16), V0=V0, guard=guard, tol=0.0, max_iters=6000,
                     check_every=6000, solver="mu_eg", eta=0.5)
    Vg = r.V.cpu().numpy().astype(np.float64)
    ang = osol.vector_angles(U, Vg)
    assert osol.eigenvector_streak(U, Vg) == k
    assert ang.max() < 1e-3


@pytest.mark.parametrize("n,c", [(1000, 5), (2000, 5), (2000, 4)])
def test_limit_degree_threshold_cliques_gpu(sped, n, c):
    """The paper's clique experiments at full size on the GPU solver, over its
    degree sweep l = 11, 51, 151, 251: the limit operator reaches the bottom-c
    subspace exactly when 2 l > lambda_max (5 cliques of 200: lambda_max 204,
    so 151 and 251 succeed; 5 cliques of 400: lambda_max 404, only 251; 4
    cliques of 500: lambda_max 503, none).  Plain L reversed always succeeds; a
    successful limit operator needs far fewer iterations.  A failure is a wrong
    subspace, a cap hit, or a non-finite operator in float32."""
    _say(f"limit-degree threshold on cliques n={n} c={c}")
    N, s, d, _ = synth.cliques_short_circuit(n, c, seed=1)
    L = sped.Laplacian(N, s, d, kind="combinatorial")
    ref = olap.laplacian(N, s, d, kind=olap.COMBINATORIAL)
    lam, U, full = osol.dense_bottom_k(ref.dense(), c)
    V0 = torch.from_numpy(synth.gaussian_block(N, c + 2, 2).astype(np.float32)).cuda()

    def outcome(p):
        try:
            r = sped.bottomk(L, c, p, V0=V0, guard=2, tol=1e-6, max_iters=200)
        except RuntimeError:
            return False, None
        ang = osol.max_principal_angle(U, r.V.cpu().numpy().astype(np.float64))
        return bool(r.converged and ang < 1e-4), r.stats["iters"]

    ok, plain_iters = outcome(None)
    assert ok
    for ell in (11, 51, 151, 251):
        ok, iters = outcome(sped.transform("limit", ell))
        assert ok == (2 * ell > full[-1]), (ell, full[-1])
        if ok:
            assert iters * 5 < plain_iters


def test_three_room_grid_steps_gpu(sped):
    """Sec. 5's 3-room grid (s = 2, h = 10), bottom 3 (+2 guard), combinatorial
    L: the GPU subspace iteration's first 3 Ritz vectors against the oracle's
    dense eigenvectors (the paper's subspace error 1 - ||U*^T Q||_F^2 / k).
    The degree-251 limit and Taylor forms of -e^{-L} reach 1e-8 within 640
    iterations; the identity transform has not reached it after 640 (it is
    still converging at 6400: the paper's order-of-magnitude reduction).
    The exact log and -e^{-L} arms run on the oracle only."""
    _say("3-room grid s=2 h=10: identity vs degree-251 series on the GPU solver")
    N, s, d = synth.three_room_grid(2, 10)
    L = sped.Laplacian(N, s, d, kind="combinatorial")
    ref = olap.laplacian(N, s, d, kind=olap.COMBINATORIAL)
    lam, U, _ = osol.dense_bottom_k(ref.dense(), 3)
    V0 = torch.from_numpy(synth.gaussian_block(N, 5, 2).astype(np.float32)).cuda()

    def error_after(p, T):
        r = sped.bottomk(L, 3, p, V0=V0, guard=2, tol=0.0, max_iters=T, check_every=T)
        return osol.subspace_error(U, r.V.cpu().numpy().astype(np.float64))

    for name in ("limit", "taylor_exp"):
        e = error_after(sped.transform(name, 251), 640)
        _say(f"  {name} 251: subspace error after 640 iterations {e:.2e}")
        assert e < 1e-8
    e640 = error_after(None, 640)
    e6400 = error_after(None, 6400)
    _say(f"  identity: subspace error after 640 {e640:.2e}, after 6400 {e6400:.2e}")
    assert e640 > 1e-8  # the series forms' target is not met by the identity in 640 steps
    assert e6400 < e640


def test_weighted_link_prediction_graph(sped):
    """Sec. 5 (link prediction): on cliques completed by common-neighbour
    weights the degree-151 limit operator (2 x 151 > lambda_max) reaches the
    oracle's bottom-5 subspace of the weighted combinatorial Laplacian in far
    fewer iterations than plain L, and k-means on it recovers the cliques."""
    _say("weighted link-prediction cliques n=500 c=5")
    N, s, d, w, labels = synth.link_prediction_cliques(500, 5, seed=2)
    L = sped.Laplacian(N, s, d, w, kind="combinatorial")
    ref = olap.laplacian(N, s, d, w, kind=olap.COMBINATORIAL)
    lam, U, full = osol.dense_bottom_k(ref.dense(), 5)
    assert 2 * 151 > full[-1]
    V0 = torch.from_numpy(synth.gaussian_block(N, 7, 2).astype(np.float32)).cuda()
    r = sped.bottomk(L, 5, sped.transform("limit", 151), V0=V0, guard=2, tol=1e-6, max_iters=500)
    r0 = sped.bottomk(L, 5, None, V0=V0, guard=2, tol=1e-6, max_iters=500)
    assert r.converged and r0.converged and r.stats["iters"] * 5 < r0.stats["iters"]
    assert osol.max_principal_angle(U, r.V.cpu().numpy().astype(np.float64)) < 1e-4
    lab, _, _, _ = sped.cluster_embed(r.V, 5, row_normalize=False, seed=1)
    assert okm.adjusted_rand_index(labels, lab.cpu().numpy()) == pytest.approx(1.0)


# ---------------------------------------------------------------- lazy node walk (variance-reduced estimator)
from oracle import lazywalk as olazy  # noqa: E402


@pytest.mark.parametrize("kind,ell", [("sym", 16), ("combinatorial", 32)])
def test_lazy_walk_same_walks(sped, kind, ell):
    """Same seed, same draws: every walk of the GPU estimator ends where the
    oracle's does, so the estimates agree to float32 summation (2,000-node
    unweighted SBM, 10 columns, 8 walks per row; combinatorial needs l >= the
    largest degree)."""
    _say(f"lazy walk same walks {kind} l={ell}")
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind=kind)
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED if kind == "sym" else olap.COMBINATORIAL)
    X = synth.gaussian_block(n, 10, 2).astype(np.float32)
    Y = sped.apply_limit_lazy(L, ell, torch.from_numpy(X).cuda(), 8, seed=5, counter=3).cpu().numpy()
    Yo = olazy.estimate_lazy(ref, ell, X.astype(np.float64), 8, seed=5, counter=3)
    assert np.abs(Y - Yo).max() <= 2e-6 * np.abs(Yo).max()


def test_lazy_walk_weighted_hub_graph(sped):
    """Weighted graph with a 9,000-edge hub, repeated edges and self-loops:
    moves use the rejection proposals and the inverse-CDF fallback.  Every
    row equals the oracle's.  A row that does not must be explained by one
    near-tied decision (a compared pair within 1e-6 relative, where the two
    sides' roundings may differ): the oracle's row with that decision taken
    the other way must then equal the GPU row."""
    _say("lazy walk weighted hub graph")
    n, src, dst, w = mixed_degree_graph()
    L = sped.Laplacian(n, src, dst, w, kind="sym")
    ref = olap.laplacian(n, src, dst, w, kind=olap.SYM_NORMALIZED)
    X = synth.gaussian_block(n, 6, 3).astype(np.float32)
    ell, walks, seed = 12, 4, 9
    Y = sped.apply_limit_lazy(L, ell, torch.from_numpy(X).cuda(), walks, seed=seed).cpu().numpy()
    Yo = olazy.estimate_lazy(ref, ell, X.astype(np.float64), walks, seed=seed)
    tol = 2e-6 * np.abs(Yo).max()
    bad = np.nonzero(~np.all(np.abs(Y - Yo) <= tol, axis=1))[0]
    _say(f"  rows differing from the oracle's walks: {bad.size} of {n}")
    for r in bad:
        paths = [olazy.walk_path(ref, ell, int(r), wi, seed) for wi in range(walks)]
        ends = [z for z, _ in paths]
        np.testing.assert_allclose(olazy.row_from_ends(ref, int(r), ends, X), Yo[r], rtol=1e-12, atol=1e-12)
        margin, wi, i = min((m, wi, i) for wi, (_, dec) in enumerate(paths) for i, (_, m) in enumerate(dec))
        assert margin < 1e-6, f"row {r} differs with no near-tied decision (smallest margin {margin:.2e})"
        ends[wi] = olazy.walk_path(ref, ell, int(r), wi, seed, flip=i)[0]
        alt = olazy.row_from_ends(ref, int(r), ends, X)
        assert np.all(np.abs(Y[r] - alt) <= tol), f"row {r} matches neither rounding of its tied decision"


def test_lazy_walk_unbiased(sped):
    """Mean over 64 seeds against the exact (I - L/16)^16 X: per-entry z-scores
    from the spread over seeds stay within a Bonferroni bound."""
    _say("lazy walk unbiasedness, 64 seeds")
    n, s, d, _ = synth.sbm_bernoulli([40] * 5, 0.2, 0.01, seed=4)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    X = synth.gaussian_block(n, 4, 1).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    est = np.stack([sped.apply_limit_lazy(L, 16, Xd, 16, seed=100 + i).cpu().numpy() for i in range(64)])
    exact = opoly.apply_limit_product(ref.L, 16, X.astype(np.float64))
    z = np.abs(est.mean(0) - exact) / (est.std(0, ddof=1) / 8.0 + 1e-12)
    assert z.max() < 5.0


def test_lazy_walk_full_size_sampled_rows(sped, c2_case):
    """The 10^6-node SBM at the bench's shape (k = 32, l = 16, 8 walks per row):
    2,000 sampled rows match the oracle's walks for those rows."""
    L, ref, X = c2_case
    _say("lazy walk full size, sampled rows")
    Y = sped.apply_limit_lazy(L, 16, torch.from_numpy(X).cuda(), 8, seed=3).cpu().numpy()
    rows = np.random.default_rng(0).choice(L.n, 2000, replace=False)
    Yo = olazy.estimate_lazy(ref, 16, X.astype(np.float64), 8, seed=3, rows=rows)
    assert np.abs(Y[rows] - Yo).max() <= 2e-6 * np.abs(Yo).max()


def test_solver_stochastic_phase_lazy_vs_edge_walks(sped):
    """Solver iterations driven only by random estimates (8 walks per row,
    degree-8 limit operator, 2,000-node SBM, 40 iterations): the lazy node
    walk leaves the iterate closer to the true bottom-10 subspace than the
    edge-chain walk; followed by exact iterations both reach 1e-6."""
    _say("solver stochastic phase: lazy vs edge walks")
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    lam, U, _ = osol.dense_bottom_k(ref.dense(), 10)
    V0 = torch.from_numpy(synth.gaussian_block(n, 14, 2).astype(np.float32)).cuda()
    p = sped.transform("limit", 8)
    err = {}
    for sampler in ("importance", "lazy"):
        r = sped.bottomk(L, 10, p, V0=V0, guard=4, tol=0.0, max_iters=40, stochastic_iters=40, walks_per_row=8,
                         sampler=sampler, exact_terms=0)
        err[sampler] = osol.subspace_error(U, r.V.cpu().numpy().astype(np.float64))
        r2 = sped.bottomk(L, 10, p, V0=V0, guard=4, tol=1e-6, max_iters=3000, stochastic_iters=20,
                          walks_per_row=8, sampler=sampler, exact_terms=0)
        assert r2.converged
        assert osol.max_principal_angle(U, r2.V.cpu().numpy().astype(np.float64)) < 1e-5
    assert err["lazy"] < err["importance"]
    _say(f"  subspace error after 40 random iterations: edge {err['importance']:.3e}, lazy {err['lazy']:.3e}")


def test_solver_stochastic_phase_exact_low_terms(sped):
    """The same random-estimate phase with the first 3 terms of the degree-8
    limit polynomial exact and the tail sampled: the iterate ends closer to
    the true bottom-10 subspace than with the plain edge walk, each iteration
    costs 3 sparse steps (counted), and exact iterations then reach 1e-6."""
    _say("solver stochastic phase: exact low-order terms")
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    lam, U, _ = osol.dense_bottom_k(ref.dense(), 10)
    V0 = torch.from_numpy(synth.gaussian_block(n, 14, 2).astype(np.float32)).cuda()
    p = sped.transform("limit", 8)
    err = {}
    for m in (0, 3):
        r = sped.bottomk(L, 10, p, V0=V0, guard=4, tol=0.0, max_iters=40, stochastic_iters=40, walks_per_row=8,
                         exact_terms=m)
        err[m] = osol.subspace_error(U, r.V.cpu().numpy().astype(np.float64))
        rr_steps = r.stats["iters"] // 1  # one Rayleigh-Ritz sparse step per check (check_every = 1)
        assert r.stats["spmm_count"] == 40 * m + rr_steps
    assert err[3] < 0.5 * err[0]
    r2 = sped.bottomk(L, 10, p, V0=V0, guard=4, tol=1e-6, max_iters=3000, stochastic_iters=20, walks_per_row=8,
                      exact_terms=3)
    assert r2.converged
    assert osol.max_principal_angle(U, r2.V.cpu().numpy().astype(np.float64)) < 1e-5
    _say(f"  subspace error after 40 random iterations: m=0 {err[0]:.3e}, m=3 {err[3]:.3e}")


def test_powerlaw_bf16_solve_and_cluster(sped):
    """A power-law graph with planted communities (Chung-Lu, exponent 2.1,
    mean degree 16, 24 communities, 95% of draws inside; largest component,
    5,960 nodes): the bottom 24 with bf16 storage and the float32 refinement
    reach the dense-eigh subspace at the 1e-5 bound (the degree-16 operator's
    float32 floor on this graph is near 2e-6), for the limit operator and for
    plain L; the bf16 phase alone stops within 1e-2 of it (measured 3.9e-3 and
    4.7e-3, the rounding floor of bf16 vectors); k-means on the rows recovers
    the planted communities."""
    _say("power-law bf16 solve, 24 communities")
    n, s, d, comm = synth.chung_lu(6000, 2.1, 16.0, 24, 0.95, seed=3)
    L = sped.Laplacian(n, s, d, kind="sym", lcc=True)
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED, lcc=True)
    assert L.n == ref.n
    lam, U, _ = osol.dense_bottom_k(ref.dense(), 24)
    V0 = torch.from_numpy(synth.gaussian_block(L.n, 32, 2).astype(np.float32)).cuda()
    for p in (sped.transform("limit", 16), None):
        r = sped.bottomk(L, 24, p, V0=V0, guard=8, tol=1e-5, max_iters=3000, storage="bf16")
        assert r.converged, r.stats
        assert osol.max_principal_angle(U, r.V.cpu().numpy().astype(np.float64)) <= 1e-5
        np.testing.assert_allclose(r.evals[1:], lam[1:], rtol=1e-5)
        coarse = r.stats["coarse_iters"]
        rc = sped.bottomk(L, 24, p, V0=V0, guard=8, tol=1e-5, max_iters=coarse, storage="bf16")
        ang_bf16 = osol.max_principal_angle(U, rc.V.cpu().numpy().astype(np.float64))
        assert ang_bf16 <= 1e-2
        _say(f"  {'limit16' if p else 'plain'}: {r.stats['iters']} iterations ({coarse} bf16), "
             f"bf16-phase angle {ang_bf16:.2e}")
    lab, _, _, _ = sped.cluster_embed(r.V, 24, row_normalize=True, seed=1)
    planted = comm[ref.old_of_new]
    assert okm.adjusted_rand_index(lab.cpu().numpy(), planted) > 0.85


@pytest.mark.parametrize("case", ["limit", "plain", "limit_check3", "mu_eg", "bf16", "stochastic_first"])
def test_solver_graph_replay_matches_eager(sped, case):
    """Iterations captured once into HIP graphs and replayed give the eager
    solve's result bit for bit (every replay feeds the next, so one wrong
    replay changes the end result): same iteration count, Ritz values and
    vectors."""
    _say(f"graph replay vs eager: {case}")
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    V0 = torch.from_numpy(synth.gaussian_block(n, 14, 2).astype(np.float32)).cuda()
    kw = dict(V0=V0, guard=4, tol=1e-6, max_iters=3000)
    p = sped.transform("limit", 8)
    if case == "plain":
        p = None
    elif case == "limit_check3":
        kw["check_every"] = 3
    elif case == "mu_eg":
        kw.update(solver="mu_eg", eta=0.5, tol=0.0, max_iters=120)
    elif case == "bf16":
        kw["storage"] = "bf16"
    elif case == "stochastic_first":
        kw.update(stochastic_iters=5, walks_per_row=4, exact_terms=2)
    eager = sped.bottomk(L, 10, p, **kw)
    graph = sped.bottomk(L, 10, p, graphs=True, **kw)
    assert graph.stats["iters"] == eager.stats["iters"]
    assert graph.stats["spmm_count"] == eager.stats["spmm_count"]
    assert graph.converged == eager.converged
    np.testing.assert_array_equal(graph.evals, eager.evals)
    assert torch.equal(graph.V, eager.V)


# ------------------------------------------------------- edge-batch products
def _pinned(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).pin_memory()


@pytest.mark.parametrize("kind", ["sym", "combinatorial"])
@pytest.mark.parametrize("k,dt,batch", [(32, "f32", 4096), (7, "f32", 1000), (50, "f32", 3001),
                                        (64, "bf16", 7919), (300, "f32", 10 ** 6)])
def test_stream_laplacian_apply_parity(sped, kind, k, dt, batch):
    """Streamed sum_e x_e x_e^T X over a pinned host edge list (weights,
    repeats, self-loops, a degree-9000 hub) against the float64 oracle on the
    same node scales and the same (rounded) X: batches that leave a ragged
    tail, one batch for everything, 1, 2 and 4 columns per lane, two column
    tiles; the streamed degrees and scales against the oracle's."""
    from oracle import stream as ost
    _say(f"stream apply {kind} k={k} {dt} batch={batch}")
    n, src, dst, w = mixed_degree_graph()
    sh, dh, wh = _pinned(src, torch.int32), _pinned(dst, torch.int32), _pinned(w, torch.float32)
    deg, scale = sped.stream_node_scales(n, sh, dh, wh, kind=kind, batch=batch)
    okind = ost.SYM_NORMALIZED if kind == "sym" else ost.COMBINATORIAL
    d_r, s_r = ost.node_scales(n, src, dst, w, kind=okind)
    np.testing.assert_allclose(deg.cpu().numpy(), d_r, rtol=1e-12)
    np.testing.assert_allclose(scale.cpu().numpy(), s_r, rtol=2 * U32)
    tdt = torch.float32 if dt == "f32" else torch.bfloat16
    X = torch.from_numpy(synth.gaussian_block(n, k, 2).astype(np.float32)).to(tdt).cuda()
    sc = scale if kind == "sym" else None
    Y = sped.stream_laplacian_apply(n, sh, dh, X, wh, scale=sc, batch=batch)
    Xn = X.float().cpu().numpy().astype(np.float64)
    s64 = scale.cpu().numpy().astype(np.float64) if kind == "sym" else np.ones(n)
    Yr = ost.edge_batch_apply(n, src, dst, w, s64, Xn)
    err = np.abs(Y.cpu().numpy() - Yr).max() / np.abs(Yr).max()
    assert err < 1e-5, err


@pytest.mark.parametrize("k", [32, 8, 72])
def test_edge_apply_source_runs(sped, k):
    """The edge-batch product walks runs of consecutive edges and adds a
    source row once per run of equal sources: a source-sorted batch whose
    sources repeat 1 to 40 times (runs crossing the walkers' boundaries),
    with repeated pairs, self-loops and invalid edges (out-of-range endpoint,
    zero weight) inside runs, against the float64 oracle over the valid
    edges; every invalid edge counted once."""
    from oracle import stream as ost
    g = np.random.default_rng(k)
    n = 3000
    reps = g.integers(1, 41, 400)
    src = np.repeat(g.choice(n, 400, replace=False), reps)
    src.sort(kind="stable")
    dst = g.integers(0, n, src.shape[0])
    dst[::17] = src[::17]                      # self-loops
    dst[5::23] = dst[4::23][: dst[5::23].shape[0]]
    src[5::23] = src[4::23][: src[5::23].shape[0]]  # repeated pairs
    w = g.uniform(0.1, 1.0, src.shape[0]).astype(np.float32)
    bad_end = np.arange(3, src.shape[0], 41)
    bad_w = np.arange(7, src.shape[0], 53)
    bad_w = np.setdiff1d(bad_w, bad_end)
    dst_bad = dst.copy()
    dst_bad[bad_end] = n + 5
    w_bad = w.copy()
    w_bad[bad_w] = 0.0
    _say(f"edge apply source runs k={k} m={src.shape[0]}")
    scale = (1.0 / np.sqrt(g.uniform(1.0, 30.0, n))).astype(np.float32)
    X = torch.from_numpy(synth.gaussian_block(n, k, 3).astype(np.float32)).cuda()
    inv = torch.zeros(1, dtype=torch.int64, device="cuda")
    Y = sped.edge_apply(n, torch.from_numpy(src.astype(np.int32)).cuda(),
                        torch.from_numpy(dst_bad.astype(np.int32)).cuda(), X,
                        w=torch.from_numpy(w_bad).cuda(), scale=torch.from_numpy(scale).cuda(), alpha=0.5,
                        invalid=inv)
    assert int(inv.item()) == bad_end.shape[0] + bad_w.shape[0]
    ok = np.ones(src.shape[0], bool)
    ok[bad_end] = False
    ok[bad_w] = False
    Yr = 0.5 * ost.edge_batch_apply(n, src[ok], dst[ok], w[ok].astype(np.float64), scale.astype(np.float64),
                                    X.cpu().numpy().astype(np.float64))
    err = np.abs(Y.cpu().numpy() - Yr).max() / np.abs(Yr).max()
    assert err < 1e-5, err


def test_stream_apply_matches_resident_laplacian(sped):
    """The streamed L X equals the resident CSR path's L X (the sparse step
    with the monomial p(L) = L) on the same graph."""
    n, src, dst, w = mixed_degree_graph()
    sh, dh, wh = _pinned(src, torch.int32), _pinned(dst, torch.int32), _pinned(w, torch.float32)
    _, scale = sped.stream_node_scales(n, sh, dh, wh, kind="sym", batch=5000)
    L = sped.Laplacian(n, src, dst, w=w, kind="sym")
    X = torch.from_numpy(synth.gaussian_block(n, 32, 2).astype(np.float32)).cuda()
    Yc = sped.apply_poly(L, sped.monomial([0.0, 1.0]), X).cpu().numpy()
    Ys = sped.stream_laplacian_apply(n, sh, dh, X, wh, scale=scale, batch=5000).cpu().numpy()
    assert np.abs(Ys - Yc).max() <= 1e-5 * np.abs(Yc).max()


def test_stream_minibatch_accumulate_and_edge_cases(sped):
    """A drawn minibatch scaled by m / b against the oracle on that batch;
    accumulate adds to the block; m = 0 gives zeros (or leaves the block);
    an endpoint outside [0, n) or a zero weight is skipped and reported."""
    from oracle import stream as ost
    n, src, dst, w = mixed_degree_graph()
    m = len(src)
    sh, dh, wh = _pinned(src, torch.int32), _pinned(dst, torch.int32), _pinned(w, torch.float32)
    _, scale = sped.stream_node_scales(n, sh, dh, wh, kind="sym", batch=1 << 20)
    s64 = scale.cpu().numpy().astype(np.float64)
    X = torch.from_numpy(synth.gaussian_block(n, 16, 4).astype(np.float32)).cuda()
    Xn = X.cpu().numpy().astype(np.float64)
    idx = np.sort(np.random.default_rng(9).choice(m, m // 7, replace=False))
    alpha = m / len(idx)
    Y0 = torch.from_numpy(synth.gaussian_block(n, 16, 5).astype(np.float32)).cuda()
    Y = sped.stream_laplacian_apply(n, _pinned(src[idx], torch.int32), _pinned(dst[idx], torch.int32), X,
                                    _pinned(w[idx], torch.float32), scale=scale, alpha=alpha, out=Y0.clone(),
                                    accumulate=True, batch=999)
    Yr = Y0.cpu().numpy() + alpha * ost.edge_batch_apply(n, src[idx], dst[idx], w[idx], s64, Xn)
    assert np.abs(Y.cpu().numpy() - Yr).max() <= 1e-5 * np.abs(Yr).max()
    empty = torch.empty(0, dtype=torch.int32)
    Z = sped.stream_laplacian_apply(n, empty, empty, X, scale=scale)
    assert not Z.any()
    Z2 = sped.stream_laplacian_apply(n, empty, empty, X, scale=scale, out=Y0.clone(), accumulate=True)
    assert torch.equal(Z2, Y0)
    for bad_src, bad_w in ((n, 1.0), (-1, 1.0), (3, 0.0)):
        s2, d2, w2 = src.copy(), dst.copy(), w.copy()
        s2[100], w2[101] = bad_src, bad_w
        with pytest.raises(sped.SpedError) as ei:
            sped.stream_laplacian_apply(n, _pinned(s2, torch.int32), _pinned(d2, torch.int32), X,
                                        _pinned(w2, torch.float32), scale=scale, batch=4096)
        assert ei.value.status == sped.E_INVALID
    # the device-batch entry point counts the skipped edges
    s2 = src.copy()
    s2[[10, 20, 30]] = n + 5
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    Yd = sped.edge_apply(n, torch.from_numpy(s2.astype(np.int32)).cuda(), torch.from_numpy(dst.astype(np.int32)).cuda(),
                         X, w=torch.from_numpy(w.astype(np.float32)).cuda(), scale=scale, invalid=cnt)
    assert int(cnt.item()) == 3
    keep = np.ones(m, bool)
    keep[[10, 20, 30]] = False
    Ydr = ost.edge_batch_apply(n, src[keep], dst[keep], w[keep], s64, Xn)
    assert np.abs(Yd.cpu().numpy() - Ydr).max() <= 1e-5 * np.abs(Ydr).max()


def test_minibatch_oja_limit_polynomial_lowers_noise_floor(sped):
    """The edge-minibatch regime end to end on the 2,000-node SBM: Oja steps
    V <- orth(V + eta M V) where M V is estimated from streamed batches of
    2,000 of the 10,834 edges (scaled by m / b).  Plain M = 2I - L stalls at
    its noise floor; the limit polynomial (I - L/8)^8, one independent batch
    per factor (so the product stays unbiased), dilates the gap and settles
    several times lower.  The oracle runs the same batches in float64."""
    from oracle import solver as osol
    from oracle import stream as ost
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    m, b, eta, T = len(s), 2000, 0.5, 100
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    _, U, _ = osol.dense_bottom_k(ref.dense(), 10)
    sh, dh = _pinned(s, torch.int32), _pinned(d, torch.int32)
    _, scale = sped.stream_node_scales(n, sh, dh, kind="sym")
    s64 = scale.cpu().numpy().astype(np.float64)
    V0 = np.linalg.qr(np.random.default_rng(3).standard_normal((n, 10)))[0]

    def run(ell, gpu):
        g = np.random.default_rng(11)
        V = torch.from_numpy(V0.astype(np.float32)).cuda() if gpu else V0.copy()
        for _ in range(T):
            W = 2.0 * V if ell == 1 else V
            for _f in range(ell):
                idx = g.choice(m, b, replace=False)
                a = -(m / b) / (1.0 if ell == 1 else ell)
                if gpu:
                    W = sped.stream_laplacian_apply(n, _pinned(s[idx], torch.int32), _pinned(d[idx], torch.int32),
                                                    V if ell == 1 else W, scale=scale, alpha=a,
                                                    out=W.clone(), accumulate=True)
                else:
                    W = W + a * ost.edge_batch_apply(n, s[idx], d[idx], None, s64, V if ell == 1 else W)
            if gpu:
                V = sped.orthonormalize((V + eta * W).contiguous())
            else:
                V = np.linalg.qr(V + eta * W)[0]
        Vn = V.cpu().numpy().astype(np.float64) if gpu else V
        return osol.max_principal_angle(U, Vn)

    plain_gpu, limit_gpu = run(1, True), run(8, True)
    plain_ref, limit_ref = run(1, False), run(8, False)
    _say(f"minibatch Oja angles: plain {plain_gpu:.3f} (oracle {plain_ref:.3f}), "
         f"limit8 {limit_gpu:.3f} (oracle {limit_ref:.3f})")
    assert limit_ref < 0.06 and limit_gpu < 0.06
    assert plain_ref > 2 * limit_ref and plain_gpu > 2 * limit_gpu


@pytest.mark.parametrize("degree", [0, 8])
def test_minibatch_oja_solver_parity(sped, degree):
    """sped_minibatch_oja against the oracle's trajectory on the same drawn
    batches (runs of 2,000 of the 10,834 edges of the shuffled 2,000-node SBM
    list from Philox offsets, eta = 0.5, 100 steps, split over two calls that
    continue one batch stream): the float32 iterate stays within 1e-4 of the
    float64 one, and the limit polynomial ends several times closer to the
    bottom-10 subspace than the plain operator."""
    from oracle import solver as osol
    from oracle import stream as ost
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    perm = np.random.default_rng(5).permutation(len(s))
    s, d = s[perm], d[perm]
    m = len(s)
    sh, dh = _pinned(s, torch.int32), _pinned(d, torch.int32)
    _, scale = sped.stream_node_scales(n, sh, dh, kind="sym")
    s64 = scale.cpu().numpy().astype(np.float64)
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    _, U, _ = osol.dense_bottom_k(ref.dense(), 10)
    V0 = np.linalg.qr(np.random.default_rng(3).standard_normal((n, 10)))[0]
    V = torch.from_numpy(V0.astype(np.float32)).cuda()
    F = max(1, degree)
    sped.minibatch_oja(n, sh, dh, V, scale=scale, degree=degree, lambda_bound=2.0, batch=2000, eta=0.5,
                       iters=40, seed=23)
    sped.minibatch_oja(n, sh, dh, V, scale=scale, degree=degree, lambda_bound=2.0, batch=2000, eta=0.5,
                       iters=60, seed=23, batch0=40 * F)
    Vr = ost.minibatch_oja(n, s, d, None, s64, degree, 2.0, V0, batch=2000, eta=0.5, iters=100, seed=23)
    assert m > 2000
    Vg = V.cpu().numpy().astype(np.float64)
    drift = osol.max_principal_angle(Vg, Vr)
    ang = osol.max_principal_angle(U, Vg)
    _say(f"minibatch_oja degree {degree}: angle to bottom-10 {ang:.4f}, to the oracle trajectory {drift:.2e}")
    assert drift < 1e-4
    np.testing.assert_allclose(Vg.T @ Vg, np.eye(10), atol=1e-5)
    assert ang < (0.03 if degree == 8 else 0.12)
    if degree == 0:
        assert ang > 0.04   # the plain operator's noise floor sits above the limit polynomial's


def test_minibatch_oja_edge_cases(sped):
    """No steps leave V unchanged; a batch larger than the list and an
    endpoint outside [0, n) are rejected."""
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    sh, dh = _pinned(s, torch.int32), _pinned(d, torch.int32)
    V0 = torch.from_numpy(np.linalg.qr(np.random.default_rng(3).standard_normal((n, 6)))[0].astype(np.float32)).cuda()
    V = V0.clone()
    sped.minibatch_oja(n, sh, dh, V, degree=4, batch=100, iters=0)
    assert torch.equal(V, V0)
    with pytest.raises(sped.SpedError) as ei:
        sped.minibatch_oja(n, sh, dh, V, degree=4, batch=len(s) + 1, iters=1)
    assert ei.value.status == sped.E_INVALID
    bad = s.copy()
    bad[5] = n
    with pytest.raises(sped.SpedError) as ei:
        sped.minibatch_oja(n, _pinned(bad, torch.int32), dh, V.clone(), degree=0, batch=1000, iters=2)
    assert ei.value.status == sped.E_INVALID


@pytest.mark.parametrize("case", ["sbm125_limit16", "hub_taylor5", "sbm_degree1", "sbm_degree2_tail"])
def test_blocked_chain_parity(sped, case):
    """sped_apply_poly_blocked (two fused steps per launch on LDS-resident row
    blocks) against the oracle's chain and against the single-step chain:
    a community-ordered SBM with blocks of 125 rows (block_rows 125, 95% of
    neighbours inside the block), the weighted hub graph with blocks that
    ignore its structure (most neighbours outside: the recompute path, an odd
    degree ending with one single step, Horner terms g X), degree 1 and 2, and
    a last block shorter than block_rows."""
    _say(f"blocked chain {case}")
    if case == "hub_taylor5":
        n, s, d, w = mixed_degree_graph()
        L = sped.Laplacian(n, s, d, w, kind="sym")
        ref = olap.laplacian(n, s, d, w, kind=olap.SYM_NORMALIZED)
        k, B, p, op = 8, 300, sped.transform("taylor_exp", 5), opoly.taylor_exp(5)
    else:
        n, s, d, _ = synth.sbm_from_degrees(25_000, 200, 19.0, 1.0, seed=3)
        L = sped.Laplacian(n, s, d, kind="sym")
        ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
        deg = {"sbm125_limit16": 16, "sbm_degree1": 1, "sbm_degree2_tail": 2}[case]
        k, B = 32, (125 if case != "sbm_degree2_tail" else 333)
        p, op = sped.transform("limit", deg), opoly.limit_exp(deg)
    X = synth.gaussian_block(n, k, 5).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    Y = sped.apply_poly_blocked(L, p, Xd, B).cpu().numpy()
    Y1 = sped.apply_poly(L, p, Xd).cpu().numpy()
    Yr = opoly.apply_terms(ref.L, op, X.astype(np.float64))
    assert _rel(Y, Yr) < 3e-5
    assert np.abs(Y - Yr).max() < 2e-4 * np.abs(Yr).max()
    # the same arithmetic as the single-step chain up to the order of the sums
    assert _rel(Y, Y1) < 1e-5


def test_stochastic_counter_base_and_check_log(sped, tmp_path):
    """counter_base shifts the walk counters of the random iterations (a
    resumed solve draws fresh walks; the same base repeats them bit for bit;
    counters past 2^32 are refused), and log_path writes one JSON line per
    check plus the result."""
    import json
    _say("solver counter_base and per-check log")
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    V0 = torch.from_numpy(synth.gaussian_block(n, 14, 2).astype(np.float32)).cuda()
    p = sped.transform("limit", 8)
    kw = dict(V0=V0, guard=4, tol=0.0, max_iters=5, stochastic_iters=5, walks_per_row=4)
    a = sped.bottomk(L, 10, p, counter_base=0, **kw).V
    b = sped.bottomk(L, 10, p, counter_base=0, **kw).V
    c = sped.bottomk(L, 10, p, counter_base=7, **kw).V
    assert torch.equal(a, b)
    assert not torch.equal(a, c)
    with pytest.raises(sped.SpedError) as e:
        sped.bottomk(L, 10, p, counter_base=(1 << 32) - 3, **kw)
    assert e.value.status == sped.E_INVALID
    log = tmp_path / "checks.jsonl"
    r = sped.bottomk(L, 10, p, V0=V0, guard=4, tol=1e-6, max_iters=300, log_path=str(log))
    lines = [json.loads(x) for x in log.read_text().splitlines()]
    assert len(lines) == r.stats["iters"] + 1  # check_every = 1
    assert lines[-1]["result"]["converged"] == 1
    assert lines[-2]["bound"] == r.stats["bound"] <= 1e-6


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_rank_deficient_start_block_reseeded(sped, storage):
    """A start block with a repeated column and a zero column: those columns
    are replaced by random ones before the first iteration (counted in the
    stats) and the solve reaches the dense-eigh subspace; a start block with
    a NaN is refused with SPED_E_NUMERIC."""
    _say(f"rank-deficient start block, storage {storage}")
    n, s, d, _ = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    lam, U, _ = osol.dense_bottom_k(ref.dense(), 10)
    V0 = synth.gaussian_block(n, 14, 2).astype(np.float32)
    V0[:, 3] = V0[:, 1]
    V0[:, 7] = 0.0
    r = sped.bottomk(L, 10, sped.transform("limit", 8), V0=torch.from_numpy(V0).cuda(), guard=4, tol=1e-6,
                     max_iters=3000, storage=storage)
    assert r.stats["reseeded"] == 2
    assert r.converged
    assert osol.max_principal_angle(U, r.V.cpu().numpy().astype(np.float64)) <= 1e-6
    V0[5, 2] = np.nan
    with pytest.raises(sped.SpedError) as e:
        sped.bottomk(L, 10, sped.transform("limit", 8), V0=torch.from_numpy(V0).cuda(), guard=4, tol=1e-6,
                     max_iters=10)
    assert e.value.status == sped.E_NUMERIC
