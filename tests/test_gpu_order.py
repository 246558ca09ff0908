"""GPU parity of the node orders and the ordered build against the oracle
(run on an MI355X; marked gpu).

Orders are integer work: the device order must equal the oracle's exactly.
The ordered build is compared with the oracle's Laplacian of the relabelled
edge list (structure exactly, values to 2u as for the plain build), and
p(L)V on it, with V's rows permuted alike, with the oracle's p(L)V on the
original ids (the p(L)X tolerance of the plain parity tests)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import laplacian as olap
from oracle import order as oorder
from oracle import poly as opoly
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


def graph(case):
    """Seeded graphs spanning the order's cases: several components and
    isolated nodes, a hub above the medium bound, a deep grid."""
    if case == "sbm_disconnected":
        n, s, d, _ = synth.sbm_sparse([300, 500, 400], 0.03, 0.0, seed=2)
        return n + 7, s, d  # 7 isolated nodes at the end
    if case == "powerlaw":
        n, s, d, _ = synth.chung_lu(20000, 2.1, 8.0, 16, 0.8, seed=3)
        return n, s, d
    if case == "grid":
        return synth.three_room_grid(4, 10)
    if case == "rmat_hub":
        n, s, d = synth.rmat(14, 8, 0.57, 0.19, 0.19, seed=4)
        g = np.random.default_rng(4)
        hub = g.choice(np.arange(1, n), 9000, replace=False)  # a row above the medium bound
        return n, np.concatenate([s, np.zeros(9000, np.int64)]), np.concatenate([d, hub])
    if case == "forest":
        g = np.random.default_rng(11)
        n = 3000
        s = np.arange(1, 2500)
        d = g.integers(0, s)
        keep = g.random(s.shape[0]) < 0.9
        return n, s[keep], d[keep]
    if case == "edgeless":
        return 5, np.zeros(0, np.int64), np.zeros(0, np.int64)
    if case == "single_edge":
        return 2, np.array([1]), np.array([0])
    raise ValueError(case)


CASES = ["sbm_disconnected", "powerlaw", "grid", "rmat_hub", "forest", "edgeless", "single_edge"]


def oracle_order(method, n, rowptr, col):
    if method == "cuthill_mckee":
        return oorder.cuthill_mckee(n, rowptr, col)
    if method == "degree":
        return oorder.degree_order(n, rowptr)
    return oorder.label_order(n, rowptr, col)


METHODS = ["cuthill_mckee", "degree", "label_propagation"]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("method", METHODS)
def test_locality_order_matches_oracle(sped, case, method):
    n, s, d = graph(case)
    _say(f"locality order {method} {case} n={n} m={s.shape[0]}")
    L = sped.Laplacian(n, s, d, kind="sym")
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    rowptr, col, _ = ref.adjacency()
    got = sped.locality_order(L, method).cpu().numpy()
    np.testing.assert_array_equal(got, oracle_order(method, n, rowptr, col))


@pytest.mark.parametrize("case,lcc,kind", [("powerlaw", True, "sym"), ("rmat_hub", False, "combinatorial"),
                                           ("sbm_disconnected", True, "combinatorial"), ("grid", False, "sym"),
                                           ("forest", True, "sym")])
@pytest.mark.parametrize("method", METHODS)
def test_ordered_build_is_the_relabelled_laplacian(sped, case, lcc, kind, method):
    n, s, d = graph(case)
    w = synth.random_weights(s.shape[0], 8).astype(np.float32).astype(np.float64)
    okind = olap.SYM_NORMALIZED if kind == "sym" else olap.COMBINATORIAL
    _say(f"ordered build {method} {case} lcc={lcc} kind={kind}")
    L = sped.Laplacian(n, s, d, w, kind=kind, lcc=lcc, order=method)
    base = olap.laplacian(n, s, d, w, kind=okind, lcc=lcc)
    rowptr0, col0, _ = base.adjacency()
    pos = oracle_order(method, base.n, rowptr0, col0)
    # the kept component's edges, in its own ids, relabelled by the order
    keep_id = -np.ones(n, np.int64)
    keep_id[base.old_of_new] = np.arange(base.n)
    a, b = keep_id[s], keep_id[d]
    inside = (a >= 0) & (b >= 0)
    s2, d2 = oorder.relabel_edges(a[inside], b[inside], pos)
    ref = olap.laplacian(base.n, s2, d2, w[inside], kind=okind)
    assert L.n == ref.n and L.nnz == ref.adjacency()[1].shape[0]
    rowptr, col, val, diag, scale = L.host_csr()
    r_rowptr, r_col, _ = ref.adjacency()
    np.testing.assert_array_equal(rowptr, r_rowptr)
    np.testing.assert_array_equal(col, r_col)
    old = np.empty(base.n, np.int64)
    old[pos] = base.old_of_new
    np.testing.assert_array_equal(L.old_of_new.cpu().numpy(), old)
    import scipy.sparse as sp
    S = sp.csr_matrix((val.astype(np.float64), col, rowptr), shape=(L.n, L.n))
    Lg = sp.diags(diag.astype(np.float64)) - S
    assert abs(Lg - ref.L).max() <= 2 * U32 * abs(ref.L).max()
    # the operator is the same up to the permutation: p(L)V on the ordered
    # rows equals the oracle's p(L)V on the original ids, rows permuted alike
    k = 8
    X = synth.gaussian_block(base.n, k, 5)
    Xo = X[np.argsort(pos)]  # row j of the ordered block is the node placed at j
    # the degree-16 limit row in Lt = L / (lambda_bound / 2), whose spectrum
    # lies in [0, 2] for both Laplacians
    c, half = opoly.limit_exp(16).coeffs, base.lambda_bound / 2
    Y = sped.apply_poly(L, sped.monomial(c, 0.0, half),
                        torch.from_numpy(Xo.astype(np.float32)).cuda()).cpu().numpy().astype(np.float64)
    Yr = opoly.apply_terms(base.L, opoly.Poly(c, 0.0, half), X.astype(np.float32).astype(np.float64))
    Yr = Yr[np.argsort(pos)]
    assert np.linalg.norm(Y - Yr) / max(np.linalg.norm(Yr), 1e-300) < 3e-5
    assert np.abs(Y - Yr).max() <= 2e-4 * max(np.abs(Yr).max(), 1e-30)


def test_ordered_build_edge_cases(sped):
    _say("ordered build: empty graph, self-loops only, invalid endpoint (all methods)")
    L = sped.Laplacian(6, [], [], kind="sym", order="cuthill_mckee")
    assert L.n == 6 and L.nnz == 0
    np.testing.assert_array_equal(L.old_of_new.cpu().numpy(), np.arange(6))
    L = sped.Laplacian(4, [1, 2], [1, 2], kind="combinatorial", order="degree")
    assert L.nnz == 0
    L = sped.Laplacian(0, [], [], order="cuthill_mckee")
    assert L.n == 0
    with pytest.raises(sped.SpedError):
        sped.Laplacian(4, [0, 5], [1, 2], order="cuthill_mckee")
    # lcc of an edgeless graph keeps one node
    L = sped.Laplacian(5, [], [], lcc=True, order="cuthill_mckee")
    assert L.n == 1
    # label propagation on the same degenerate inputs
    L = sped.Laplacian(6, [], [], kind="sym", order="label_propagation")
    assert L.n == 6 and L.nnz == 0
    np.testing.assert_array_equal(L.old_of_new.cpu().numpy(), np.arange(6))
    L = sped.Laplacian(4, [1, 2], [1, 2], kind="combinatorial", order="label_propagation")
    assert L.nnz == 0
    L = sped.Laplacian(0, [], [], order="label_propagation")
    assert L.n == 0
    with pytest.raises(sped.SpedError):
        sped.Laplacian(4, [0, 5], [1, 2], order="label_propagation")


@pytest.mark.parametrize("method", METHODS)
def test_solve_on_ordered_laplacian(sped, method):
    """The bottom-10 span solved on a Laplacian numbered by each order,
    mapped back through old_of_new, is the dense-eigh span of the original
    graph (SBM n=2000, 10 blocks, plus an isolated pair outside the largest
    component), and k-means labels map back the same way."""
    from oracle import kmeans as okm
    from oracle import solver as osol
    n, s, d, labels = synth.sbm_bernoulli([200] * 10, 0.05, 0.0005, seed=1)
    s = np.concatenate([s, [n]])
    d = np.concatenate([d, [n + 1]])
    n_all = n + 2
    _say(f"bottom-10 solve on the {method}-ordered Laplacian, mapped back")
    L = sped.Laplacian(n_all, s, d, kind="sym", lcc=True, order=method)
    base = olap.laplacian(n_all, s, d, kind=olap.SYM_NORMALIZED, lcc=True)
    assert L.n == base.n == n
    lam, U, _ = osol.dense_bottom_k(base.dense(), 10)
    oon = L.old_of_new.long().cpu().numpy()          # original id of each ordered row
    pos = np.empty(base.n, np.int64)
    pos[np.searchsorted(base.old_of_new, oon)] = np.arange(L.n)  # ordered row of each kept node
    k, guard = 10, 4
    V0 = synth.gaussian_block(n, k + guard, 2).astype(np.float32)
    V0o = torch.from_numpy(V0[np.argsort(pos)]).cuda()
    r = sped.bottomk(L, k, sped.transform("limit", 8), V0=V0o, guard=guard, tol=1e-6, max_iters=3000)
    assert r.converged, r.stats
    Vback = r.V.cpu().numpy().astype(np.float64)[pos]
    ang = osol.max_principal_angle(U, Vback)
    assert ang <= 1e-6, (ang, r.stats)
    np.testing.assert_allclose(r.evals[1:], lam[1:], rtol=1e-6)
    lab, _, _, _ = sped.cluster_embed(r.V, 10, seed=1)
    lab_back = lab.cpu().numpy()[pos]
    assert okm.adjusted_rand_index(lab_back, labels) > 0.99
