"""sped_apply_poly_noalloc (the allocation-free form of sped_apply_poly, for
callers that cannot allocate device memory) against sped_apply_poly on the
same inputs, through the C ABI: the two share every kernel, so the outputs
must agree bit for bit; the float64 oracle bounds both.  Two calls in a row,
the second on a smaller graph and block, so the second reads nothing the
first left in the library's scratch.  Sizes beyond the scratch are refused
before any launch."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


def _hub_graph(seed=5):
    """SBM rows plus a 9,000-edge hub (heavy bin) and two 300-edge hubs
    (medium bin), weighted."""
    n0, s, d, _ = synth.sbm_bernoulli([700, 900, 1400], 0.01, 0.0008, seed=seed)
    n = 12000
    g = np.random.default_rng(seed)
    src = np.concatenate([s, np.zeros(9000, dtype=np.int64), np.repeat([17, 1200], 300), g.integers(3000, n, 20000)])
    dst = np.concatenate([d, g.choice(np.arange(1, n), 9000, replace=False), g.integers(3000, n, 600),
                          g.integers(3000, n, 20000)])
    w = synth.random_weights(src.shape[0], seed + 1).astype(np.float32).astype(np.float64)
    return n, src, dst, w


def _same_call(sped, L, p, X, out_dtype):
    """Run both entry points on the same inputs; return (noalloc, workspace) outputs."""
    Y1 = torch.full((L.n, X.shape[1]), float("nan"), dtype=out_dtype, device=X.device)
    sped.apply_poly_noalloc(L, p, X, Y1)
    Y2 = sped.apply_poly(L, p, X, out_dtype=out_dtype)
    torch.cuda.synchronize()
    return Y1, Y2


def test_noalloc_matches_workspace_entry_point(sped):
    # call 1: 60,000-node SBM, 32 float32 columns, (I - L/16)^16 (two scratch blocks)
    n, s, d, _ = synth.sbm_bernoulli([6000] * 10, 0.003, 0.00002, seed=11)
    _say(f"noalloc call 1: SBM n={n} k=32 limit 16 f32")
    L = sped.Laplacian(n, s, d, kind="sym")
    X = synth.gaussian_block(n, 32, 4).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    Y1, Y2 = _same_call(sped, L, sped.transform("limit", 16), Xd, torch.float32)
    assert torch.equal(Y1, Y2)
    ref = olap.laplacian(n, s, d, kind=olap.SYM_NORMALIZED)
    Yr = opoly.apply_limit_product(ref.L, 16, X.astype(np.float64))
    assert np.linalg.norm(Y1.cpu().numpy() - Yr) <= 3e-5 * np.linalg.norm(Yr)

    # call 2, smaller: 12,000-node hub graph (all three row bins), 8 bf16
    # columns, degree-7 Taylor series of -exp(-L) by Horner, bf16 output
    n, s, d, w = _hub_graph()
    _say(f"noalloc call 2: hub graph n={n} k=8 taylor_exp 7 bf16")
    L = sped.Laplacian(n, s, d, w, kind="sym")
    X = synth.gaussian_block(n, 8, 5).astype(np.float32)
    Xb = torch.from_numpy(X).cuda().to(torch.bfloat16)
    Y1, Y2 = _same_call(sped, L, sped.transform("taylor_exp", 7), Xb, torch.bfloat16)
    assert torch.equal(Y1.view(torch.int16), Y2.view(torch.int16))
    ref = olap.laplacian(n, s, d, w, kind=olap.SYM_NORMALIZED)
    Yr = opoly.apply_terms(ref.L, opoly.taylor_exp(7), Xb.float().cpu().numpy().astype(np.float64))
    # bf16 output: one rounding of at most 2^-9 relative on top of the float32 chain
    err = np.abs(Y1.float().cpu().numpy() - Yr)
    assert np.all(err <= 2.0 ** -8 * np.abs(Yr) + 1e-5 * np.abs(Yr).max())


@pytest.mark.parametrize("degree", [1, 2])
def test_noalloc_low_degrees(sped, degree):
    """Degree 1 needs no scratch block and degree 2 one."""
    n, s, d, _ = synth.sbm_bernoulli([500] * 4, 0.02, 0.001, seed=3)
    _say(f"noalloc degree {degree}")
    L = sped.Laplacian(n, s, d, kind="sym")
    X = torch.from_numpy(synth.gaussian_block(n, 12, 6).astype(np.float32)).cuda()
    Y1, Y2 = _same_call(sped, L, sped.transform("limit", degree), X, torch.float32)
    assert torch.equal(Y1, Y2)


def test_noalloc_rejects_blocks_beyond_scratch(sped):
    """n k above the static scratch returns SPED_E_WORKSPACE and launches
    nothing (the output keeps its contents)."""
    n = 300_000  # a path graph
    L = sped.Laplacian(n, np.arange(n - 1), np.arange(1, n), kind="sym")
    k = 32  # 300,000 x 32 floats per block: two blocks exceed 64 MiB
    _say(f"noalloc oversize n={n} k={k}")
    X = torch.zeros(n, k, device="cuda")
    Y = torch.full((n, k), 7.0, device="cuda")
    with pytest.raises(sped.SpedError) as e:
        sped.apply_poly_noalloc(L, sped.transform("limit", 4), X, Y)
    assert e.value.status == sped.E_WORKSPACE
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((Y == 7.0).all())
    # degree 2 needs one block only, which fits
    sped.apply_poly_noalloc(L, sped.transform("limit", 2), X, Y)
    torch.cuda.synchronize()
    assert bool((Y == 0.0).all())
