"""The C-ABI library loads, exports every symbol include/sped.h declares, and
its host-only logic (argument validation, Table 2 coefficients) behaves; no
GPU needed."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import poly as opoly
from paper_2207_14589_amd import sped

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sped.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sped_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sped.LIB_PATH):
        pytest.fail("libsped.so is not built (run python -m paper_2207_14589_amd.build)")
    return sped.lib()


def test_every_declared_symbol_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(sped.SIGNATURES), "binding and header disagree"


def test_version_and_error_string(lib):
    assert lib.sped_version() == 10000
    assert lib.sped_last_error() == b""


def test_transform_coeffs_match_table2(lib):
    lam = 2.0
    for ell in (3, 8, 16, 251):
        np.testing.assert_allclose(sped.transform("limit", ell, lam, product_form=False).coeffs,
                                   opoly.limit_exp(ell).coeffs, rtol=1e-14, atol=1e-300)
        np.testing.assert_allclose(sped.transform("taylor_exp", ell, lam).coeffs, opoly.taylor_exp(ell).coeffs,
                                   rtol=1e-14, atol=1e-320)
    for ell in (3, 9, 15):
        t = sped.transform("taylor_log", ell, lam, eps=1e-3)
        o = opoly.taylor_log(ell, lam, 1e-3)
        np.testing.assert_allclose(t.coeffs, o.coeffs, rtol=1e-13)
        assert t.shift == pytest.approx(o.shift)
    np.testing.assert_allclose(sped.transform("plain", 1, 3.5).coeffs, [3.5, -1.0])


@pytest.mark.parametrize("ell", [2, 8, 16])
def test_even_taylor_log_rejected(lib, ell):
    """Table 2 takes l odd: the even-degree log series is not increasing on
    [0, 2] (the oracle's test_even_log_not_monotone), so it is refused."""
    out = np.zeros(ell + 1)
    sh, sc = ctypes.c_double(), ctypes.c_double()
    assert lib.sped_transform_coeffs(sped.T_TAYLOR_LOG, ell, 2.0, 1e-3,
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     ctypes.byref(sh), ctypes.byref(sc)) == sped.E_UNSUPPORTED
    assert b"odd" in lib.sped_last_error()


@pytest.mark.parametrize("shift,scale", [(1.0, 1.0), (0.5, 2.0), (0.0, 1.0)])
def test_poly_rebase(lib, shift, scale):
    """Rebased coefficients evaluate to the same polynomial: sum_i out_i
    ((lam - shift)/scale)^i against the oracle's Table 2 rows on [0, 2]."""
    lam = np.linspace(0.0, 2.0, 41)
    y = (lam - shift) / scale
    for spec, ref in ((sped.transform("limit", 12), opoly.limit_exp(12)),
                      (sped.transform("taylor_log", 7, 2.0), opoly.taylor_log(7, 2.0)),
                      (sped.transform("taylor_exp", 9), opoly.taylor_exp(9))):
        c = spec.rebase(shift, scale)
        np.testing.assert_allclose(np.polynomial.polynomial.polyval(y, c), ref(lam), rtol=1e-11, atol=1e-12)


def test_monomial_expansion(lib):
    t = sped.transform("taylor_log", 7, 2.0)
    np.testing.assert_allclose(t.monomial(), opoly.monomial_in_L(opoly.taylor_log(7, 2.0)), rtol=1e-11, atol=1e-12)
    lim = sped.transform("limit", 16, 2.0, product_form=True)
    np.testing.assert_allclose(lim.monomial(), opoly.limit_exp(16).coeffs, rtol=1e-13, atol=1e-300)


def test_invalid_arguments_rejected_on_host(lib):
    need = ctypes.c_size_t(0)
    # NULL csr
    st = lib.sped_apply_poly(None, None, 4, None, 4, 0, None, 4, 0, None, ctypes.byref(need), None)
    assert st == sped.E_INVALID
    assert b"csr" in lib.sped_last_error()
    # degree 0 polynomial
    c = sped.CSR()
    c.n, c.nnz, c.kind = 0, 0, sped.SYM_NORMALIZED
    p = sped.Poly()
    p.kind, p.degree = sped.POLY_MONOMIAL, 0
    st = lib.sped_apply_poly(ctypes.byref(c), ctypes.byref(p), 4, None, 4, 0, None, 4, 0, None, ctypes.byref(need),
                             None)
    assert st == sped.E_INVALID
    # bad transform degree for plain
    out = np.zeros(3)
    sh, sc = ctypes.c_double(), ctypes.c_double()
    assert lib.sped_transform_coeffs(sped.T_PLAIN, 2, 2.0, 0.0, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     ctypes.byref(sh), ctypes.byref(sc)) == sped.E_INVALID
    # stochastic counter out of range, unsupported rejection dtype
    coef = np.array([1.0, 0.5])
    cp = coef.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    c.n = 0
    assert lib.sped_apply_poly_stochastic(ctypes.byref(c), cp, 1, 4, None, 4, 0, None, 4, 0, 0, 8, 1, 1 << 33, None,
                                          None, ctypes.byref(need), None) == sped.E_INVALID
    assert lib.sped_apply_poly_stochastic(ctypes.byref(c), cp, 1, 4, None, 4, 0, None, 4, 1, 1, 8, 1, 0, None,
                                          None, ctypes.byref(need), None) == sped.E_UNSUPPORTED
    # lazy walk: ell outside [1, 255]; combinatorial with ell below the largest degree
    assert lib.sped_apply_limit_lazy(ctypes.byref(c), 0, 4, None, 4, 0, None, 4, 0, 8, 1, 0, None,
                                     ctypes.byref(need), None) == sped.E_INVALID
    cc = sped.CSR()
    cc.n, cc.nnz, cc.kind, cc.lambda_bound = 0, 0, sped.COMBINATORIAL, 40.0
    assert lib.sped_apply_limit_lazy(ctypes.byref(cc), 16, 4, None, 4, 0, None, 4, 0, 8, 1, 0, None,
                                     ctypes.byref(need), None) == sped.E_INVALID
    assert b"largest weighted degree" in lib.sped_last_error()
    assert lib.sped_apply_limit_lazy(ctypes.byref(cc), 20, 4, None, 4, 0, None, 4, 0, 8, 1, 0, None,
                                     ctypes.byref(need), None) == sped.OK
    # orthonormalize: k > n
    assert lib.sped_orthonormalize(3, 5, None, 5, 0, 2, None, None, ctypes.byref(need), None) == sped.E_INVALID
    # cluster: too many clusters
    assert lib.sped_cluster_embed(None, 10, 2, 2, 0, 11, 1, 0, 10, None, None, None, None, None, None,
                                  ctypes.byref(need), None) == sped.E_INVALID


def test_workspace_size_query_without_device(lib):
    """Size queries are pure host arithmetic."""
    c = sped.CSR()
    c.n, c.nnz, c.kind = 1000, 8000, sped.SYM_NORMALIZED
    c.rowptr = c.diag = c.scale = c.col = c.val = 16
    p = sped.transform("limit", 16).struct()
    need = ctypes.c_size_t(0)
    st = lib.sped_apply_poly(ctypes.byref(c), ctypes.byref(p), 32, 256, 32, 0, 512, 32, 0, None,
                             ctypes.byref(need), None)
    assert st == sped.OK and need.value >= 2 * 1000 * 32 * 4
    need2 = ctypes.c_size_t(0)
    assert lib.sped_gram(1000, 32, 32, 256, 32, 256, 32, 0, 512, None, ctypes.byref(need2), None) == sped.OK
    assert need2.value > 0
    small = ctypes.c_size_t(16)
    ws = ctypes.create_string_buffer(1024)
    aligned = (ctypes.addressof(ws) + 255) // 256 * 256
    assert lib.sped_gram(1000, 32, 32, 256, 32, 256, 32, 0, 512, aligned, ctypes.byref(small), None) == \
        sped.E_WORKSPACE


def test_hybrid_validation(lib):
    """exact_terms outside [0, degree]; the exact split (m = degree) needs no
    walk records; X and Y may not overlap."""
    c = sped.CSR()
    c.n, c.nnz, c.kind = 0, 0, sped.SYM_NORMALIZED
    coeffs = (ctypes.c_double * 5)(0.5, -0.5, 0.25, -0.1, 0.05)
    need = ctypes.c_size_t(0)
    for m in (-1, 5):
        assert lib.sped_apply_poly_hybrid(ctypes.byref(c), coeffs, 4, m, 8, None, 8, 0, None, 8, 0, 0, 4, 1, 0,
                                          None, ctypes.byref(need), None) == sped.E_INVALID
        assert b"exact_terms" in lib.sped_last_error()
    c.n, c.nnz = 100, 400
    c.rowptr = c.diag = c.scale = c.col = c.val = c.bins = 16
    assert lib.sped_apply_poly_hybrid(ctypes.byref(c), coeffs, 4, 2, 8, 256, 8, 0, 512, 8, 0, 0, 4, 1, 0,
                                      None, ctypes.byref(need), None) == sped.E_INVALID
    assert b"walk records" in lib.sped_last_error()
    assert lib.sped_apply_poly_hybrid(ctypes.byref(c), coeffs, 4, 4, 8, 256, 8, 0, 512, 8, 0, 0, 4, 1, 0,
                                      None, ctypes.byref(need), None) == sped.OK
    assert need.value >= 2 * 100 * 8 * 4
    assert lib.sped_apply_poly_hybrid(ctypes.byref(c), coeffs, 4, 1, 8, 256, 8, 0, 512, 8, 0, 0, 4, 1, 0,
                                      None, ctypes.byref(need), None) == sped.E_INVALID
    c.wentry = c.wnode = 16
    assert lib.sped_apply_poly_hybrid(ctypes.byref(c), coeffs, 4, 1, 8, 256, 8, 0, 512, 8, 0, 0, 4, 1, 0,
                                      None, ctypes.byref(need), None) == sped.OK
    assert 100 * 8 * 4 <= need.value < 2 * 100 * 8 * 4
    ws = ctypes.create_string_buffer(need.value + 512)
    aligned = (ctypes.addressof(ws) + 255) // 256 * 256
    assert lib.sped_apply_poly_hybrid(ctypes.byref(c), coeffs, 4, 1, 8, 4096, 8, 0, 4096 + 64, 8, 0, 0, 4, 1,
                                      0, aligned, ctypes.byref(need), None) == sped.E_INVALID
    assert b"overlap" in lib.sped_last_error()


def test_gather_probe_validation(lib):
    need_out = 16
    assert lib.sped_gather_probe(None, 128, 8, 1, 1, need_out, None) == sped.E_INVALID
    assert lib.sped_gather_probe(256, 100, 8, 1, 1, need_out, None) == sped.E_INVALID   # not a power of two
    assert lib.sped_gather_probe(256, 128, 12, 1, 1, need_out, None) == sped.E_INVALID  # iters not a multiple of 8
    assert lib.sped_gather_probe(256, 128, 8, 1, 0, need_out, None) == sped.E_INVALID   # no blocks
    assert lib.sped_gather_probe(260, 128, 8, 1, 1, need_out, None) == sped.E_INVALID   # misaligned table


def test_edge_batch_validation(lib):
    """Argument checks of the edge-batch entry points run on the host, before
    any device work; the streamed calls answer a workspace size query."""
    X, Y, s, d = 4096, 8192, 1024, 2048   # fake, never dereferenced
    f = lib.sped_edge_apply
    assert f(10, 5, s, d, None, None, 0, X, 4, sped.F32, Y, 4, 1.0, None, None) == sped.E_INVALID        # k < 1
    assert f(10, 5, s, d, None, None, 4, X, 3, sped.F32, Y, 4, 1.0, None, None) == sped.E_INVALID        # ldx < k
    assert f(10, 5, s, d, None, None, 4, X, 4, sped.F64, Y, 4, 1.0, None, None) == sped.E_UNSUPPORTED    # dtype
    assert f(10, 5, None, d, None, None, 4, X, 4, sped.F32, Y, 4, 1.0, None, None) == sped.E_INVALID     # src NULL
    assert f(10, 5, s, d, None, None, 4, X, 4, sped.F32, X, 4, 1.0, None, None) == sped.E_INVALID        # Y = X
    assert f(10, 5, s, d, None, None, 4, X, 4, sped.F32, Y, 4, float("nan"), None, None) == sped.E_INVALID
    assert f(10, -1, s, d, None, None, 4, X, 4, sped.F32, Y, 4, 1.0, None, None) == sped.E_INVALID       # m < 0
    need = ctypes.c_size_t(0)
    g = lib.sped_stream_laplacian_apply
    assert g(10, 100, s, d, None, None, 4, X, 4, sped.F32, Y, 4, 1.0, 0, 0, None, ctypes.byref(need),
             None) == sped.E_INVALID                                                                    # batch < 1
    assert g(10, 100, s, d, None, None, 4, X, 4, sped.F32, Y, 4, 1.0, 0, 64, None, ctypes.byref(need),
             None) == sped.OK
    assert need.value >= 2 * 64 * 12   # two staging batches of (src, dst, w)
    h = lib.sped_stream_node_scales
    assert h(10, 100, s, d, None, 7, 64, Y, X, None, ctypes.byref(need), None) == sped.E_INVALID         # kind
    assert h(10, 100, s, d, None, sped.SYM_NORMALIZED, 64, None, X, None, ctypes.byref(need),
             None) == sped.E_INVALID                                                                    # degree NULL
    assert h(10, 100, s, d, None, sped.SYM_NORMALIZED, 64, Y, X, None, ctypes.byref(need), None) == sped.OK


def test_minibatch_oja_validation(lib):
    """Host checks of the minibatch solver, and its workspace size query (two
    staging batches, two n x k float blocks and the orthonormalisation's)."""
    s, d, V = 1024, 2048, 4096   # fake, never dereferenced
    f = lib.sped_minibatch_oja
    need = ctypes.c_size_t(0)
    q = ctypes.byref(need)
    assert f(100, 50, s, d, None, None, 8, 2.0, 10, V, 10, 51, 0.5, 3, 0, 0, None, q, None) == sped.E_INVALID  # batch > m
    assert f(100, 50, s, d, None, None, 8, 2.0, 97, V, 97, 10, 0.5, 3, 0, 0, None, q, None) == sped.E_UNSUPPORTED
    assert f(100, 50, s, d, None, None, 8, 2.0, 10, V, 9, 10, 0.5, 3, 0, 0, None, q, None) == sped.E_INVALID   # ldv < k
    assert f(100, 50, s, d, None, None, 0, 0.0, 10, V, 10, 10, 0.5, 3, 0, 0, None, q, None) == sped.E_INVALID  # lambda
    assert f(100, 50, s, d, None, None, 8, 2.0, 10, V, 10, 10, 0.0, 3, 0, 0, None, q, None) == sped.E_INVALID  # eta
    assert f(100, 50, s, d, None, None, -1, 2.0, 10, V, 10, 10, 0.5, 3, 0, 0, None, q, None) == sped.E_INVALID  # degree
    assert f(100, 0, s, d, None, None, 8, 2.0, 10, V, 10, 10, 0.5, 3, 0, 0, None, q, None) == sped.E_INVALID   # m = 0
    assert f(100, 50, s, d, None, None, 8, 2.0, 10, V, 10, 10, 0.5, 3, 0, -1, None, q, None) == sped.E_INVALID  # batch0
    assert f(100, 50, s, d, None, None, 8, 2.0, 10, V, 10, 10, 0.5, 3, 0, 0, None, q, None) == sped.OK
    assert need.value >= 2 * 100 * 10 * 4 + 2 * 10 * 12


def test_edge_apply_binding_rejects_bad_tensors(lib):
    """The binding checks device, dtype and length of every tensor before it
    hands raw pointers to the library (a host tensor or a short array would
    otherwise be dereferenced by a kernel)."""
    import torch
    X = torch.zeros(10, 4)
    with pytest.raises(TypeError):
        sped.edge_apply(10, torch.zeros(3, dtype=torch.int32), torch.zeros(3, dtype=torch.int32), X)
    with pytest.raises(TypeError):
        sped.stream_laplacian_apply(10, torch.zeros(3, dtype=torch.int32), torch.zeros(3, dtype=torch.int32), X)
    with pytest.raises(TypeError):
        sped.minibatch_oja(10, torch.zeros(3, dtype=torch.int32), torch.zeros(3, dtype=torch.int32), X)
    cpu = torch.device("cpu")
    with pytest.raises(TypeError):
        sped._device_vector(torch.zeros(3, dtype=torch.int64), "src", torch.int32, 0, cpu)
    with pytest.raises(ValueError):
        sped._device_vector(torch.zeros(3, dtype=torch.float32), "scale", torch.float32, 10, cpu)
    with pytest.raises(TypeError):
        sped._device_vector(torch.zeros(6, dtype=torch.int32)[::2], "dst", torch.int32, 3, cpu)
    sped._device_vector(torch.zeros(10, dtype=torch.float32), "scale", torch.float32, 10, cpu)
    with pytest.raises(TypeError):
        sped._device_block(torch.zeros(4, 3, dtype=torch.float64), "X")


def test_blocked_chain_validation(lib):
    """Host checks of the two-steps-per-launch chain: float32 blocks, k a power
    of two from 4 to 64, block_rows within the LDS and register budget, and
    the workspace size query (two n x k float blocks)."""
    c = sped.CSR()
    c.n, c.nnz, c.kind = 1000, 8000, sped.SYM_NORMALIZED
    c.rowptr = c.diag = c.scale = c.col = c.val = 16
    p = sped.transform("limit", 16).struct()
    X, Y = 4096, 1 << 20   # fake, 16-byte aligned, never dereferenced
    need = ctypes.c_size_t(0)
    f = lib.sped_apply_poly_blocked
    assert f(ctypes.byref(c), ctypes.byref(p), 125, 12, X, 12, sped.F32, Y, 12, sped.F32, None,
             ctypes.byref(need), None) == sped.E_UNSUPPORTED                       # k = 12
    assert f(ctypes.byref(c), ctypes.byref(p), 125, 32, X, 32, sped.BF16, Y, 32, sped.F32, None,
             ctypes.byref(need), None) == sped.E_UNSUPPORTED                       # bf16 X
    assert f(ctypes.byref(c), ctypes.byref(p), 1281, 32, X, 32, sped.F32, Y, 32, sped.F32, None,
             ctypes.byref(need), None) == sped.E_INVALID                           # 1281 x 32 floats > 160 KiB
    assert f(ctypes.byref(c), ctypes.byref(p), 0, 32, X, 32, sped.F32, Y, 32, sped.F32, None,
             ctypes.byref(need), None) == sped.E_INVALID                           # block_rows 0
    assert f(ctypes.byref(c), ctypes.byref(p), 125, 32, X + 4, 32, sped.F32, Y, 32, sped.F32, None,
             ctypes.byref(need), None) == sped.E_INVALID                           # misaligned X
    assert f(ctypes.byref(c), ctypes.byref(p), 1000, 32, X, 32, sped.F32, Y, 32, sped.F32, None,
             ctypes.byref(need), None) == sped.OK
    assert need.value >= 2 * 1000 * 32 * 4


def test_binding_refuses_host_blocks(lib):
    """Every dense block passes through the binding's leading-dimension check,
    which refuses host tensors before a pointer reaches the library."""
    import torch
    with pytest.raises(TypeError):
        sped.gram(torch.zeros(16, 4))
    with pytest.raises(TypeError):
        sped.orthonormalize(torch.zeros(16, 4))
    with pytest.raises(TypeError):
        sped.cluster_embed(torch.zeros(16, 4), 2)


def test_locality_order_validation(lib):
    """Node orders: an unknown method or a NULL input is refused before any
    device work; the ordered build's size query is host arithmetic."""
    need = ctypes.c_size_t(0)
    c = sped.CSR()
    c.n, c.nnz, c.kind = 100, 400, sped.SYM_NORMALIZED
    assert lib.sped_locality_order(ctypes.byref(c), 3, None, None, ctypes.byref(need), None) == sped.E_INVALID
    assert lib.sped_locality_order(None, 0, None, None, ctypes.byref(need), None) == sped.E_INVALID
    assert lib.sped_locality_order(ctypes.byref(c), 0, None, None, ctypes.byref(need), None) == sped.OK
    assert need.value >= 100 * (5 * 4 + 2 * 8)
    # label propagation sorts two 8-byte keys per stored entry
    assert lib.sped_locality_order(ctypes.byref(c), 2, None, None, ctypes.byref(need), None) == sped.OK
    assert need.value >= 2 * 400 * 8 + 100 * (7 * 4 + 2 * 8)
    c.nnz = -1
    assert lib.sped_locality_order(ctypes.byref(c), 2, None, None, ctypes.byref(need), None) == sped.E_INVALID
    # an entry-free Laplacian still needs the labels of two rounds (n int32
    # each) and one key per entry array
    c.n, c.nnz = 1000, 0
    cm, lp = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.sped_locality_order(ctypes.byref(c), 0, None, None, ctypes.byref(cm), None) == sped.OK
    assert lib.sped_locality_order(ctypes.byref(c), 2, None, None, ctypes.byref(lp), None) == sped.OK
    assert lp.value >= cm.value + 2 * 1000 * 4 + 2 * 8
    out = sped.CSR()
    assert lib.sped_laplacian_csr_ordered(100, 200, 16, 16, None, sped.SYM_NORMALIZED, 1, 7, ctypes.byref(out), None,
                                          None, ctypes.byref(need), None) == sped.E_INVALID
    assert b"method" in lib.sped_last_error()
    assert lib.sped_laplacian_csr_ordered(100, 200, None, None, None, sped.SYM_NORMALIZED, 1, 0, ctypes.byref(out),
                                          None, None, ctypes.byref(need), None) == sped.E_INVALID
    assert lib.sped_laplacian_csr_ordered(100, 200, 16, 16, None, 9, 1, 0, ctypes.byref(out), None, None,
                                          ctypes.byref(need), None) == sped.E_INVALID
    assert lib.sped_laplacian_csr_ordered(100, 200, 16, 16, None, sped.SYM_NORMALIZED, 1, 0, ctypes.byref(out),
                                          None, None, ctypes.byref(need), None) == sped.OK
    assert need.value >= 2 * 200 * 4 + 3 * 100 * 4
    # label propagation: room for the keys of the at most 2m stored entries
    assert lib.sped_laplacian_csr_ordered(100, 200, 16, 16, None, sped.SYM_NORMALIZED, 1, 2, ctypes.byref(out),
                                          None, None, ctypes.byref(need), None) == sped.OK
    assert need.value >= 2 * (2 * 200) * 8 + 2 * 200 * 4 + 3 * 100 * 4
    with pytest.raises(ValueError):
        sped.Laplacian(3, [0], [1], order="rcm")


def test_polynomial_degree_limit(lib):
    """Degree 1024 is the largest the chain takes; 1025 is refused on the
    host (size query and transform) before any launch."""
    need = ctypes.c_size_t(0)
    c = sped.CSR()
    c.n, c.nnz, c.kind = 100, 400, sped.SYM_NORMALIZED
    c.rowptr = c.diag = c.scale = c.col = c.val = 16
    for deg, want in ((1024, sped.OK), (1025, sped.E_INVALID)):
        p = sped.Poly()
        p.kind, p.degree = sped.POLY_LIMIT, deg
        assert lib.sped_apply_poly(ctypes.byref(c), ctypes.byref(p), 8, 256, 8, 0, 512, 8, 0, None,
                                   ctypes.byref(need), None) == want
        out = np.zeros(deg + 1)
        sh, sc = ctypes.c_double(), ctypes.c_double()
        assert lib.sped_transform_coeffs(sped.T_LIMIT, deg, 2.0, 0.0, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         ctypes.byref(sh), ctypes.byref(sc)) == want
