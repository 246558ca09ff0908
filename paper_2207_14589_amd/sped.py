"""ctypes binding of libsped (include/sped.h) over torch device tensors.

Argument marshalling only: every computation runs in the HIP library.  torch
provides device memory (inputs, outputs, workspaces) and the current stream.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsped.so")

OK, E_INVALID, E_WORKSPACE, E_DEVICE, E_NUMERIC, E_NOT_CONVERGED, E_UNSUPPORTED = range(7)
F32, BF16, F64 = 0, 1, 2
COMBINATORIAL, SYM_NORMALIZED = 0, 1
POLY_MONOMIAL, POLY_LIMIT = 0, 1
T_PLAIN, T_LIMIT, T_TAYLOR_EXP, T_TAYLOR_LOG = 0, 1, 2, 3
LIGHT_MAX, MEDIUM_MAX = 128, 8192

_c_i32, _c_i64, _c_u64, _c_f64, _c_vp, _c_sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                                ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t)


class CSR(ctypes.Structure):
    _fields_ = [("n", _c_i64), ("nnz", _c_i64), ("rowptr", _c_vp), ("col", _c_vp), ("val", _c_vp),
                ("rev", _c_vp), ("diag", _c_vp), ("scale", _c_vp), ("bins", _c_vp),
                ("wentry", _c_vp), ("wnode", _c_vp), ("n_medium", _c_i64), ("n_heavy", _c_i64), ("max_degree", _c_i32), ("kind", _c_i32),
                ("lambda_bound", _c_f64), ("xcd_rows", _c_i64 * 9)]


class Poly(ctypes.Structure):
    _fields_ = [("kind", _c_i32), ("degree", _c_i32), ("coeffs", ctypes.POINTER(_c_f64)),
                ("shift", _c_f64), ("scale", _c_f64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("solver", _c_i32), ("eta", _c_f64), ("tol", _c_f64), ("max_iters", _c_i32),
                ("check_every", _c_i32), ("guard", _c_i32), ("orth_passes", _c_i32),
                ("stochastic_iters", _c_i32), ("walks_per_row", _c_i64), ("seed", _c_u64),
                ("coarse_tol", _c_f64), ("stochastic_sampler", _c_i32), ("stochastic_exact_terms", _c_i32),
                ("use_graphs", _c_i32), ("polish_checks", _c_i32), ("trace", ctypes.POINTER(_c_f64)),
                ("trace_cap", _c_i32), ("counter_base", _c_u64)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", _c_i32), ("spmm_count", _c_i64), ("seconds", _c_f64), ("max_residual", _c_f64),
                ("gap_estimate", _c_f64), ("bound", _c_f64), ("converged", _c_i32),
                ("cholqr_shifts", _c_i32), ("coarse_iters", _c_i32), ("polish_iters", _c_i32),
                ("trace_len", _c_i32), ("reseeded", _c_i32)]


_P = ctypes.POINTER
SIGNATURES = {
    "sped_laplacian_csr": [_c_i64, _c_i64, _c_vp, _c_vp, _c_vp, _c_i32, _c_i32, _P(CSR), _c_vp, _c_vp,
                           _P(_c_sz), _c_vp],
    "sped_locality_order": [_P(CSR), _c_i32, _c_vp, _c_vp, _P(_c_sz), _c_vp],
    "sped_laplacian_csr_ordered": [_c_i64, _c_i64, _c_vp, _c_vp, _c_vp, _c_i32, _c_i32, _c_i32, _P(CSR), _c_vp,
                                   _c_vp, _P(_c_sz), _c_vp],
    "sped_transform_coeffs": [_c_i32, _c_i32, _c_f64, _c_f64, _P(_c_f64), _P(_c_f64), _P(_c_f64)],
    "sped_poly_monomial": [_P(Poly), _P(_c_f64)],
    "sped_poly_rebase": [_P(Poly), _c_f64, _c_f64, _P(_c_f64)],
    "sped_apply_poly": [_P(CSR), _P(Poly), _c_i64, _c_vp, _c_i64, _c_i32, _c_vp, _c_i64, _c_i32, _c_vp,
                        _P(_c_sz), _c_vp],
    "sped_apply_poly_noalloc": [_P(CSR), _P(Poly), _c_i64, _c_vp, _c_i64, _c_i32, _c_vp, _c_i64, _c_i32, _c_vp],
    "sped_apply_poly_blocked": [_P(CSR), _P(Poly), _c_i64, _c_i64, _c_vp, _c_i64, _c_i32, _c_vp, _c_i64, _c_i32,
                                _c_vp, _P(_c_sz), _c_vp],
    "sped_apply_poly_stochastic": [_P(CSR), _P(_c_f64), _c_i32, _c_i64, _c_vp, _c_i64, _c_i32, _c_vp, _c_i64,
                                   _c_i32, _c_i32, _c_i64, _c_u64, _c_u64, _c_vp, _c_vp, _P(_c_sz), _c_vp],
    "sped_apply_poly_hybrid": [_P(CSR), _P(_c_f64), _c_i32, _c_i32, _c_i64, _c_vp, _c_i64, _c_i32, _c_vp,
                               _c_i64, _c_i32, _c_i32, _c_i64, _c_u64, _c_u64, _c_vp, _P(_c_sz), _c_vp],
    "sped_apply_limit_lazy": [_P(CSR), _c_i32, _c_i64, _c_vp, _c_i64, _c_i32, _c_vp, _c_i64, _c_i32, _c_i64,
                              _c_u64, _c_u64, _c_vp, _P(_c_sz), _c_vp],
    "sped_poly_backward": [_P(CSR), _c_i32, _c_f64, _c_f64, _c_i64, _c_vp, _c_i64, _c_vp, _c_i64, _c_vp, _c_vp,
                           _P(_c_sz), _c_vp],
    "sped_gram": [_c_i64, _c_i64, _c_i64, _c_vp, _c_i64, _c_vp, _c_i64, _c_i32, _c_vp, _c_vp, _P(_c_sz), _c_vp],
    "sped_orthonormalize": [_c_i64, _c_i64, _c_vp, _c_i64, _c_i32, _c_i32, _c_vp, _c_vp, _P(_c_sz), _c_vp],
    "sped_rayleigh_ritz": [_P(CSR), _c_i64, _c_vp, _c_i64, _c_i32, _c_vp, _c_vp, _c_vp, _P(_c_sz), _c_vp],
    "sped_bottomk_solve": [_P(CSR), _P(Poly), _c_i64, _c_vp, _c_i64, _c_vp, _c_i64, _c_i32, _P(_c_f64),
                           _P(_c_f64), _P(SolveOpts), _P(SolveStats), _c_vp, _P(_c_sz), _c_vp],
    "sped_cluster_embed": [_c_vp, _c_i64, _c_i64, _c_i64, _c_i32, _c_i32, _c_i32, _c_u64, _c_i32, _c_vp, _c_vp,
                           _c_vp, _P(_c_f64), _P(_c_i32), _c_vp, _P(_c_sz), _c_vp],
    "sped_edge_apply": [_c_i64, _c_i64, _c_vp, _c_vp, _c_vp, _c_vp, _c_i64, _c_vp, _c_i64, _c_i32, _c_vp, _c_i64,
                        ctypes.c_float, _c_vp, _c_vp],
    "sped_stream_node_scales": [_c_i64, _c_i64, _c_vp, _c_vp, _c_vp, _c_i32, _c_i64, _c_vp, _c_vp, _c_vp,
                                _P(_c_sz), _c_vp],
    "sped_stream_laplacian_apply": [_c_i64, _c_i64, _c_vp, _c_vp, _c_vp, _c_vp, _c_i64, _c_vp, _c_i64, _c_i32,
                                    _c_vp, _c_i64, ctypes.c_float, _c_i32, _c_i64, _c_vp, _P(_c_sz), _c_vp],
    "sped_minibatch_oja": [_c_i64, _c_i64, _c_vp, _c_vp, _c_vp, _c_vp, _c_i32, _c_f64, _c_i64, _c_vp, _c_i64,
                           _c_i64, _c_f64, _c_i32, _c_u64, _c_i64, _c_vp, _P(_c_sz), _c_vp],
    "sped_stream_copy": [_c_vp, _c_vp, _c_sz, _c_vp],
    "sped_gather_probe": [_c_vp, _c_i64, _c_i32, _c_i32, _c_i32, _c_vp, _c_vp],
    "sped_last_error": [],
    "sped_version": [],
}

_lib = None


class SpedError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def lib():
    """Load libsped.so (built by paper_2207_14589_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2207_14589_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name == "sped_last_error" else _c_i32
        _lib = L
    return _lib


def _check(status, where, allow=()):
    if status != OK and status not in allow:
        raise SpedError(status, where, lib().sped_last_error().decode())
    return status


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dt(t):
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ld(t):
    """Leading dimension of a device block; every block handed to the library
    goes through here, so a host tensor is refused before any pointer is."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("blocks must be CUDA tensors on the library's device")
    if t.dim() != 2:
        raise ValueError("blocks must be 2-D with unit column stride")
    if t.shape[0] == 0:  # an empty block has no layout (torch may give it zero strides)
        return max(int(t.shape[1]), 1)
    if t.stride(1) != 1 and t.shape[1] > 1:
        raise ValueError("blocks must be 2-D with unit column stride")
    if t.shape[0] == 1:  # one row: its stride is not a layout either
        return max(t.stride(0), int(t.shape[1]))
    return t.stride(0)


def _workspace(nbytes, device):
    if nbytes == 0:
        return None
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + int(nbytes)]


def _call_ws(fn, where, args_before_ws, device, allow=()):
    """Size query (ws = NULL), allocate, then run; stream is the last argument."""
    need = ctypes.c_size_t(0)
    _check(fn(*args_before_ws, None, ctypes.byref(need), _stream(device)), where + " (size query)")
    ws = _workspace(need.value, device)
    if ws is None:   # no workspace needed: ws = NULL with ws_bytes = NULL runs the call
        st = fn(*args_before_ws, None, None, _stream(device))
    else:
        st = fn(*args_before_ws, _ptr(ws), ctypes.byref(need), _stream(device))
    _check(st, where, allow)
    return st, ws


# ------------------------------------------------------------------ Laplacian
ORDERS = {"cuthill_mckee": 0, "cm": 0, "degree": 1, "label_propagation": 2, "lp": 2}


class Laplacian:
    """Device split CSR of L = diag - S built by sped_laplacian_csr.

    order: None keeps the given ids (the largest component, if `lcc`, in
    increasing id); "cuthill_mckee" / "cm" or "degree" numbers the rows in
    that order (sped_laplacian_csr_ordered).  old_of_new holds the original id
    of each row either way."""

    def __init__(self, n, src, dst, w=None, kind="sym", lcc=False, device="cuda", walk_records=True, order=None):
        dev = torch.device(device)
        if order is not None and order not in ORDERS:
            raise ValueError(f"order must be None or one of {sorted(ORDERS)}")

        def dev_tensor(x, dt):
            if isinstance(x, torch.Tensor):
                return x.to(device=dev, dtype=dt).contiguous()
            return torch.as_tensor(np.asarray(x), dtype=dt).to(dev)

        src = dev_tensor(src, torch.int32)
        dst = dev_tensor(dst, torch.int32)
        wt = None if w is None else dev_tensor(w, torch.float32)
        m = src.numel()
        n = int(n)
        if dst.numel() != m or (wt is not None and wt.numel() != m):
            raise ValueError("src, dst and w must have the same length")
        self.device = dev
        self.rowptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
        self.col = torch.empty(max(2 * m, 1), dtype=torch.int32, device=dev)
        self.val = torch.empty(max(2 * m, 1), dtype=torch.float32, device=dev)
        self.rev = torch.empty(max(2 * m, 1), dtype=torch.int64, device=dev)
        self.diag = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
        self.scale = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
        self.bins = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        self.old_of_new = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        # walk records (32-byte entries, 16-byte nodes) for the stochastic estimators
        self.wentry = (torch.empty(max(2 * m, 1) * 8, dtype=torch.int32, device=dev) if walk_records else None)
        self.wnode = torch.empty(max(n, 1) * 2, dtype=torch.int64, device=dev) if walk_records else None
        c = CSR()
        c.rowptr, c.col, c.val, c.rev = (self.rowptr.data_ptr(), self.col.data_ptr(), self.val.data_ptr(),
                                         self.rev.data_ptr())
        c.diag, c.scale, c.bins = self.diag.data_ptr(), self.scale.data_ptr(), self.bins.data_ptr()
        c.wentry, c.wnode = (self.wentry.data_ptr(), self.wnode.data_ptr()) if walk_records else (None, None)
        kind_i = {"sym": SYM_NORMALIZED, "combinatorial": COMBINATORIAL}[kind] if isinstance(kind, str) else kind
        self.kind = kind_i
        if order is None:
            _call_ws(lib().sped_laplacian_csr, "sped_laplacian_csr",
                     (n, m, _ptr(src), _ptr(dst), _ptr(wt), kind_i, int(bool(lcc)), ctypes.byref(c),
                      _ptr(self.old_of_new)), dev)
        else:
            _call_ws(lib().sped_laplacian_csr_ordered, "sped_laplacian_csr_ordered",
                     (n, m, _ptr(src), _ptr(dst), _ptr(wt), kind_i, int(bool(lcc)), ORDERS[order],
                      ctypes.byref(c), _ptr(self.old_of_new)), dev)
        self.order = order
        self.c = c
        self.n, self.nnz = c.n, c.nnz
        self.max_degree, self.lambda_bound = c.max_degree, c.lambda_bound
        self.n_medium, self.n_heavy = c.n_medium, c.n_heavy
        self.xcd_rows = list(c.xcd_rows)
        self.old_of_new = self.old_of_new[: self.n]

    @property
    def ref(self):
        return ctypes.byref(self.c)

    def host_csr(self):
        """(rowptr, col, val, diag, scale) as numpy arrays, for checks."""
        n, nnz = self.n, self.nnz
        return (self.rowptr[: n + 1].cpu().numpy(), self.col[:nnz].cpu().numpy(), self.val[:nnz].cpu().numpy(),
                self.diag[:n].cpu().numpy(), self.scale[:n].cpu().numpy())


def locality_order(L: Laplacian, method="cuthill_mckee"):
    """Position of each row of L in the order `method` (device int32 [L.n])."""
    if method not in ORDERS:
        raise ValueError(f"method must be one of {sorted(ORDERS)}")
    out = torch.empty(max(L.n, 1), dtype=torch.int32, device=L.device)
    _call_ws(lib().sped_locality_order, "sped_locality_order", (L.ref, ORDERS[method], _ptr(out)), L.device)
    return out[: L.n]


# ------------------------------------------------------------------ polynomials
@dataclass
class PolySpec:
    kind: int
    degree: int
    coeffs: np.ndarray = field(default_factory=lambda: np.zeros(1))
    shift: float = 0.0
    scale: float = 1.0

    def struct(self):
        self._buf = np.ascontiguousarray(self.coeffs, dtype=np.float64)
        p = Poly()
        p.kind, p.degree = self.kind, self.degree
        p.coeffs = self._buf.ctypes.data_as(ctypes.POINTER(_c_f64))
        p.shift, p.scale = float(self.shift), float(self.scale)
        return p

    def monomial(self):
        out = np.zeros(self.degree + 1)
        p = self.struct()
        _check(lib().sped_poly_monomial(ctypes.byref(p), out.ctypes.data_as(ctypes.POINTER(_c_f64))),
               "sped_poly_monomial")
        return out

    def rebase(self, shift, scale):
        """Coefficients of the same polynomial in Lt = (L - shift I) / scale."""
        out = np.zeros(self.degree + 1)
        p = self.struct()
        _check(lib().sped_poly_rebase(ctypes.byref(p), float(shift), float(scale),
                                      out.ctypes.data_as(ctypes.POINTER(_c_f64))), "sped_poly_rebase")
        return out


def transform(name, degree, lambda_bound=2.0, eps=1e-3, product_form=True):
    """Table 2 operator M reversed by eq. reveig: 'plain', 'limit', 'taylor_exp', 'taylor_log'."""
    t = {"plain": T_PLAIN, "limit": T_LIMIT, "taylor_exp": T_TAYLOR_EXP, "taylor_log": T_TAYLOR_LOG}[name]
    if name == "plain":
        degree = 1
    c = np.zeros(degree + 1)
    sh, sc = _c_f64(0), _c_f64(1)
    _check(lib().sped_transform_coeffs(t, degree, lambda_bound, eps, c.ctypes.data_as(ctypes.POINTER(_c_f64)),
                                       ctypes.byref(sh), ctypes.byref(sc)), "sped_transform_coeffs")
    if name == "limit" and product_form:
        return PolySpec(POLY_LIMIT, degree, c, 0.0, 1.0)
    return PolySpec(POLY_MONOMIAL, degree, c, sh.value, sc.value)


def monomial(coeffs, shift=0.0, scale=1.0):
    c = np.asarray(coeffs, dtype=np.float64)
    return PolySpec(POLY_MONOMIAL, len(c) - 1, c, shift, scale)


# ------------------------------------------------------------------ operations
def apply_poly(L: Laplacian, p: PolySpec, X: torch.Tensor, out=None, out_dtype=None):
    k = X.shape[1]
    if out is None:
        out = torch.empty(L.n, k, dtype=out_dtype or X.dtype, device=X.device)
    ps = p.struct()
    _call_ws(lib().sped_apply_poly, "sped_apply_poly",
             (L.ref, ctypes.byref(ps), k, _ptr(X), _ld(X), _dt(X), _ptr(out), _ld(out), _dt(out)), X.device)
    return out


def apply_poly_noalloc(L: Laplacian, p: PolySpec, X: torch.Tensor, out: torch.Tensor):
    """Y = p(L) X through sped_apply_poly_noalloc: the library's static scratch
    instead of a workspace, so the call itself allocates nothing; `out` is the
    caller's.  Calls on one GPU must not overlap in time."""
    k = X.shape[1]
    ps = p.struct()
    _check(lib().sped_apply_poly_noalloc(L.ref, ctypes.byref(ps), k, _ptr(X), _ld(X), _dt(X), _ptr(out), _ld(out),
                                         _dt(out), _stream(X.device)), "sped_apply_poly_noalloc")
    return out


def apply_poly_blocked(L: Laplacian, p: PolySpec, X: torch.Tensor, block_rows: int, out=None):
    """Y = p(L) X with pairs of steps fused on LDS-resident blocks of
    `block_rows` consecutive rows (sped_apply_poly_blocked); float32 only."""
    k = X.shape[1]
    if out is None:
        out = torch.empty(L.n, k, dtype=torch.float32, device=X.device)
    ps = p.struct()
    _call_ws(lib().sped_apply_poly_blocked, "sped_apply_poly_blocked",
             (L.ref, ctypes.byref(ps), int(block_rows), k, _ptr(X), _ld(X), _dt(X), _ptr(out), _ld(out), _dt(out)),
             X.device)
    return out


def apply_poly_stochastic(L: Laplacian, coeffs, X, walks, seed, counter=0, sampler="importance", out=None,
                          out_dtype=None, accept_counts=False):
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    k = X.shape[1]
    smp = {"importance": 0, "reject": 1}[sampler]
    if out is None:
        out = torch.empty(L.n, k, dtype=out_dtype or (torch.float32 if smp == 1 else X.dtype), device=X.device)
    counts = torch.zeros(len(c) - 1, dtype=torch.int64, device=X.device) if accept_counts else None
    _call_ws(lib().sped_apply_poly_stochastic, "sped_apply_poly_stochastic",
             (L.ref, c.ctypes.data_as(ctypes.POINTER(_c_f64)), len(c) - 1, k, _ptr(X), _ld(X), _dt(X), _ptr(out),
              _ld(out), _dt(out), smp, int(walks), int(seed), int(counter), _ptr(counts)), X.device)
    return (out, counts) if accept_counts else out


def apply_poly_hybrid(L: Laplacian, coeffs, X, exact_terms, walks, seed, counter=0, sampler="importance",
                      out=None, out_dtype=None):
    """Estimate of sum_i c_i L^i X with terms i < exact_terms exact and the
    tail sampled by walks (sped_apply_poly_hybrid)."""
    c = np.ascontiguousarray(coeffs, dtype=np.float64)
    k = X.shape[1]
    smp = {"importance": 0, "reject": 1}[sampler]
    if out is None:
        out = torch.empty(L.n, k, dtype=out_dtype or X.dtype, device=X.device)
    _call_ws(lib().sped_apply_poly_hybrid, "sped_apply_poly_hybrid",
             (L.ref, c.ctypes.data_as(ctypes.POINTER(_c_f64)), len(c) - 1, int(exact_terms), k, _ptr(X), _ld(X),
              _dt(X), _ptr(out), _ld(out), _dt(out), smp, int(walks), int(seed), int(counter)), X.device)
    return out


def apply_limit_lazy(L: Laplacian, ell, X, walks, seed, counter=0, out=None, out_dtype=None):
    """Unbiased lazy node-walk estimate of (I - L/ell)^ell X."""
    k = X.shape[1]
    if out is None:
        out = torch.empty(L.n, k, dtype=out_dtype or X.dtype, device=X.device)
    _call_ws(lib().sped_apply_limit_lazy, "sped_apply_limit_lazy",
             (L.ref, int(ell), k, _ptr(X), _ld(X), _dt(X), _ptr(out), _ld(out), _dt(out), int(walks), int(seed),
              int(counter)), X.device)
    return out


def poly_backward(L: Laplacian, degree, X, dY, shift=0.0, scale=1.0):
    dtheta = torch.empty(degree + 1, dtype=torch.float64, device=X.device)
    _call_ws(lib().sped_poly_backward, "sped_poly_backward",
             (L.ref, degree, shift, scale, X.shape[1], _ptr(X), _ld(X), _ptr(dY), _ld(dY), _ptr(dtheta)), X.device)
    return dtheta


def gram(A, B=None):
    B = A if B is None else B
    G = torch.empty(A.shape[1], B.shape[1], dtype=torch.float64, device=A.device)
    _call_ws(lib().sped_gram, "sped_gram",
             (A.shape[0], A.shape[1], B.shape[1], _ptr(A), _ld(A), _ptr(B), _ld(B), _dt(A), _ptr(G)), A.device)
    return G


def orthonormalize(V, passes=2, want_r=False):
    R = torch.empty(V.shape[1], V.shape[1], dtype=torch.float64, device=V.device) if want_r else None
    _call_ws(lib().sped_orthonormalize, "sped_orthonormalize",
             (V.shape[0], V.shape[1], _ptr(V), _ld(V), _dt(V), passes, _ptr(R)), V.device)
    return (V, R) if want_r else V


def rayleigh_ritz(L: Laplacian, Q):
    k = Q.shape[1]
    theta = torch.empty(k, dtype=torch.float64, device=Q.device)
    resid = torch.empty(k, dtype=torch.float64, device=Q.device)
    _call_ws(lib().sped_rayleigh_ritz, "sped_rayleigh_ritz",
             (L.ref, k, _ptr(Q), _ld(Q), _dt(Q), _ptr(theta), _ptr(resid)), Q.device)
    return theta, resid


@dataclass
class SolveResult:
    evals: np.ndarray
    V: torch.Tensor
    residuals: np.ndarray
    stats: dict
    converged: bool


def bottomk(L: Laplacian, k, poly: PolySpec | None = None, V0=None, guard=4, tol=1e-6, max_iters=1000,
            check_every=1, orth_passes=2, solver="subspace", eta=1.0, stochastic_iters=0, walks_per_row=8,
            seed=3, v0_seed=2, storage="f32", coarse_tol=1e-2, sampler="importance", exact_terms=None,
            graphs=False, polish=0, trace_cap=0, counter_base=0, log_path=None):
    dev = L.device
    kb = k + guard
    if exact_terms is None:
        # random iterations with edge walks default to the first two terms of
        # the polynomial exact and the tail sampled (about 9x less error on
        # the iterate than the all-sampled estimate for 4% more time); the
        # lazy node walk takes none
        deg = 1 if poly is None else poly.degree
        exact_terms = min(2, deg) if (stochastic_iters > 0 and sampler == "importance") else 0
    if V0 is None:
        g = torch.Generator(device="cpu").manual_seed(v0_seed)
        V0 = torch.randn(L.n, kb, generator=g, dtype=torch.float64).to(torch.float32).to(dev)
    V_out = torch.empty(L.n, k, dtype=torch.float32, device=dev)
    ev = np.zeros(k)
    rs = np.zeros(k)
    o = SolveOpts(solver={"subspace": 0, "oja": 1, "mu_eg": 2}[solver], eta=eta, tol=tol, max_iters=max_iters,
                  check_every=check_every, guard=guard, orth_passes=orth_passes,
                  stochastic_iters=stochastic_iters, walks_per_row=walks_per_row, seed=seed,
                  coarse_tol=coarse_tol, stochastic_sampler={"importance": 0, "lazy": 1}[sampler],
                  stochastic_exact_terms=int(exact_terms), use_graphs=int(bool(graphs)),
                  polish_checks=int(polish), counter_base=int(counter_base))
    if log_path is not None and trace_cap <= 0:
        trace_cap = max_iters
    trace = np.zeros((max(int(trace_cap), 1), 4))
    if trace_cap > 0:
        o.trace = trace.ctypes.data_as(ctypes.POINTER(_c_f64))
        o.trace_cap = int(trace_cap)
    st = SolveStats()
    ps = poly.struct() if poly is not None else None
    status, _ = _call_ws(lib().sped_bottomk_solve, "sped_bottomk_solve",
                         (L.ref, ctypes.byref(ps) if ps is not None else None, k, _ptr(V0), _ld(V0), _ptr(V_out),
                          _ld(V_out), {"f32": F32, "bf16": BF16}[storage], ev.ctypes.data_as(ctypes.POINTER(_c_f64)),
                          rs.ctypes.data_as(ctypes.POINTER(_c_f64)), ctypes.byref(o), ctypes.byref(st)), dev,
                         allow=(E_NOT_CONVERGED,))
    stats = {f: getattr(st, f) for f, _ in SolveStats._fields_}
    if trace_cap > 0:
        stats["trace"] = trace[: st.trace_len].tolist()
    if log_path is not None:
        # one JSON line per check, then one for the result
        import json
        with open(log_path, "a") as fh:
            for it, sec, bound, rmax in stats["trace"]:
                fh.write(json.dumps({"iter": int(it), "seconds": sec, "bound": bound, "max_residual": rmax}) + "\n")
            fh.write(json.dumps({"result": {f: getattr(st, f) for f, _ in SolveStats._fields_},
                                 "status": int(status)}) + "\n")
    return SolveResult(ev, V_out, rs, stats, status == OK)


def cluster_embed(V, n_clusters, row_normalize=True, seed=0, max_iters=300, init=None):
    n, k = V.shape
    labels = torch.empty(n, dtype=torch.int32, device=V.device)
    cent = torch.empty(n_clusters, k, dtype=torch.float64, device=V.device)
    inertia = _c_f64(0)
    iters = _c_i32(0)
    init_t = None if init is None else torch.as_tensor(init, dtype=torch.float64).to(V.device).contiguous()
    _call_ws(lib().sped_cluster_embed, "sped_cluster_embed",
             (_ptr(V), n, k, _ld(V), _dt(V), n_clusters, int(bool(row_normalize)), int(seed), max_iters,
              _ptr(init_t), _ptr(labels), _ptr(cent), ctypes.byref(inertia), ctypes.byref(iters)), V.device)
    return labels, cent, inertia.value, iters.value


# ------------------------------------------------------- edge-batch products
def _host_edges(src_h, dst_h, w_h):
    """Host edge arrays as contiguous CPU tensors (int32, int32, float32 or
    None); pinned memory lets the library overlap copies with kernels."""
    def chk(t, dt, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cpu" or t.dtype != dt or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous CPU tensor of {dt}")
        return t
    src_h = chk(src_h, torch.int32, "src")
    dst_h = chk(dst_h, torch.int32, "dst")
    if dst_h.numel() != src_h.numel() or (w_h is not None and w_h.numel() != src_h.numel()):
        raise ValueError("src, dst and w must have the same length")
    return src_h, dst_h, (None if w_h is None else chk(w_h, torch.float32, "w"))


def _device_block(X, name, dtype=None):
    """X must be a 2-D CUDA tensor with unit column stride (rows may be
    padded: the leading dimension is passed), of dtype float32/bfloat16 or the
    one given."""
    if not isinstance(X, torch.Tensor) or X.device.type != "cuda" or X.dim() != 2 or \
            (X.shape[0] > 0 and X.stride(1) != 1):
        raise TypeError(f"{name} must be a 2-D CUDA tensor with contiguous rows")
    ok = (X.dtype == dtype) if dtype is not None else X.dtype in (torch.float32, torch.bfloat16)
    if not ok:
        raise TypeError(f"{name} has dtype {X.dtype}")


def _device_vector(t, name, dtype, min_len, device):
    if not isinstance(t, torch.Tensor) or t.device != device or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor on {device}")
    if t.numel() < min_len:
        raise ValueError(f"{name} has {t.numel()} elements, needs at least {min_len}")


def edge_apply(n, src, dst, X, w=None, scale=None, alpha=1.0, out=None, invalid=None):
    """out += alpha sum_e x_e x_e^T X over a batch of DEVICE edges (int32 src,
    dst; float32 w or None; node scales or None for the combinatorial L).
    out is float32 n x k (a new zero block when None); invalid is an optional
    DEVICE int64 counter of skipped edges.  Every tensor must sit on X's
    device with the dtype and length named; violations raise before the
    library is called."""
    _device_block(X, "X")
    k = X.shape[1]
    if X.shape[0] < int(n):
        raise ValueError("X has fewer than n rows")
    m = src.numel() if isinstance(src, torch.Tensor) else -1
    _device_vector(src, "src", torch.int32, 0, X.device)
    _device_vector(dst, "dst", torch.int32, m, X.device)
    if dst.numel() != m:
        raise ValueError("src and dst differ in length")
    if w is not None:
        _device_vector(w, "w", torch.float32, m, X.device)
        if w.numel() != m:
            raise ValueError("w and src differ in length")
    if scale is not None:
        _device_vector(scale, "scale", torch.float32, int(n), X.device)
    if invalid is not None:
        _device_vector(invalid, "invalid", torch.int64, 1, X.device)
    if out is None:
        out = torch.zeros(n, k, dtype=torch.float32, device=X.device)
    _device_block(out, "out", torch.float32)
    if out.device != X.device or out.shape[0] < int(n) or out.shape[1] != k:
        raise ValueError("out must be a float32 block of n x k on X's device")
    _check(lib().sped_edge_apply(int(n), m, _ptr(src), _ptr(dst), _ptr(w), _ptr(scale), k, _ptr(X), _ld(X),
                                 _dt(X), _ptr(out), _ld(out), float(alpha), _ptr(invalid), _stream(X.device)),
           "sped_edge_apply")
    return out


def stream_node_scales(n, src_h, dst_h, w_h=None, kind="sym", batch=1 << 22, device="cuda"):
    """(degree float64, scale float32) DEVICE tensors from a HOST edge list
    read in batches."""
    src_h, dst_h, w_h = _host_edges(src_h, dst_h, w_h)
    kind_i = {"sym": SYM_NORMALIZED, "combinatorial": COMBINATORIAL}[kind] if isinstance(kind, str) else kind
    dev = torch.device(device)
    degree = torch.empty(max(int(n), 1), dtype=torch.float64, device=dev)
    scale = torch.empty(max(int(n), 1), dtype=torch.float32, device=dev)
    _call_ws(lib().sped_stream_node_scales, "sped_stream_node_scales",
             (int(n), src_h.numel(), _c_vp(src_h.data_ptr()), _c_vp(dst_h.data_ptr()),
              _c_vp(w_h.data_ptr() if w_h is not None else None), kind_i, int(batch), _ptr(degree), _ptr(scale)), dev)
    return degree[: int(n)], scale[: int(n)]


def stream_laplacian_apply(n, src_h, dst_h, X, w_h=None, scale=None, alpha=1.0, out=None, accumulate=False,
                           batch=1 << 22):
    """alpha sum_e x_e x_e^T X over a HOST edge list streamed in batches
    (accumulate: added to out).  scale: node scales (DEVICE) or None for the
    combinatorial Laplacian.  Returns the float32 n x k result."""
    src_h, dst_h, w_h = _host_edges(src_h, dst_h, w_h)
    _device_block(X, "X")
    k = X.shape[1]
    if X.shape[0] < int(n):
        raise ValueError("X has fewer than n rows")
    if scale is not None:
        _device_vector(scale, "scale", torch.float32, int(n), X.device)
    if out is None:
        out = torch.empty(int(n), k, dtype=torch.float32, device=X.device)
        accumulate = False
    _device_block(out, "out", torch.float32)
    if out.device != X.device or out.shape[0] < int(n) or out.shape[1] != k:
        raise ValueError("out must be a float32 block of n x k on X's device")
    _call_ws(lib().sped_stream_laplacian_apply, "sped_stream_laplacian_apply",
             (int(n), src_h.numel(), _c_vp(src_h.data_ptr()), _c_vp(dst_h.data_ptr()),
              _c_vp(w_h.data_ptr() if w_h is not None else None), _ptr(scale), k, _ptr(X), _ld(X), _dt(X),
              _ptr(out), _ld(out), float(alpha), int(bool(accumulate)), int(batch)), X.device)
    return out


def minibatch_oja(n, src_h, dst_h, V, w_h=None, scale=None, degree=0, lambda_bound=2.0, batch=1 << 16, eta=0.5,
                  iters=100, seed=0, batch0=0):
    """In place: `iters` Oja steps V <- orth(V + eta M_hat V) with M_hat from
    batches of a HOST edge list, each the run of `batch` edges from a random
    offset (Philox keyed by seed; batch0 = batches drawn by earlier calls of
    the same solve).  degree 0: lambda_bound I - L; degree l: the limit
    polynomial (I - L/l)^l, one batch per factor.  V: DEVICE float32 n x k."""
    src_h, dst_h, w_h = _host_edges(src_h, dst_h, w_h)
    _device_block(V, "V", torch.float32)
    if scale is not None:
        _device_vector(scale, "scale", torch.float32, int(n), V.device)
    _call_ws(lib().sped_minibatch_oja, "sped_minibatch_oja",
             (int(n), src_h.numel(), _c_vp(src_h.data_ptr()), _c_vp(dst_h.data_ptr()),
              _c_vp(w_h.data_ptr() if w_h is not None else None), _ptr(scale), int(degree), float(lambda_bound),
              V.shape[1], _ptr(V), _ld(V), int(batch), float(eta), int(iters), int(seed), int(batch0)), V.device)
    return V


def gather_probe(table, iters, scattered, blocks, out):
    """Launch the row-load rate probe over `table` (rows x 32 float32)."""
    rows = table.shape[0]
    _check(lib().sped_gather_probe(_ptr(table), rows, int(iters), int(bool(scattered)), int(blocks), _ptr(out),
                                   _stream(table.device)), "sped_gather_probe")


def stream_copy(src, dst):
    _check(lib().sped_stream_copy(_ptr(src), _ptr(dst), src.numel() * src.element_size(), _stream(src.device)),
           "sped_stream_copy")
