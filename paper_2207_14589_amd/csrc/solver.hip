// Bottom-k block eigensolver on the dilated, reversed operator (Sec. 3,
// eq. reveig; Sec. 4; Sec. 5 solvers):
//   W = M Q                 M = p(L), or lambda_bound I - L for the plain solver
//   Q = W R^{-1}            Cholesky QR (twice by default), float64 Gram
//   every c iterations:     Rayleigh-Ritz on L: Z = L Q, H = Q^T Z = S Theta S^T,
//                           Q <- Q S, residual block R = Z S - Q Theta and its
//                           float64 Gram R^T R (column norms, ||R||_2 bound)
// Block Oja with step eta iterates on M + I/eta (the same subspace update).
// mu-EigenGame (solver 2) replaces the Cholesky QR by the game's update,
// V <- normalise(V + eta grad), which recovers the ordered eigenvectors one by
// one; its checks run Rayleigh-Ritz on an orthonormalised copy of V.
// The host loop only reads 2(k + guard) doubles and 3 flags per check.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace sped {
namespace {

constexpr int kBlock = 256;

template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void copy_block_kernel(int64_t n, int k, const TI *__restrict__ in, int64_t ldi,
                                                            TO *__restrict__ out, int64_t ldo) {
  const int64_t total = n * k;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < total; i += int64_t(gridDim.x) * kBlock) {
    int64_t r = i / k, c = i - r * k;
    out[r * ldo + c] = from_f32<TO>(to_f32<TI>(in[r * ldi + c]));
  }
}

__global__ void set_double_kernel(double *p, double v) {
  if (threadIdx.x == 0) *p = v;
}

__global__ void zero_int_kernel(int *p, int count) {
  if (int(threadIdx.x) < count) p[threadIdx.x] = 0;
}

sped_status copy_block(int64_t n, int k, const void *in, int64_t ldi, int ti, void *out, int64_t ldo, int to,
                       hipStream_t s) {
  if (n == 0 || k == 0) return SPED_OK;
  int64_t blocks = (n * k + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
#define SPED_COPY(TI_, TO_)                                                                          \
  hipLaunchKernelGGL((copy_block_kernel<TI_, TO_>), dim3(unsigned(blocks)), dim3(kBlock), 0, s, n, k, \
                     static_cast<const TI_ *>(in), ldi, static_cast<TO_ *>(out), ldo)
  if (ti == SPED_F32 && to == SPED_F32) SPED_COPY(float, float);
  else if (ti == SPED_F32 && to == SPED_BF16) SPED_COPY(float, bf16_t);
  else if (ti == SPED_BF16 && to == SPED_F32) SPED_COPY(bf16_t, float);
  else if (ti == SPED_BF16 && to == SPED_BF16) SPED_COPY(bf16_t, bf16_t);
  else return fail(SPED_E_UNSUPPORTED, "copy dtype");
#undef SPED_COPY
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

// mu-EigenGame coefficients, one thread per player i.  G1 = V^T (M V) and G3
// is the Gram of the unnormalised iterate V' with V = V' D^{-1},
// D = diag(sqrt(G3_ii)), so (V^T V)_ji = G3_ji / (D_j D_i).  The projected
// gradient of player i is
//   grad_i = M v_i - sum_{j<i} G1_ji v_j - d_i v_i,
//   d_i = <M v_i - sum_{j<i} G1_ji v_j, v_i> = G1_ii - sum_{j<i} G1_ji (V^T V)_ji,
// and V + eta grad = V A + eta M V with A = I - eta (striu(G1) + diag(d))
// (A row-major, A[j][i] multiplies column j into column i).
__global__ void mueg_coeffs_kernel(int k, const double *__restrict__ G1, const double *__restrict__ G3, double eta,
                                   double *__restrict__ A) {
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const double di_ = sqrt(G3[i * k + i]);
    double d = G1[i * k + i];
    for (int j = 0; j < i; ++j) d -= G1[j * k + i] * (G3[j * k + i] / (sqrt(G3[j * k + j]) * di_));
    for (int r = 0; r < k; ++r) A[r * k + i] = (r == i) ? 1.0 - eta * d : (r < i ? -eta * G1[r * k + i] : 0.0);
  }
}

// Q[:, c] = X[:, c] / sqrt(G3_cc): unit columns from the Gram of X.
__global__ __launch_bounds__(kBlock) void scale_cols_kernel(int64_t n, int k, const float *__restrict__ X,
                                                            int64_t ldx, const double *__restrict__ G3,
                                                            float *__restrict__ Q, int64_t ldq) {
  const int64_t total = n * k;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < total; i += int64_t(gridDim.x) * kBlock) {
    const int64_t r = i / k;
    const int c = int(i - r * k);
    Q[r * ldq + c] = float(double(X[r * ldx + c]) / sqrt(G3[c * k + c]));
  }
}

sped_status scale_cols(int64_t n, int k, const float *X, int64_t ldx, const double *G3, float *Q, int64_t ldq,
                       hipStream_t s) {
  if (n == 0) return SPED_OK;
  int64_t blocks = (n * k + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(scale_cols_kernel, dim3(unsigned(blocks)), dim3(kBlock), 0, s, n, k, X, ldx, G3, Q, ldq);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

// Columns of an orthonormalised start block whose squared norm came out
// below 1/4 (the start block was rank deficient there: a repeated or zero
// column, which the shifted Cholesky leaves near zero); bad[k] counts them,
// and bad[k + 1] is set when the Gram is not finite.
__global__ void flag_columns_kernel(int k, const double *__restrict__ G, int *__restrict__ bad) {
  if (threadIdx.x == 0) {
    bad[k] = 0;
    bad[k + 1] = 0;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    const double d = G[j * k + j];
    bool finite = isfinite(d);
    for (int c = 0; c < k; ++c) finite = finite && isfinite(G[j * k + c]);
    bad[j] = finite && d < 0.25 ? 1 : 0;
    if (bad[j]) atomicAdd(bad + k, 1);
    if (!finite) atomicOr(bad + k + 1, 1);
  }
}

// Fresh uniform [-1, 1) entries in the flagged columns: Philox keyed by the
// solver seed, counter (row, column, 0xFFFFFFFF - attempt, 0).
template <typename T>
__global__ __launch_bounds__(kBlock) void reseed_columns_kernel(int64_t n, int k, T *__restrict__ Q, int64_t ld,
                                                                const int *__restrict__ bad, uint32_t k0,
                                                                uint32_t k1, uint32_t attempt) {
  const int64_t total = n * k;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < total; i += int64_t(gridDim.x) * kBlock) {
    const int64_t r = i / k;
    const int c = int(i - r * k);
    if (!bad[c]) continue;
    const double u = uniform53(k0, k1, uint32_t(r), uint32_t(c), 0xFFFFFFFFu - attempt, 0);
    Q[r * ld + c] = from_f32<T>(float(2.0 * u - 1.0));
  }
}

struct OrthWs {
  double *G, *T, *partials;
  int *flags;
};

// Q <- W R^{-1} (out of place when W != Q), then `passes - 1` more in place.
// W and Q share the storage type dt (float32 or bf16); the Gram and R are float64.
sped_status cholqr(int64_t n, int k, const void *W, void *Q, int64_t ld, int dt, int passes, double *R_out,
                   const OrthWs &w, hipStream_t s) {
  const void *src = W;
  for (int pass = 0; pass < passes; ++pass) {
    SPED_TRY(launch_gram(n, k, k, src, ld, dt, src, ld, dt, w.G, w.partials, s));
    SPED_TRY(launch_chol_inv(k, w.G, w.T, pass == passes - 1 ? R_out : nullptr, w.flags, s));
    SPED_TRY(launch_tsmm(n, k, k, src, ld, dt, w.T, Q, ld, dt, s));
    src = Q;
  }
  return SPED_OK;
}

struct RRWs {
  float *Z, *ZS;
  void *Qtmp;
  double *H, *S, *theta, *resid, *partials, *G, *norm2;
  int *flags;
  const double *jacobi_rel = nullptr;  // device scalar: where the k x k eigensolver stops (NULL: 1e-12)
  void *step_ws = nullptr;             // spmm_step_ws_bytes(L, k) for the product Z = L Q
};

// Rayleigh-Ritz of L on span(Q) (Q of storage type dt, Z = L Q in float32);
// the Ritz vectors are written to Qtmp, the residual Gram to w.G, and
// *w.norm2 bounds the spectral norm of the first kn residual columns.
sped_status rayleigh_ritz(const sped_csr *L, int64_t n, int k, int kn, const void *Q, int64_t ld, int dt,
                          const RRWs &w, hipStream_t s) {
  StepArgs a{};
  a.heavy_ws = w.step_ws;
  a.U = Q; a.ldu = ld; a.tu = dt;
  a.V = nullptr; a.ldv = ld; a.tv = dt;
  a.O = w.Z; a.ldo = ld; a.to = SPED_F32;
  a.a = 1.f; a.b = 0.f; a.g = 0.f;
  SPED_TRY(launch_spmm_step(L, k, a, s));
  SPED_TRY(launch_gram(n, k, k, Q, ld, dt, w.Z, ld, SPED_F32, w.H, w.partials, s));
  SPED_TRY(launch_jacobi(k, w.H, w.theta, w.S, w.flags, s, 1e-12, w.jacobi_rel));
  SPED_TRY(launch_tsmm(n, k, k, Q, ld, dt, w.S, w.Qtmp, ld, dt, s));
  SPED_TRY(launch_tsmm(n, k, k, w.Z, ld, SPED_F32, w.S, w.ZS, ld, SPED_F32, s));
  SPED_TRY(launch_resid(n, k, kn, w.ZS, w.Qtmp, ld, dt, w.theta, w.G, w.resid, w.norm2, w.partials, s));
  return SPED_OK;
}

}  // namespace
}  // namespace sped

using namespace sped;

extern "C" sped_status sped_orthonormalize(int64_t n, int64_t k, void *V, int64_t ldv, int32_t dt, int32_t passes,
                                           double *R_out, void *ws, size_t *ws_bytes, sped_stream_t stream) {
  clear_error();
  if (n < 0 || k < 1 || k > dense_max_k()) return fail(SPED_E_INVALID, "orthonormalize shape (k in [1, 96])");
  if (n < k) return fail(SPED_E_INVALID, "orthonormalize needs n >= k");
  if (ldv < k) return fail(SPED_E_INVALID, "ldv < k");
  if (dt != SPED_F32 && dt != SPED_BF16) return fail(SPED_E_UNSUPPORTED, "orthonormalize dtype must be F32 or BF16");
  if (passes < 1 || passes > 4) return fail(SPED_E_INVALID, "passes outside [1, 4]");
  if (!V) return fail(SPED_E_INVALID, "V NULL");
  Carver c(ws);
  OrthWs w;
  w.G = c.take<double>(size_t(k) * k);
  w.T = c.take<double>(size_t(k) * k);
  w.partials = c.take<double>(gram_ws_doubles(n, k, k));
  w.flags = c.take<int>(4);
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, c.bytes(), &query));
  if (query) return SPED_OK;
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, s, w.flags, 4);
  SPED_CHECK_HIP(hipGetLastError());
  SPED_TRY(cholqr(n, int(k), V, V, ldv, dt, passes, R_out, w, s));
  int flags[4];
  SPED_CHECK_HIP(hipMemcpyAsync(flags, w.flags, sizeof(flags), hipMemcpyDeviceToHost, s));
  SPED_CHECK_HIP(hipStreamSynchronize(s));
  if (flags[1]) return fail(SPED_E_NUMERIC, "Cholesky QR broke down after shifting");
  return SPED_OK;
}

extern "C" sped_status sped_rayleigh_ritz(const sped_csr *L, int64_t k, void *Q, int64_t ldq, int32_t dt,
                                          double *theta, double *resid, void *ws, size_t *ws_bytes,
                                          sped_stream_t stream) {
  clear_error();
  SPED_TRY(validate_csr(L));
  if (k < 1 || k > dense_max_k()) return fail(SPED_E_INVALID, "k outside [1, 96]");
  if (ldq < k) return fail(SPED_E_INVALID, "ldq < k");
  if (dt != SPED_F32) return fail(SPED_E_UNSUPPORTED, "rayleigh_ritz dtype must be F32");
  if (!Q || !theta || !resid) return fail(SPED_E_INVALID, "NULL pointer");
  const int64_t n = L->n;
  Carver c(ws);
  RRWs w;
  w.Z = c.take<float>(size_t(n) * ldq);
  w.ZS = c.take<float>(size_t(n) * ldq);
  w.Qtmp = c.take<float>(size_t(n) * ldq);
  w.H = c.take<double>(size_t(k) * k);
  w.S = c.take<double>(size_t(k) * k);
  w.theta = theta;
  w.resid = resid;
  w.partials = c.take<double>(gram_ws_doubles(n, k, k));
  w.G = c.take<double>(size_t(k) * k);
  w.norm2 = c.take<double>(1);
  w.flags = c.take<int>(4);
  const size_t sw = spmm_step_ws_bytes(L, k);
  w.step_ws = sw ? c.take<char>(sw) : nullptr;
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, c.bytes(), &query));
  if (query) return SPED_OK;
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, s, w.flags, 4);
  SPED_CHECK_HIP(hipGetLastError());
  SPED_TRY(rayleigh_ritz(L, n, int(k), int(k), Q, ldq, SPED_F32, w, s));
  SPED_TRY(copy_block(n, int(k), w.Qtmp, ldq, SPED_F32, Q, ldq, SPED_F32, s));
  return SPED_OK;
}

extern "C" sped_status sped_bottomk_solve(const sped_csr *L, const sped_poly *p, int64_t k, const void *V0,
                                          int64_t ldv0, void *V_out, int64_t ldvo, int32_t vdt, double *evals,
                                          double *resid_out, const sped_solve_opts *o, sped_solve_stats *st,
                                          void *ws, size_t *ws_bytes, sped_stream_t stream) {
  clear_error();
  SPED_TRY(validate_csr(L));
  if (!o) return fail(SPED_E_INVALID, "opts NULL");
  if (p) SPED_TRY(validate_poly(p));
  if (o->guard < 1) return fail(SPED_E_INVALID, "guard must be >= 1");
  const int64_t kb = k + o->guard;
  if (k < 1 || kb > dense_max_k()) return fail(SPED_E_INVALID, "k + guard outside [2, 96]");
  const int64_t n = L->n;
  if (n < kb) return fail(SPED_E_INVALID, "n < k + guard");
  if (ldv0 < kb || ldvo < k) return fail(SPED_E_INVALID, "leading dimension");
  if (vdt != SPED_F32 && vdt != SPED_BF16) return fail(SPED_E_UNSUPPORTED, "solver block dtype must be F32 or BF16");
  if (!V0 || !V_out || !evals) return fail(SPED_E_INVALID, "NULL pointer");
  if (o->max_iters < 1 || o->check_every < 1) return fail(SPED_E_INVALID, "max_iters/check_every");
  if (o->orth_passes < 1 || o->orth_passes > 4) return fail(SPED_E_INVALID, "orth_passes");
  if (o->solver < 0 || o->solver > 2) return fail(SPED_E_INVALID, "solver");
  if (o->solver != 0 && !(o->eta > 0.0 && std::isfinite(o->eta))) return fail(SPED_E_INVALID, "eta");
  if (o->solver == 2 && vdt != SPED_F32) return fail(SPED_E_UNSUPPORTED, "mu-EigenGame needs F32 storage");
  if (!(o->tol >= 0.0)) return fail(SPED_E_INVALID, "tol");
  if (o->stochastic_iters < 0) return fail(SPED_E_INVALID, "stochastic_iters");
  if (o->stochastic_sampler != 0 && o->stochastic_sampler != 1) return fail(SPED_E_INVALID, "stochastic_sampler");
  const bool lazy = o->stochastic_iters > 0 && o->stochastic_sampler == 1;
  if (o->use_graphs != 0 && o->use_graphs != 1) return fail(SPED_E_INVALID, "use_graphs must be 0 or 1");
  if (o->polish_checks < 0) return fail(SPED_E_INVALID, "polish_checks < 0");
  if (o->trace_cap < 0 || (o->trace_cap > 0 && !o->trace)) return fail(SPED_E_INVALID, "trace / trace_cap");
  if (o->polish_checks > 0 && o->solver != 0)
    return fail(SPED_E_UNSUPPORTED, "the plain polish follows subspace iteration (solver 0) only");
  if (o->stochastic_exact_terms < 0 || (lazy && o->stochastic_exact_terms != 0))
    return fail(SPED_E_INVALID, "stochastic_exact_terms (edge walks only, >= 0)");
  if (o->stochastic_iters > 0 && !lazy && (o->walks_per_row < 1 || !L->wentry || !L->wnode))
    return fail(SPED_E_INVALID, "stochastic iterations need walks_per_row >= 1 and the walk records");
  if (o->stochastic_iters > 0 &&
      (o->counter_base >= (uint64_t(1) << 32) || o->counter_base + uint64_t(o->max_iters) >= (uint64_t(1) << 32)))
    return fail(SPED_E_INVALID, "walk counters (counter_base + iterations) must stay below 2^32");
  if (lazy) {
    if (!p || p->kind != SPED_POLY_LIMIT) return fail(SPED_E_INVALID, "lazy walks estimate the limit polynomial only");
    if (o->solver == 1) return fail(SPED_E_UNSUPPORTED, "lazy walks with block Oja (M + I/eta) are not supported");
    SPED_TRY(validate_lazy(L, p->degree, o->walks_per_row, o->counter_base + uint64_t(o->max_iters)));
  }

  // the operator actually iterated on (op_id 1 once the plain polish starts)
  std::vector<double> plain_c = {L->lambda_bound, -1.0};
  const sped_poly plain_M{SPED_POLY_MONOMIAL, 1, plain_c.data(), 0.0, 1.0};
  sped_poly M = plain_M;
  if (p) M = *p;
  int op_id = 0;
  std::vector<double> oja_c;
  if (o->solver == 1) {
    oja_c = (M.kind == SPED_POLY_LIMIT) ? monomial_in_L(M) : std::vector<double>(M.coeffs, M.coeffs + M.degree + 1);
    if (M.kind == SPED_POLY_LIMIT) {
      M.shift = 0.0;
      M.scale = 1.0;
    }
    oja_c[0] += 1.0 / o->eta;
    M.kind = SPED_POLY_MONOMIAL;
    M.coeffs = oja_c.data();
  }
  std::vector<double> walk_c;
  if (o->stochastic_iters > 0 && !lazy) {
    walk_c = monomial_in_L(M);
    if (M.degree > 255) return fail(SPED_E_UNSUPPORTED, "stochastic iterations need degree <= 255");
    if (o->stochastic_exact_terms > M.degree) return fail(SPED_E_INVALID, "stochastic_exact_terms > degree");
  }

  const bool two_phase = vdt == SPED_BF16;
  const double coarse_tol = o->coarse_tol > 0.0 ? o->coarse_tol : 1e-2;
  Carver c(ws);
  float *Q32 = c.take<float>(size_t(n) * kb);
  float *W32 = c.take<float>(size_t(n) * kb);
  float *bufA = c.take<float>(size_t(n) * kb);
  float *bufB = c.take<float>(size_t(n) * kb);
  bf16_t *Q16 = two_phase ? c.take<bf16_t>(size_t(n) * kb) : nullptr;
  bf16_t *W16 = two_phase ? c.take<bf16_t>(size_t(n) * kb) : nullptr;
  OrthWs ow;
  ow.G = c.take<double>(size_t(kb) * kb);
  ow.T = c.take<double>(size_t(kb) * kb);
  ow.partials = c.take<double>(gram_ws_doubles(n, kb, kb));
  RRWs rw;
  rw.H = c.take<double>(size_t(kb) * kb);
  rw.S = c.take<double>(size_t(kb) * kb);
  rw.G = c.take<double>(size_t(kb) * kb);
  // what a check reads on the host (Ritz values, residual norms, the norm
  // bound, the flags) sits in one block: one copy per check instead of four
  // (each small copy into pageable memory waits on its own)
  const size_t nchk = size_t(2) * kb + 3;
  double *chk = c.take<double>(nchk);
  rw.theta = chk;
  rw.resid = chk ? chk + kb : nullptr;
  rw.norm2 = chk ? chk + 2 * kb : nullptr;
  rw.partials = ow.partials;
  int *flags = chk ? reinterpret_cast<int *>(chk + 2 * kb + 1) : nullptr;  // 4 ints
  ow.flags = rw.flags = flags;
  double *jrel = c.take<double>(1);
  rw.jacobi_rel = jrel;
  // mu-EigenGame: its Grams and update matrix, and a buffer for the Ritz
  // vectors of the checks (the game's iterate itself is kept)
  const bool mueg = o->solver == 2;
  double *G1 = mueg ? c.take<double>(size_t(kb) * kb) : nullptr;
  double *G3 = mueg ? c.take<double>(size_t(kb) * kb) : nullptr;
  double *Amu = mueg ? c.take<double>(size_t(kb) * kb) : nullptr;
  float *Rtmp = mueg ? c.take<float>(size_t(n) * kb) : nullptr;
  double *lz_max = lazy ? c.take<double>(size_t(n)) : nullptr;
  const size_t sw = spmm_step_ws_bytes(L, kb);
  void *step_ws = sw ? c.take<char>(sw) : nullptr;
  rw.step_ws = step_ws;
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, c.bytes(), &query));
  if (query) return SPED_OK;

  hipStream_t s = as_stream(stream);
  auto t_start = std::chrono::steady_clock::now();
  sped_solve_stats stats{};
  stats.bound = INFINITY;  // no check yet
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, s, flags, 4);
  SPED_CHECK_HIP(hipGetLastError());
  if (lazy) SPED_TRY(lazy_row_max(L, lz_max, s));  // graph-only, shared by every iteration

  std::vector<double> h_theta(kb), h_resid(kb);
  // the checks' host copy lands in pinned host memory (a direct transfer,
  // no staging through a pageable buffer); released on every return
  struct PinnedChk {
    double *p = nullptr;
    ~PinnedChk() {
      if (p) (void)hipHostFree(p);
    }
  } h_chk;
  SPED_CHECK_HIP(hipHostMalloc(reinterpret_cast<void **>(&h_chk.p), sizeof(double) * nchk, hipHostMallocDefault));
  double h_norm2 = 0.0;
  int h_flags[4] = {0, 0, 0, 0};
  int t = 0;
  // One phase of iterations with the iterate stored as dt in (Q, W); returns
  // with the Ritz vectors in Q after the last check.
  // With stall_checks > 0 the phase also ends when the largest residual has
  // not dropped below 0.98 x its best value for that many consecutive checks
  // (the storage's rounding floor has been reached).
  // The device work of one iteration: the operator (exact, or a random
  // estimate for the first stochastic_iters iterations), the orthonormalisation
  // or mu-EigenGame update, and with `check` the Rayleigh-Ritz step.
  auto enqueue = [&](int dt, void *Q, void *W, bool check, bool stoch, hipStream_t q) -> sped_status {
    if (stoch && lazy) {
      SPED_TRY(lazy_walk_impl(L, M.degree, kb, Q, kb, dt, W, kb, dt, o->walks_per_row, o->seed,
                              o->counter_base + uint64_t(t),
                              lz_max, q));
    } else if (stoch) {
      SPED_TRY(hybrid_estimate_impl(L, walk_c.data(), M.degree, o->stochastic_exact_terms, kb, Q, kb, dt, W, kb, dt,
                                    0, o->walks_per_row, o->seed, o->counter_base + uint64_t(t), bufA, bufB,
                                    step_ws, q,
                                    &stats.spmm_count));
    } else {
      SPED_TRY(apply_poly_impl(L, &M, kb, Q, kb, dt, W, kb, dt, bufA, bufB, step_ws, q, &stats.spmm_count));
    }
    if (mueg) {
      // V <- normalise(V + eta grad), grad the projected mu-EG gradients
      SPED_TRY(launch_gram(n, int(kb), int(kb), Q, kb, dt, W, kb, dt, G1, ow.partials, q));
      hipLaunchKernelGGL(mueg_coeffs_kernel, dim3(1), dim3(128), 0, q, int(kb), G1, G3, o->eta, Amu);
      SPED_CHECK_HIP(hipGetLastError());
      SPED_TRY(launch_tsmm(n, int(kb), int(kb), Q, kb, dt, Amu, W, kb, dt, q, W, kb, float(o->eta)));
      SPED_TRY(launch_gram(n, int(kb), int(kb), W, kb, dt, W, kb, dt, G3, ow.partials, q));
      SPED_TRY(scale_cols(n, int(kb), static_cast<const float *>(W), kb, G3, static_cast<float *>(Q), kb, q));
    } else {
      SPED_TRY(cholqr(n, int(kb), W, Q, kb, dt, o->orth_passes, nullptr, ow, q));
    }
    if (check) {
      rw.Z = bufA;
      rw.ZS = bufB;
      if (mueg) {  // Ritz pairs of L on span(V), from an orthonormalised copy
        SPED_TRY(cholqr(n, int(kb), Q, W, kb, dt, o->orth_passes, nullptr, ow, q));
        rw.Qtmp = Rtmp;
        SPED_TRY(rayleigh_ritz(L, n, int(kb), int(k), W, kb, dt, rw, q));
      } else {
        rw.Qtmp = W;  // Ritz vectors land in W
        SPED_TRY(rayleigh_ritz(L, n, int(kb), int(k), Q, kb, dt, rw, q));
      }
      stats.spmm_count += 1;
    }
    return SPED_OK;
  };
  // With use_graphs the exact iterations are captured once per (buffers,
  // storage, check) into a HIP graph and replayed; the graph holds the same
  // launches in the same order, so results are bit-identical.  Capture runs on
  // a stream of its own (the caller's may be the legacy default stream, which
  // cannot capture); replays run on the caller's stream.
  struct Captured {
    const void *Q, *W;
    int dt;
    bool check;
    int op;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int64_t spmm;
  };
  std::vector<Captured> graphs;
  hipStream_t cap = nullptr;
  struct Cleanup {
    std::vector<Captured> &g;
    hipStream_t &c;
    hipStream_t s;
    ~Cleanup() {
      if (!g.empty()) (void)hipStreamSynchronize(s);  // no replay may still be running
      for (auto &x : g) {
        (void)hipGraphExecDestroy(x.exec);
        (void)hipGraphDestroy(x.graph);
      }
      if (c) (void)hipStreamDestroy(c);
    }
  } cleanup{graphs, cap, s};
  auto run_graph = [&](int dt, void *Q, void *W, bool check) -> sped_status {
    Captured *hit = nullptr;
    for (auto &x : graphs)
      if (x.Q == Q && x.W == W && x.dt == dt && x.check == check && x.op == op_id) hit = &x;
    if (!hit) {
      if (!cap) SPED_CHECK_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      Captured c{Q, W, dt, check, op_id, nullptr, nullptr, 0};
      const int64_t before = stats.spmm_count;
      SPED_CHECK_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
      const sped_status st = enqueue(dt, Q, W, check, false, cap);
      const hipError_t ec = hipStreamEndCapture(cap, &c.graph);
      if (st != SPED_OK) {
        if (ec == hipSuccess && c.graph) (void)hipGraphDestroy(c.graph);
        return st;
      }
      SPED_CHECK_HIP(ec);
      const hipError_t ei = hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0);
      if (ei != hipSuccess) {
        (void)hipGraphDestroy(c.graph);
        SPED_CHECK_HIP(ei);
      }
      c.spmm = stats.spmm_count - before;  // counted again at every replay
      stats.spmm_count = before;
      graphs.push_back(c);
      hit = &graphs.back();
    }
    SPED_CHECK_HIP(hipGraphLaunch(hit->exec, s));
    stats.spmm_count += hit->spmm;
    return SPED_OK;
  };
  // One phase of iterations with the iterate stored as dt in (Q, W); returns
  // with the Ritz vectors in Q after the last check.
  // With stall_checks > 0 the phase also ends when the largest residual has
  // not dropped below 0.98 x its best value for that many consecutive checks
  // (the storage's rounding floor has been reached).
  // Stalls are counted only while the bound is at or below stall_below (the
  // first iterations of a large block can leave the largest residual flat
  // while the subspace turns).
  auto phase = [&](int dt, void *&Q, void *&W, double tol, int iter_cap, int stall_checks, double stall_below,
                   bool *done) -> sped_status {
    *done = false;
    const int first = t + 1;
    double best = INFINITY;
    int since_best = 0;
    for (t = first; t <= iter_cap; ++t) {
      const bool check = (t - first + 1) % o->check_every == 0 || t == iter_cap;
      const bool stoch = t <= o->stochastic_iters;
      if (check) {
        // Far from convergence the Ritz pairs need not be exact: an early stop
        // leaves S orthogonal (the same subspace) and can only raise the
        // residuals, so the stopping bound stays valid.  The k x k eigensolver
        // stops at 1e-3 x the last bound, within [1e-12, 1e-6] of ||H||.
        const double rel = std::min(1e-6, std::max(1e-12, 1e-3 * stats.bound));
        hipLaunchKernelGGL(set_double_kernel, dim3(1), dim3(64), 0, s, jrel, rel);
        SPED_CHECK_HIP(hipGetLastError());
      }
      if (o->use_graphs && !stoch) SPED_TRY(run_graph(dt, Q, W, check));
      else SPED_TRY(enqueue(dt, Q, W, check, stoch, s));
      if (check) {
        if (!mueg) std::swap(Q, W);  // Ritz vectors now in Q
        SPED_CHECK_HIP(hipMemcpyAsync(h_chk.p, chk, sizeof(double) * nchk, hipMemcpyDeviceToHost, s));
        SPED_CHECK_HIP(hipStreamSynchronize(s));
        std::copy(h_chk.p, h_chk.p + kb, h_theta.begin());
        std::copy(h_chk.p + kb, h_chk.p + 2 * kb, h_resid.begin());
        h_norm2 = h_chk.p[2 * kb];
        std::memcpy(h_flags, h_chk.p + 2 * kb + 1, sizeof(h_flags));
        if (h_flags[1]) return fail(SPED_E_NUMERIC, "Cholesky QR broke down after shifting");
        double rmax = 0.0;
        bool finite = std::isfinite(h_norm2);
        for (int i = 0; i < k; ++i) {
          rmax = std::max(rmax, h_resid[i]);
          finite = finite && std::isfinite(h_resid[i]) && std::isfinite(h_theta[i]);
        }
        if (!finite) return fail(SPED_E_NUMERIC, "non-finite Ritz value or residual");
        // the first guard Ritz value overestimates lambda_{k+1}; its residual
        // bounds by how much, so the gap estimate subtracts it
        double gap = h_theta[k] - h_resid[k] - h_theta[k - 1];
        stats.gap_estimate = gap;
        stats.max_residual = rmax;
        // Davis-Kahan: sin of the largest angle <= ||R||_2 / gap, with
        // ||R||_2 <= sqrt(min(||R^T R||_inf, ||R||_F^2)); the infinity norm is
        // the tighter one when the residual columns are nearly orthogonal
        stats.bound = gap > 0 ? h_norm2 / gap : INFINITY;
        if (stats.trace_len < o->trace_cap) {
          double *tr = o->trace + 4 * stats.trace_len++;
          tr[0] = t;
          tr[1] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
          tr[2] = stats.bound;
          tr[3] = rmax;
        }
        if (stats.bound <= tol) {
          *done = true;
          return SPED_OK;
        }
        // progress is judged on the largest residual, which is finite from the
        // first check (the bound is infinite while the gap estimate is not
        // positive, which would otherwise read as a stall)
        if (rmax < 0.98 * best) {
          best = rmax;
          since_best = 0;
        } else if (stall_checks > 0 && stats.bound <= stall_below && ++since_best >= stall_checks) {
          return SPED_OK;
        }
      }
    }
    t = iter_cap;
    return SPED_OK;
  };

  // First orthonormalisation of the start block (W -> Q, storage dt): one
  // Cholesky-QR pass, then columns left near zero (V0 rank deficient there)
  // are replaced by random ones and the block orthonormalised again, up to 3
  // times; then the remaining passes.
  int *bad = reinterpret_cast<int *>(rw.resid);  // kb + 2 ints inside the kb doubles of resid (kb >= 2)
  auto start_block = [&](int dt, const void *Win, void *Qout) -> sped_status {
    SPED_TRY(cholqr(n, int(kb), Win, Qout, kb, dt, 1, nullptr, ow, s));
    for (int attempt = 0; attempt < 3; ++attempt) {
      SPED_TRY(launch_gram(n, int(kb), int(kb), Qout, kb, dt, Qout, kb, dt, ow.G, ow.partials, s));
      hipLaunchKernelGGL(flag_columns_kernel, dim3(1), dim3(128), 0, s, int(kb), ow.G, bad);
      SPED_CHECK_HIP(hipGetLastError());
      int hb[2] = {0, 0};
      SPED_CHECK_HIP(hipMemcpyAsync(hb, bad + kb, sizeof(hb), hipMemcpyDeviceToHost, s));
      SPED_CHECK_HIP(hipStreamSynchronize(s));
      if (hb[1]) return fail(SPED_E_NUMERIC, "start block is not finite");
      if (hb[0] == 0) break;
      stats.reseeded += hb[0];
      int64_t blocks = (n * kb + kBlock - 1) / kBlock;
      if (blocks > 8192) blocks = 8192;
      const uint32_t k0 = uint32_t(o->seed), k1 = uint32_t(o->seed >> 32);
      if (dt == SPED_BF16)
        hipLaunchKernelGGL(reseed_columns_kernel<bf16_t>, dim3(unsigned(blocks)), dim3(kBlock), 0, s, n, int(kb),
                           static_cast<bf16_t *>(Qout), kb, bad, k0, k1, uint32_t(attempt));
      else
        hipLaunchKernelGGL(reseed_columns_kernel<float>, dim3(unsigned(blocks)), dim3(kBlock), 0, s, n, int(kb),
                           static_cast<float *>(Qout), kb, bad, k0, k1, uint32_t(attempt));
      SPED_CHECK_HIP(hipGetLastError());
      SPED_TRY(cholqr(n, int(kb), Qout, Qout, kb, dt, 1, nullptr, ow, s));
    }
    if (o->orth_passes > 1) SPED_TRY(cholqr(n, int(kb), Qout, Qout, kb, dt, o->orth_passes - 1, nullptr, ow, s));
    return SPED_OK;
  };

  void *Q = Q32, *W = W32;
  bool done = false;
  if (two_phase) {
    void *Qh = Q16, *Wh = W16;
    SPED_TRY(copy_block(n, int(kb), V0, ldv0, SPED_F32, Wh, kb, SPED_BF16, s));
    SPED_TRY(start_block(SPED_BF16, Wh, Qh));
    SPED_TRY(phase(SPED_BF16, Qh, Wh, coarse_tol, o->max_iters, 8, INFINITY, &done));
    stats.coarse_iters = t;
    // refinement sweep: the bf16 iterate seeds float32 iterations
    SPED_TRY(copy_block(n, int(kb), Qh, kb, SPED_BF16, W, kb, SPED_F32, s));
  } else {
    SPED_TRY(copy_block(n, int(kb), V0, ldv0, SPED_F32, W, kb, SPED_F32, s));
  }
  if (mueg) {  // the game starts from V0 with unit columns
    SPED_TRY(launch_gram(n, int(kb), int(kb), W, kb, SPED_F32, W, kb, SPED_F32, G3, ow.partials, s));
    SPED_TRY(scale_cols(n, int(kb), static_cast<const float *>(W), kb, G3, static_cast<float *>(Q), kb, s));
  } else {
    SPED_TRY(start_block(SPED_F32, W, Q));
  }
  done = false;
  const bool polish = o->polish_checks > 0 && p != nullptr;
  // the polynomial's float32 floor lies within a few hundred times tol; stalls
  // farther up are the block still turning
  if (t < o->max_iters)
    SPED_TRY(phase(SPED_F32, Q, W, o->tol, o->max_iters, polish ? o->polish_checks : 0, 1e3 * o->tol, &done));
  if (polish && !done && t < o->max_iters) {
    // p(L) has reached its rounding floor: plain iterations from its Ritz vectors (in Q)
    const int before = t;
    M = plain_M;
    op_id = 1;
    SPED_TRY(phase(SPED_F32, Q, W, o->tol, o->max_iters, 0, INFINITY, &done));
    stats.polish_iters = t - before;
  }
  sped_status result = done ? SPED_OK : SPED_E_NOT_CONVERGED;
  stats.iters = t;
  stats.converged = result == SPED_OK;
  SPED_TRY(copy_block(n, int(k), Q, kb, SPED_F32, V_out, ldvo, SPED_F32, s));
  SPED_CHECK_HIP(hipMemcpyAsync(h_flags, flags, sizeof(h_flags), hipMemcpyDeviceToHost, s));
  SPED_CHECK_HIP(hipStreamSynchronize(s));
  stats.cholqr_shifts = h_flags[0];
  stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  for (int i = 0; i < k; ++i) evals[i] = h_theta[i];
  if (resid_out)
    for (int i = 0; i < k; ++i) resid_out[i] = h_resid[i];
  if (st) *st = stats;
  if (result != SPED_OK) return fail(SPED_E_NOT_CONVERGED, "iteration cap reached before the tolerance");
  return SPED_OK;
}
