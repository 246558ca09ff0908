// Polynomial of the Laplacian applied to a block (Sec. 4.1-4.2, Table 2,
// reversed by eq. reveig) and the gradient of its coefficients.
//
// Horner's rule for M = sum_i c_i Lt^i, Lt = (L - shift I)/scale, costs one
// fused sparse step per degree:
//   U_1 = c_l Lt X + c_{l-1} X          (a = c_l/scale, b = c_{l-1} - c_l shift/scale)
//   U_i = Lt U_{i-1} + c_{l-i} X        (a = 1/scale,   b = -shift/scale, g = c_{l-i})
// and the limit form (I - L/l)^l is l steps of U <- U - L U / l.  Intermediate
// blocks are float32 in two workspace buffers used alternately.
#include <cmath>
#include <mutex>

#include "common.h"

namespace sped {

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void dot_kernel(int64_t n, int64_t k, const float *__restrict__ A,
                                                     int64_t lda, const float *__restrict__ B,
                                                     int64_t ldb, double *__restrict__ partials) {
  __shared__ double red[kBlock / 64];
  double s = 0.0;
  const int64_t total = n * k;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < total; i += int64_t(gridDim.x) * kBlock) {
    int64_t r = i / k, c = i - r * k;
    s += double(A[r * lda + c]) * double(B[r * ldb + c]);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

constexpr int kDotBlocks = 1024;

sped_status validate_block(const void *p, int64_t n, int64_t k, int64_t ld, int dt, const char *name) {
  if (n > 0 && k > 0 && !p) return fail(SPED_E_INVALID, std::string(name) + " is NULL");
  if (ld < k) return fail(SPED_E_INVALID, std::string(name) + " leading dimension < k");
  if (dt != SPED_F32 && dt != SPED_BF16) return fail(SPED_E_UNSUPPORTED, std::string(name) + " dtype");
  return SPED_OK;
}

}  // namespace

sped_status apply_poly_impl(const sped_csr *L, const sped_poly *p, int64_t k, const void *X,
                            int64_t ldx, int xdt, void *Y, int64_t ldy, int ydt, float *bufA,
                            float *bufB, void *step_ws, hipStream_t s, int64_t *spmm_count) {
  const int ell = p->degree;
  float *buf[2] = {bufA, bufB};
  const void *in = X;
  int64_t ldin = ldx;
  int tin = xdt;
  for (int i = 1; i <= ell; ++i) {
    StepArgs a{};
    a.heavy_ws = step_ws;
    a.U = in; a.ldu = ldin; a.tu = tin;
    a.V = X; a.ldv = ldx; a.tv = xdt;
    if (i == ell) {
      a.O = Y; a.ldo = ldy; a.to = ydt;
    } else {
      a.O = buf[(i - 1) & 1]; a.ldo = k; a.to = SPED_F32;
    }
    if (p->kind == SPED_POLY_LIMIT) {
      a.a = float(-1.0 / ell); a.b = 1.f; a.g = 0.f;
    } else {
      const double *c = p->coeffs;
      const double tau = p->scale, sig = p->shift;
      if (i == 1) {
        a.a = float(c[ell] / tau);
        a.b = float(c[ell - 1] - c[ell] * sig / tau);
        a.g = 0.f;
      } else {
        a.a = float(1.0 / tau);
        a.b = float(-sig / tau);
        a.g = float(c[ell - i]);
      }
    }
    SPED_TRY(launch_spmm_step(L, k, a, s));
    in = a.O; ldin = a.ldo; tin = a.to;
  }
  if (spmm_count) *spmm_count += ell;
  return SPED_OK;
}

sped_status validate_poly(const sped_poly *p) {
  if (!p) return fail(SPED_E_INVALID, "poly is NULL");
  if (p->degree < 1 || p->degree > 1024) return fail(SPED_E_INVALID, "poly degree outside [1, 1024]");
  if (p->kind == SPED_POLY_MONOMIAL) {
    if (!p->coeffs) return fail(SPED_E_INVALID, "poly coeffs NULL");
    if (!(std::isfinite(p->scale) && p->scale != 0.0) || !std::isfinite(p->shift))
      return fail(SPED_E_INVALID, "poly shift/scale");
    for (int i = 0; i <= p->degree; ++i)
      if (!std::isfinite(p->coeffs[i])) return fail(SPED_E_INVALID, "poly coefficient not finite");
  } else if (p->kind != SPED_POLY_LIMIT) {
    return fail(SPED_E_INVALID, "poly kind");
  }
  return SPED_OK;
}

sped_status launch_dot(int64_t n, int64_t k, const float *A, int64_t lda, const float *B, int64_t ldb,
                       double *partials, double *out, hipStream_t s) {
  hipLaunchKernelGGL(dot_kernel, dim3(kDotBlocks), dim3(kBlock), 0, s, n, k, A, lda, B, ldb, partials);
  SPED_CHECK_HIP(hipGetLastError());
  return launch_reduce_partials(partials, kDotBlocks, out, s);
}

}  // namespace sped

using namespace sped;

extern "C" sped_status sped_apply_poly(const sped_csr *L, const sped_poly *p, int64_t k, const void *X,
                                       int64_t ldx, int32_t xdt, void *Y, int64_t ldy, int32_t ydt,
                                       void *ws, size_t *ws_bytes, sped_stream_t stream) {
  clear_error();
  SPED_TRY(validate_csr(L));
  SPED_TRY(validate_poly(p));
  if (k < 1) return fail(SPED_E_INVALID, "k < 1");
  SPED_TRY(validate_block(X, L->n, k, ldx, xdt, "X"));
  SPED_TRY(validate_block(Y, L->n, k, ldy, ydt, "Y"));
  const int nbuf = p->degree >= 3 ? 2 : p->degree - 1;
  Carver c(ws);
  float *A = nbuf >= 1 ? c.take<float>(size_t(L->n) * k) : nullptr;
  float *B = nbuf >= 2 ? c.take<float>(size_t(L->n) * k) : nullptr;
  const size_t sw = spmm_step_ws_bytes(L, k);
  void *step_ws = sw ? c.take<char>(sw) : nullptr;
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, c.bytes(), &query));
  if (query || L->n == 0) return SPED_OK;
  // X and Y must not overlap (the Horner term g X is re-read every step)
  const char *xb = static_cast<const char *>(X), *yb = static_cast<const char *>(Y);
  size_t xs = size_t((L->n - 1) * ldx + k) * dtype_size(xdt), ys = size_t((L->n - 1) * ldy + k) * dtype_size(ydt);
  if (xb < yb + ys && yb < xb + xs) return fail(SPED_E_INVALID, "X and Y overlap");
  return apply_poly_impl(L, p, k, X, ldx, xdt, Y, ldy, ydt, A, B, step_ws, as_stream(stream), nullptr);
}

// Allocation-free form of sped_apply_poly: the chain's intermediate float32
// blocks live in this library-owned array instead of a caller workspace.  Each
// GPU the library runs on holds its own copy from the module's load until the
// process ends.  In host code `scratch` names a host-side stand-in: kernels get
// the device address that hipGetSymbolAddress returns for the current device.
namespace {
constexpr size_t kScratchBytes = SPED_NOALLOC_SCRATCH_BYTES;
constexpr int kScratchDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
sped_status scratch_address(void **out) {
  int dev = -1;
  SPED_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return fail(SPED_E_DEVICE, "device ordinal outside the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail(SPED_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    if (!p) return fail(SPED_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SPED_OK;
}
}  // namespace

extern "C" sped_status sped_apply_poly_noalloc(const sped_csr *L, const sped_poly *p, int64_t k, const void *X,
                                               int64_t ldx, int32_t xdt, void *Y, int64_t ldy, int32_t ydt,
                                               sped_stream_t stream) {
  clear_error();
  SPED_TRY(validate_csr(L));
  SPED_TRY(validate_poly(p));
  if (k < 1) return fail(SPED_E_INVALID, "k < 1");
  SPED_TRY(validate_block(X, L->n, k, ldx, xdt, "X"));
  SPED_TRY(validate_block(Y, L->n, k, ldy, ydt, "Y"));
  // the same two buffers sped_apply_poly carves from its workspace, each
  // rounded up to 256 bytes
  const int nbuf = p->degree >= 3 ? 2 : p->degree - 1;
  const size_t one = (size_t(L->n) * size_t(k) * sizeof(float) + 255) / 256 * 256;
  if (L->n > 0 && k > int64_t(kScratchBytes / sizeof(float)) / L->n)
    return fail(SPED_E_WORKSPACE, "n x k beyond the allocation-free scratch (64 MiB)");
  const size_t sw = (spmm_step_ws_bytes(L, k) + 255) / 256 * 256;
  if (size_t(nbuf) * one + sw > kScratchBytes)
    return fail(SPED_E_WORKSPACE, "n x k beyond the allocation-free scratch: " +
                                      std::to_string(size_t(nbuf) * one + sw) + " bytes needed, 64 MiB available");
  if (L->n == 0) return SPED_OK;
  const char *xb = static_cast<const char *>(X), *yb = static_cast<const char *>(Y);
  size_t xs = size_t((L->n - 1) * ldx + k) * dtype_size(xdt), ys = size_t((L->n - 1) * ldy + k) * dtype_size(ydt);
  if (xb < yb + ys && yb < xb + xs) return fail(SPED_E_INVALID, "X and Y overlap");
  void *base = nullptr;
  SPED_TRY(scratch_address(&base));
  float *A = nbuf >= 1 ? static_cast<float *>(base) : nullptr;
  float *B = nbuf >= 2 ? reinterpret_cast<float *>(static_cast<char *>(base) + one) : nullptr;
  void *step_ws = sw ? static_cast<char *>(base) + size_t(nbuf) * one : nullptr;
  return apply_poly_impl(L, p, k, X, ldx, xdt, Y, ldy, ydt, A, B, step_ws, as_stream(stream), nullptr);
}

extern "C" sped_status sped_poly_backward(const sped_csr *L, int32_t degree, double shift, double scale,
                                          int64_t k, const float *X, int64_t ldx, const float *dY,
                                          int64_t lddy, double *dtheta, void *ws, size_t *ws_bytes,
                                          sped_stream_t stream) {
  clear_error();
  SPED_TRY(validate_csr(L));
  if (degree < 0 || degree > 1024) return fail(SPED_E_INVALID, "degree outside [0, 1024]");
  if (!(std::isfinite(scale) && scale != 0.0) || !std::isfinite(shift))
    return fail(SPED_E_INVALID, "shift/scale");
  if (k < 1) return fail(SPED_E_INVALID, "k < 1");
  SPED_TRY(validate_block(X, L->n, k, ldx, SPED_F32, "X"));
  SPED_TRY(validate_block(dY, L->n, k, lddy, SPED_F32, "dY"));
  if (!dtheta) return fail(SPED_E_INVALID, "dtheta is NULL");
  Carver c(ws);
  float *P[2] = {c.take<float>(size_t(L->n) * k), c.take<float>(size_t(L->n) * k)};
  int64_t np = spmm_partials(L, k);
  double *partials = c.take<double>(size_t(np > kDotBlocks ? np : kDotBlocks));
  const size_t sw = spmm_step_ws_bytes(L, k);
  void *step_ws = sw ? c.take<char>(sw) : nullptr;
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, c.bytes(), &query));
  if (query) return SPED_OK;
  hipStream_t s = as_stream(stream);
  if (L->n == 0) {
    SPED_CHECK_HIP(hipMemsetAsync(dtheta, 0, sizeof(double) * (degree + 1), s));
    return SPED_OK;
  }
  SPED_TRY(launch_dot(L->n, k, X, ldx, dY, lddy, partials, dtheta, s));
  const float *in = X;
  int64_t ldin = ldx;
  for (int j = 1; j <= degree; ++j) {
    StepArgs a{};
    a.U = in; a.ldu = ldin; a.tu = SPED_F32;
    a.V = nullptr; a.ldv = k; a.tv = SPED_F32;
    a.O = P[(j - 1) & 1]; a.ldo = k; a.to = SPED_F32;
    a.a = float(1.0 / scale); a.b = float(-shift / scale); a.g = 0.f;
    a.dotw = dY; a.lddw = lddy; a.dot_partials = partials;
    a.heavy_ws = step_ws;
    int64_t written = 0;
    SPED_TRY(launch_spmm_step(L, k, a, s, &written));
    SPED_TRY(launch_reduce_partials(partials, written, dtheta + j, s));
    in = P[(j - 1) & 1];
    ldin = k;
  }
  return SPED_OK;
}
