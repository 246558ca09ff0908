// Error state, argument validation helpers and small utility entry points.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"

namespace sped {

namespace {
thread_local std::string g_last_error;
}

sped_status fail(sped_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

void clear_error() { g_last_error.clear(); }

int pick_vec(int64_t k, std::initializer_list<int64_t> lds, std::initializer_list<const void *> ptrs,
             std::initializer_list<int> elem_sizes) {
  for (int vec : {4, 2}) {
    bool ok = (k % vec) == 0;
    for (int64_t ld : lds) ok = ok && (ld % vec) == 0;
    auto es = elem_sizes.begin();
    for (const void *p : ptrs) {
      int e = es != elem_sizes.end() ? *es++ : 4;
      if (p) ok = ok && (reinterpret_cast<uintptr_t>(p) % (uintptr_t(vec) * e)) == 0;
    }
    if (ok) return vec;
  }
  return 1;
}

sped_status validate_csr(const sped_csr *L) {
  if (!L) return fail(SPED_E_INVALID, "csr is NULL");
  if (L->n < 0 || L->n >= (int64_t(1) << 31)) return fail(SPED_E_INVALID, "csr n out of range");
  if (L->nnz < 0) return fail(SPED_E_INVALID, "csr nnz negative");
  if (L->n > 0 && (!L->rowptr || !L->diag || !L->scale))
    return fail(SPED_E_INVALID, "csr rowptr/diag/scale NULL");
  if (L->nnz > 0 && (!L->col || !L->val)) return fail(SPED_E_INVALID, "csr col/val NULL");
  if (L->n_medium < 0 || L->n_heavy < 0 || L->n_medium + L->n_heavy > L->n)
    return fail(SPED_E_INVALID, "csr bin counts out of range");
  if (L->n_medium + L->n_heavy > 0 && !L->bins) return fail(SPED_E_INVALID, "csr bins NULL");
  if (L->kind != SPED_LAP_COMBINATORIAL && L->kind != SPED_LAP_SYM_NORMALIZED)
    return fail(SPED_E_INVALID, "csr kind");
  return SPED_OK;
}

std::vector<double> monomial_in_L(const sped_poly &p) {
  const int ell = p.degree;
  std::vector<double> c(ell + 1, 0.0), out(ell + 1, 0.0);
  if (p.kind == SPED_POLY_LIMIT) {
    double binom = 1.0;
    for (int i = 0; i <= ell; ++i) {
      out[i] = binom * std::pow(-1.0 / ell, i);
      binom = binom * (ell - i) / (i + 1);
    }
    return out;
  }
  for (int i = 0; i <= ell; ++i) c[i] = p.coeffs[i];
  // ((L - a)/s)^i = s^-i sum_j C(i, j) L^j (-a)^(i-j)
  for (int i = 0; i <= ell; ++i) {
    double binom = 1.0;
    for (int j = 0; j <= i; ++j) {
      out[j] += c[i] * binom * std::pow(-p.shift, i - j) / std::pow(p.scale, i);
      binom = binom * (i - j) / (j + 1);
    }
  }
  return out;
}


namespace {
__global__ void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n16) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  size_t stride = size_t(gridDim.x) * blockDim.x;
  for (; i < n16; i += stride) dst[i] = src[i];
}

// Row-load rate probe: each wavefront loads 128-byte rows of `table` with 8
// lanes x 16 bytes per row and 8 rows per load instruction (the layout of the
// sparse step's neighbour-row gathers at 32 float32 columns), 8 loads in
// flight, `iters` rows per lane.  scattered: each 8-lane group takes its own
// pseudo-random row; otherwise the wavefront reads 8 consecutive rows (1 KB).
// Row indices are masked into the table.
__global__ __launch_bounds__(256) void gather_probe_kernel(const uint4 *__restrict__ table, uint32_t rows_mask,
                                                           int iters, int scattered, uint32_t *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 3, l8 = lane & 7;
  const uint32_t h = (blockIdx.x * 256u + threadIdx.x) * 2654435761u;
  uint32_t acc = 0;
  for (int it = 0; it < iters; it += 8) {
    uint4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      uint32_t x = h + uint32_t(it + u) * 0x9E3779B9u;
      if (scattered) x ^= uint32_t(g) * 0x85EBCA6Bu;
      x ^= x >> 15;
      x *= 0x2C1B3C6Du;
      x ^= x >> 12;
      uint32_t idx;
      if (scattered) {
        idx = (uint32_t(__shfl(int(x), lane & ~7, 64)) & rows_mask) * 8u + uint32_t(l8);
      } else {
        idx = (uint32_t(__shfl(int(x), 0, 64)) & (rows_mask & ~7u)) * 8u + uint32_t(lane);
      }
      v[u] = table[idx];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  out[blockIdx.x * 256u + threadIdx.x] = acc;
}
}  // namespace

}  // namespace sped

using namespace sped;

extern "C" const char *sped_last_error(void) { return g_last_error.c_str(); }

extern "C" int32_t sped_version(void) { return 1 * 10000 + 0 * 100 + 0; }

extern "C" sped_status sped_stream_copy(const void *src, void *dst, size_t bytes, sped_stream_t stream) {
  clear_error();
  if (bytes == 0) return SPED_OK;
  if (!src || !dst) return fail(SPED_E_INVALID, "NULL pointer");
  if ((bytes & 15) || (reinterpret_cast<uintptr_t>(src) & 15) || (reinterpret_cast<uintptr_t>(dst) & 15))
    return fail(SPED_E_INVALID, "copy needs 16-byte multiples and alignment");
  size_t n16 = bytes / 16;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 256 * 64) blocks = 256 * 64;
  hipLaunchKernelGGL(copy_kernel, dim3(unsigned(blocks)), dim3(256), 0, as_stream(stream),
                     static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n16);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

extern "C" sped_status sped_gather_probe(const void *table, int64_t rows, int32_t iters, int32_t scattered,
                                         int32_t blocks, uint32_t *out, sped_stream_t stream) {
  clear_error();
  if (!table || !out) return fail(SPED_E_INVALID, "NULL pointer");
  if (rows < 8 || rows > (int64_t(1) << 31) || (rows & (rows - 1)))
    return fail(SPED_E_INVALID, "rows must be a power of two in [8, 2^31]");
  if (iters < 8 || (iters & 7)) return fail(SPED_E_INVALID, "iters must be a positive multiple of 8");
  if (blocks < 1) return fail(SPED_E_INVALID, "blocks < 1");
  if (reinterpret_cast<uintptr_t>(table) & 15) return fail(SPED_E_INVALID, "table must be 16-byte aligned");
  hipLaunchKernelGGL(gather_probe_kernel, dim3(unsigned(blocks)), dim3(256), 0, as_stream(stream),
                     static_cast<const uint4 *>(table), uint32_t(rows - 1), int(iters), int(scattered != 0), out);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

extern "C" sped_status sped_transform_coeffs(int32_t transform, int32_t degree, double lambda_bound, double eps,
                                             double *coeffs, double *shift, double *scale) {
  clear_error();
  if (!coeffs || !shift || !scale) return fail(SPED_E_INVALID, "NULL output");
  if (!(std::isfinite(lambda_bound) && lambda_bound > 0.0)) return fail(SPED_E_INVALID, "lambda_bound");
  *shift = 0.0;
  *scale = 1.0;
  switch (transform) {
    case SPED_T_PLAIN:
      if (degree != 1) return fail(SPED_E_INVALID, "the plain operator has degree 1");
      coeffs[0] = lambda_bound;
      coeffs[1] = -1.0;
      return SPED_OK;
    case SPED_T_LIMIT: {
      if (degree < 1 || degree > 1024) return fail(SPED_E_INVALID, "degree");
      sped_poly p{SPED_POLY_LIMIT, degree, nullptr, 0.0, 1.0};
      std::vector<double> c = monomial_in_L(p);
      for (int i = 0; i <= degree; ++i) coeffs[i] = c[i];
      return SPED_OK;
    }
    case SPED_T_TAYLOR_EXP: {
      if (degree < 1 || degree > 1024) return fail(SPED_E_INVALID, "degree");
      double f = 1.0;  // (-1)^i / i!
      for (int i = 0; i <= degree; ++i) {
        coeffs[i] = f;
        f = -f / double(i + 1);
      }
      return SPED_OK;
    }
    case SPED_T_TAYLOR_LOG: {
      if (degree < 1 || degree > 1024) return fail(SPED_E_INVALID, "degree");
      // Table 2 takes l odd: an even-degree truncation of the log series turns
      // down at the top of [0, 2], so M would not reverse the spectrum.
      if (degree % 2 == 0) return fail(SPED_E_UNSUPPORTED, "Taylor log needs an odd degree");
      if (!(eps > 0.0 && eps < 1.0)) return fail(SPED_E_INVALID, "eps outside (0, 1)");
      const double y = lambda_bound - (1.0 - eps);
      double ftop = 0.0, yp = 1.0;
      for (int i = 1; i <= degree; ++i) {
        yp *= y;
        ftop += ((i & 1) ? 1.0 : -1.0) * yp / double(i);
      }
      coeffs[0] = ftop;
      for (int i = 1; i <= degree; ++i) coeffs[i] = ((i & 1) ? -1.0 : 1.0) / double(i);
      *shift = 1.0 - eps;
      return SPED_OK;
    }
    default:
      return fail(SPED_E_INVALID, "transform");
  }
}

extern "C" sped_status sped_poly_rebase(const sped_poly *p, double shift, double scale, double *out) {
  clear_error();
  SPED_TRY(validate_poly(p));
  if (!out) return fail(SPED_E_INVALID, "out NULL");
  if (!(std::isfinite(shift) && std::isfinite(scale) && scale != 0.0))
    return fail(SPED_E_INVALID, "shift and scale must be finite, scale nonzero");
  const int l = p->degree;
  if (p->kind == SPED_POLY_LIMIT) {
    // 1 - L/l = a + b Lt with a = 1 - shift/l, b = -scale/l: binomial expansion
    const double a = 1.0 - shift / l, b = -scale / l;
    double c = 1.0;  // C(l, i)
    for (int i = 0; i <= l; ++i) {
      out[i] = c * std::pow(a, l - i) * std::pow(b, i);
      c = c * double(l - i) / double(i + 1);
    }
    return SPED_OK;
  }
  // monomial in L first, then L = scale Lt + shift: Horner in the new variable
  std::vector<double> m = monomial_in_L(*p);
  std::vector<double> acc(size_t(l) + 1, 0.0);
  for (int j = l; j >= 0; --j) {  // acc <- acc * (scale Lt + shift) + m_j
    for (int i = l; i >= 1; --i) acc[i] = acc[i] * shift + acc[i - 1] * scale;
    acc[0] = acc[0] * shift + m[j];
  }
  for (int i = 0; i <= l; ++i) out[i] = acc[i];
  return SPED_OK;
}

extern "C" sped_status sped_poly_monomial(const sped_poly *p, double *out) {
  clear_error();
  SPED_TRY(validate_poly(p));
  if (!out) return fail(SPED_E_INVALID, "out NULL");
  std::vector<double> c = monomial_in_L(*p);
  for (int i = 0; i <= p->degree; ++i) out[i] = c[i];
  return SPED_OK;
}
