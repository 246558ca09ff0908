// Internal helpers shared by the libsped HIP sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <string>
#include <vector>

#include "sped.h"

namespace sped {

// the walk estimators read an entry record with one 32-byte load
static_assert(sizeof(sped_walk_entry) == 32 && alignof(sped_walk_entry) == 8, "walk entry layout");
static_assert(sizeof(sped_walk_node) == 16, "walk node layout");

// ---------------------------------------------------------------- errors
sped_status fail(sped_status st, const std::string &msg);
void clear_error();

#define SPED_CHECK_HIP(call)                                                      \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return ::sped::fail(SPED_E_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

#define SPED_TRY(expr)                   \
  do {                                   \
    sped_status s_ = (expr);             \
    if (s_ != SPED_OK) return s_;        \
  } while (0)

inline hipStream_t as_stream(sped_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- workspace carving
struct Carver {
  char *base;      // NULL in size-query mode
  size_t off = 0;
  explicit Carver(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  size_t bytes() const { return (off + 255) & ~size_t(255); }
};

// Size-query / size-check protocol shared by every entry point:
//   ws == NULL, ws_bytes != NULL  -> query: *ws_bytes = need, nothing runs
//   ws == NULL, ws_bytes == NULL  -> run without workspace (only if need == 0)
//   ws != NULL                    -> run; *ws_bytes must be >= need
inline sped_status check_ws(void *ws, size_t *ws_bytes, size_t need, bool *query) {
  if (!ws_bytes) {
    *query = false;
    if (ws || need == 0) return SPED_OK;
    return fail(SPED_E_WORKSPACE, "workspace of " + std::to_string(need) + " bytes required");
  }
  if (!ws) {
    *ws_bytes = need;
    *query = true;
    return SPED_OK;
  }
  *query = false;
  if (*ws_bytes < need)
    return fail(SPED_E_WORKSPACE, "workspace too small: need " + std::to_string(need) +
                                      " bytes, got " + std::to_string(*ws_bytes));
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(SPED_E_INVALID, "workspace not 256-byte aligned");
  return SPED_OK;
}

inline size_t dtype_size(int dt) { return dt == SPED_F64 ? 8 : dt == SPED_BF16 ? 2 : 4; }

sped_status validate_csr(const sped_csr *L);

// ---------------------------------------------------------------- bf16 storage
typedef uint16_t bf16_t;

__host__ __device__ inline float bf16_to_f32(bf16_t h) {
  uint32_t u = uint32_t(h) << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

// Round to nearest, ties to even; NaN stays NaN.
__host__ __device__ inline bf16_t f32_to_bf16(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return bf16_t((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return bf16_t(u >> 16);
}

template <typename T>
__device__ inline float to_f32(T x);
template <>
__device__ inline float to_f32<float>(float x) { return x; }
template <>
__device__ inline float to_f32<bf16_t>(bf16_t x) { return bf16_to_f32(x); }

template <typename T>
__device__ inline T from_f32(float x);
template <>
__device__ inline float from_f32<float>(float x) { return x; }
template <>
__device__ inline bf16_t from_f32<bf16_t>(float x) { return f32_to_bf16(x); }

// Vector load/store of VEC consecutive elements converted to/from float.
template <typename T, int VEC>
struct VecIO;

template <>
struct VecIO<float, 4> {
  __device__ static void load(const float *p, float (&o)[4]) {
    float4 v = *reinterpret_cast<const float4 *>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
  __device__ static void store(float *p, const float (&o)[4]) {
    *reinterpret_cast<float4 *>(p) = make_float4(o[0], o[1], o[2], o[3]);
  }
};
template <>
struct VecIO<float, 2> {
  __device__ static void load(const float *p, float (&o)[2]) {
    float2 v = *reinterpret_cast<const float2 *>(p);
    o[0] = v.x; o[1] = v.y;
  }
  __device__ static void store(float *p, const float (&o)[2]) {
    *reinterpret_cast<float2 *>(p) = make_float2(o[0], o[1]);
  }
};
template <>
struct VecIO<float, 1> {
  __device__ static void load(const float *p, float (&o)[1]) { o[0] = *p; }
  __device__ static void store(float *p, const float (&o)[1]) { *p = o[0]; }
};
template <>
struct VecIO<bf16_t, 4> {
  __device__ static void load(const bf16_t *p, float (&o)[4]) {
    uint2 v = *reinterpret_cast<const uint2 *>(p);
    o[0] = bf16_to_f32(bf16_t(v.x & 0xffff)); o[1] = bf16_to_f32(bf16_t(v.x >> 16));
    o[2] = bf16_to_f32(bf16_t(v.y & 0xffff)); o[3] = bf16_to_f32(bf16_t(v.y >> 16));
  }
  __device__ static void store(bf16_t *p, const float (&o)[4]) {
    uint2 v;
    v.x = uint32_t(f32_to_bf16(o[0])) | (uint32_t(f32_to_bf16(o[1])) << 16);
    v.y = uint32_t(f32_to_bf16(o[2])) | (uint32_t(f32_to_bf16(o[3])) << 16);
    *reinterpret_cast<uint2 *>(p) = v;
  }
};
template <>
struct VecIO<bf16_t, 2> {
  __device__ static void load(const bf16_t *p, float (&o)[2]) {
    uint32_t v = *reinterpret_cast<const uint32_t *>(p);
    o[0] = bf16_to_f32(bf16_t(v & 0xffff)); o[1] = bf16_to_f32(bf16_t(v >> 16));
  }
  __device__ static void store(bf16_t *p, const float (&o)[2]) {
    *reinterpret_cast<uint32_t *>(p) = uint32_t(f32_to_bf16(o[0])) | (uint32_t(f32_to_bf16(o[1])) << 16);
  }
};
template <>
struct VecIO<bf16_t, 1> {
  __device__ static void load(const bf16_t *p, float (&o)[1]) { o[0] = bf16_to_f32(*p); }
  __device__ static void store(bf16_t *p, const float (&o)[1]) { *p = f32_to_bf16(o[0]); }
};

// Streaming (non-temporal) variants: data read or written once per kernel,
// kept out of the way of the cache lines that gathers re-use.
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));

template <typename T, int VEC>
struct VecNT {
  __device__ static void store(T *p, const float (&o)[VEC]) { VecIO<T, VEC>::store(p, o); }
};
template <>
struct VecNT<float, 4> {
  __device__ static void store(float *p, const float (&o)[4]) {
    f32x4_t v = {o[0], o[1], o[2], o[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<f32x4_t *>(p));
  }
};
template <>
struct VecNT<float, 2> {
  __device__ static void store(float *p, const float (&o)[2]) {
    f32x2_t v = {o[0], o[1]};
    __builtin_nontemporal_store(v, reinterpret_cast<f32x2_t *>(p));
  }
};
template <>
struct VecNT<bf16_t, 4> {
  __device__ static void store(bf16_t *p, const float (&o)[4]) {
    u32x2_t v = {uint32_t(f32_to_bf16(o[0])) | (uint32_t(f32_to_bf16(o[1])) << 16),
                 uint32_t(f32_to_bf16(o[2])) | (uint32_t(f32_to_bf16(o[3])) << 16)};
    __builtin_nontemporal_store(v, reinterpret_cast<u32x2_t *>(p));
  }
};

// Eight elements per lane (16 bytes of bf16; two 16-byte halves of float).
template <>
struct VecIO<float, 8> {
  __device__ static void load(const float *p, float (&o)[8]) {
    const float4 a = reinterpret_cast<const float4 *>(p)[0], b = reinterpret_cast<const float4 *>(p)[1];
    o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w; o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
  }
  __device__ static void store(float *p, const float (&o)[8]) {
    reinterpret_cast<float4 *>(p)[0] = make_float4(o[0], o[1], o[2], o[3]);
    reinterpret_cast<float4 *>(p)[1] = make_float4(o[4], o[5], o[6], o[7]);
  }
};
template <>
struct VecIO<bf16_t, 8> {
  __device__ static void load(const bf16_t *p, float (&o)[8]) {
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = bf16_to_f32(bf16_t(w[i] & 0xffff));
      o[2 * i + 1] = bf16_to_f32(bf16_t(w[i] >> 16));
    }
  }
  __device__ static void store(bf16_t *p, const float (&o)[8]) {
    uint4 v;
    v.x = uint32_t(f32_to_bf16(o[0])) | (uint32_t(f32_to_bf16(o[1])) << 16);
    v.y = uint32_t(f32_to_bf16(o[2])) | (uint32_t(f32_to_bf16(o[3])) << 16);
    v.z = uint32_t(f32_to_bf16(o[4])) | (uint32_t(f32_to_bf16(o[5])) << 16);
    v.w = uint32_t(f32_to_bf16(o[6])) | (uint32_t(f32_to_bf16(o[7])) << 16);
    *reinterpret_cast<uint4 *>(p) = v;
  }
};
template <>
struct VecNT<float, 8> {
  __device__ static void store(float *p, const float (&o)[8]) {
    f32x4_t a = {o[0], o[1], o[2], o[3]}, b = {o[4], o[5], o[6], o[7]};
    __builtin_nontemporal_store(a, reinterpret_cast<f32x4_t *>(p));
    __builtin_nontemporal_store(b, reinterpret_cast<f32x4_t *>(p) + 1);
  }
};
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
template <>
struct VecNT<bf16_t, 8> {
  __device__ static void store(bf16_t *p, const float (&o)[8]) {
    u32x4_t v = {uint32_t(f32_to_bf16(o[0])) | (uint32_t(f32_to_bf16(o[1])) << 16),
                 uint32_t(f32_to_bf16(o[2])) | (uint32_t(f32_to_bf16(o[3])) << 16),
                 uint32_t(f32_to_bf16(o[4])) | (uint32_t(f32_to_bf16(o[5])) << 16),
                 uint32_t(f32_to_bf16(o[6])) | (uint32_t(f32_to_bf16(o[7])) << 16)};
    __builtin_nontemporal_store(v, reinterpret_cast<u32x4_t *>(p));
  }
};

// One neighbour row's VEC elements as loaded, before conversion: bf16 rows
// stay packed (two per register) until the multiply-add, so the 8 row loads a
// lane keeps in flight take half the registers.
template <typename T, int VEC>
struct RawRow {
  float f[VEC];
  __device__ void load(const T *p) { VecIO<T, VEC>::load(p, f); }
  __device__ void zero() {
#pragma unroll
    for (int v = 0; v < VEC; ++v) f[v] = 0.f;
  }
  __device__ float get(int v) const { return f[v]; }
};
template <int VEC>
struct RawRow<bf16_t, VEC> {
  static_assert(VEC % 2 == 0 || VEC == 1, "bf16 rows are held in pairs");
  static constexpr int W = VEC >= 2 ? VEC / 2 : 1;
  uint32_t w[W];
  __device__ void load(const bf16_t *p) {
    if constexpr (VEC == 8) {
      const uint4 v = *reinterpret_cast<const uint4 *>(p);
      w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    } else if constexpr (VEC == 4) {
      const uint2 v = *reinterpret_cast<const uint2 *>(p);
      w[0] = v.x; w[1] = v.y;
    } else if constexpr (VEC == 2) {
      w[0] = *reinterpret_cast<const uint32_t *>(p);
    } else {
      w[0] = uint32_t(*p);
    }
  }
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < W; ++i) w[i] = 0u;
  }
  __device__ float get(int v) const {
    const uint32_t x = w[v >> 1];
    return bf16_to_f32(bf16_t((v & 1) ? (x >> 16) : (x & 0xffff)));
  }
};

// Workgroups are handed to the 8 XCDs round-robin in dispatch order.  This
// maps hardware block b to logical block (b % 8) * per + b / 8 so that each
// XCD walks one contiguous stretch of logical blocks (rows), keeping the rows
// its neighbourhoods re-read in its own L2.  The grid is padded to 8 * per;
// logical ids >= nb have nothing to do.
constexpr int kXcds = 8;
__device__ inline int64_t xcd_logical_block(int64_t nb) {
  const int64_t per = gridDim.x / kXcds;
  const int64_t b = blockIdx.x;
  return (b % kXcds) * per + b / kXcds;
}
inline int64_t xcd_padded_grid(int64_t nb) { return (nb + kXcds - 1) / kXcds * kXcds; }

// Largest element vector width (4, 2 or 1) that divides k and every leading
// dimension and keeps every base pointer aligned.
int pick_vec(int64_t k, std::initializer_list<int64_t> lds, std::initializer_list<const void *> ptrs,
             std::initializer_list<int> elem_sizes);

// Allow a kernel more than 64 KiB of dynamic LDS (gfx950 has 160 KiB per CU).
template <typename F>
inline sped_status set_max_lds(F kernel, size_t bytes) {
  if (bytes > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
    if (e != hipSuccess) return fail(SPED_E_DEVICE, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  }
  return SPED_OK;
}

inline int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}
inline int ilog2(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

// ---------------------------------------------------------------- Philox4x32-10 / Lemire
// Salmon et al., SC'11: ten rounds of two 32x32->64 multiplies, key bumped by
// the Weyl constants between rounds.
struct Philox4 {
  uint32_t w[4];
};

__host__ __device__ inline Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = uint64_t(M0) * c0;
    uint64_t p1 = uint64_t(M1) * c2;
    uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
    uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  Philox4 o;
  o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
  return o;
}

// Lemire (2019) bounded draw in [0, s), 1 <= s < 2^32, from the word stream of
// counter (c0, c1, c2, (step << 8) | j), j = 0, 1, ...
// The rejection threshold (2^32 - s) mod s is below s, so a low word >= s is
// always accepted and the (slow) modulo is only needed when the low word falls
// below s; it is computed in 32 bits as (0 - s) mod s.  Same draws as testing
// every word against the threshold.
__host__ __device__ inline uint32_t lemire_draw(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                                                uint32_t c2, uint32_t step, uint32_t s) {
  uint32_t thresh = 0;
  bool have_thresh = false;
  for (uint32_t j = 0; j < 256; ++j) {
    Philox4 r = philox4x32_10(c0, c1, c2, (step << 8) | j, k0, k1);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint64_t m = uint64_t(r.w[i]) * s;
      const uint32_t lo = uint32_t(m);
      if (lo >= s) return uint32_t(m >> 32);
      if (!have_thresh) {
        thresh = (0u - s) % s;
        have_thresh = true;
      }
      if (lo >= thresh) return uint32_t(m >> 32);
    }
  }
  return 0;  // unreachable in practice: 1024 consecutive rejections
}

__host__ __device__ inline double uniform53(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                                            uint32_t c2, uint32_t step) {
  Philox4 r = philox4x32_10(c0, c1, c2, step << 8, k0, k1);
  uint64_t top = (uint64_t(r.w[0]) << 21) + (r.w[1] >> 11);
  return double(top) * 0x1.0p-53;
}

// ---------------------------------------------------------------- launches used across files
struct StepArgs {
  const void *U;  int64_t ldu; int tu;
  const void *V;  int64_t ldv; int tv;   // V may be NULL when g == 0
  void *O;        int64_t ldo; int to;
  float a, b, g;
  const float *dotw; int64_t lddw;      // non-NULL: accumulate <O, dotw>
  double *dot_partials;                 // [spmm_partials(L)]
  void *heavy_ws;                       // [spmm_step_ws_bytes(L, k)], 256-byte aligned; NULL if no heavy rows
};
// Scratch one fused step needs (the heavy rows' piece partials); 0 without heavy rows.
size_t spmm_step_ws_bytes(const sped_csr *L, int64_t k);
// One fused step O = a (L U) + b U + g V over all rows (light, medium, heavy bins).
sped_status launch_spmm_step(const sped_csr *L, int64_t k, const StepArgs &a, hipStream_t s,
                             int64_t *partials_written = nullptr);
int64_t spmm_partials(const sped_csr *L, int64_t k);

sped_status launch_reduce_partials(const double *partials, int64_t count, double *out, hipStream_t s);

sped_status validate_poly(const sped_poly *p);
// Coefficients of p in powers of L itself (binomial expansion of the shift, or
// of the limit product).
std::vector<double> monomial_in_L(const sped_poly &p);
sped_status launch_dot(int64_t n, int64_t k, const float *A, int64_t lda, const float *B, int64_t ldb,
                       double *partials, double *out, hipStream_t s);

// gram.hip
size_t gram_ws_doubles(int64_t n, int64_t ka, int64_t kb);
sped_status launch_gram(int64_t n, int ka, int kb, const void *A, int64_t lda, int ta, const void *B, int64_t ldb,
                        int tb, double *G, double *partials, hipStream_t s);
// O = X T (+ beta Y when Y is given; O may alias X or Y; Y and O float32)
sped_status launch_tsmm(int64_t n, int kin, int kout, const void *X, int64_t ldx, int tx, const double *T,
                        void *O, int64_t ldo, int to, hipStream_t s, const void *Y = nullptr, int64_t ldy = 0,
                        float beta = 0.f);
// G = R^T R for R = Z - Q diag(theta) (k columns, shared leading dimension
// ld), resid[i] = ||R e_i||, *norm2 >= ||R||_2 of the first kn columns.
// partials as for the symmetric Gram of width k.
sped_status launch_resid(int64_t n, int k, int kn, const float *Z, const void *Q, int64_t ld, int tq,
                         const double *theta, double *G, double *resid, double *norm2, double *partials,
                         hipStream_t s);

// dense.hip (flags: [0] Cholesky shifts, [1] Cholesky failures, [2] Jacobi caps)
int dense_max_k();
sped_status launch_chol_inv(int k, const double *G, double *T, double *R_out, int *flags, hipStream_t s);
// Sweeps stop once the off-diagonal Frobenius norm is at most rel times the
// whole matrix's; with rel_dev, rel is read from that device scalar instead.
sped_status launch_jacobi(int k, const double *H, double *theta, double *S, int *flags, hipStream_t s,
                          double rel = 1e-12, const double *rel_dev = nullptr);

// walk.hip
sped_status walk_estimate_impl(const sped_csr *L, const double *coeffs, int degree, int64_t k, const void *X,
                               int64_t ldx, int xdt, void *Y, int64_t ldy, int ydt, int sampler, int64_t walks,
                               uint64_t seed, uint64_t counter, int64_t *accept_counts, hipStream_t s);

// Y = sum_{i<m} c_i L^i X + L^m (walk estimate of the tail); T0 (m >= 1) and
// T1 (m >= 2) are n x k float32 scratch; counts the sparse steps.
sped_status hybrid_estimate_impl(const sped_csr *L, const double *coeffs, int degree, int m, int64_t k,
                                 const void *X, int64_t ldx, int xdt, void *Y, int64_t ldy, int ydt, int sampler,
                                 int64_t walks, uint64_t seed, uint64_t counter, float *T0, float *T1,
                                 void *step_ws, hipStream_t s, int64_t *spmm_count = nullptr);
// lazy node walks: the per-row largest move weight (n doubles; depends on the
// graph only), then the walk estimate of (I - L/ell)^ell X that uses it
sped_status lazy_row_max(const sped_csr *L, double *xmax, hipStream_t s);
sped_status lazy_walk_impl(const sped_csr *L, int ell, int64_t k, const void *X, int64_t ldx, int xdt, void *Y,
                           int64_t ldy, int ydt, int64_t walks, uint64_t seed, uint64_t counter, const double *xmax,
                           hipStream_t s);
sped_status validate_lazy(const sped_csr *L, int ell, int64_t walks, uint64_t counter);

// step_ws: spmm_step_ws_bytes(L, k) of scratch for every fused step
sped_status apply_poly_impl(const sped_csr *L, const sped_poly *p, int64_t k, const void *X,
                            int64_t ldx, int xdt, void *Y, int64_t ldy, int ydt, float *bufA,
                            float *bufB, void *step_ws, hipStream_t s, int64_t *spmm_count);

}  // namespace sped
