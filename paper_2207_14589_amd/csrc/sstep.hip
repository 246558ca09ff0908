// Two consecutive fused steps per launch on row blocks held in LDS (a
// matrix-powers form of the chain p(L) X for graphs whose rows are ordered by
// community; Sec. 4.3 weighs ways of forming a product of l factors, and this
// fuses consecutive factors per block of rows):
//   U1 = a1 (L U) + b1 U + g1 X,   U2 = a2 (L U1) + b2 U1 + g2 X
// One workgroup owns the B consecutive rows [b B, (b+1) B).  It loads those
// rows of U into LDS with coalesced reads, forms U1 for them (neighbour rows
// inside the block come from LDS, the others from U in global memory), keeps
// U1 in registers, overwrites the LDS copy with it, and forms U2 (neighbour
// rows inside the block from LDS; for a neighbour j outside the block the
// group recomputes U1[j] from U in global memory, since another workgroup
// owns it).  U1 never reaches global memory, and most neighbour-row reads
// are LDS reads instead of texture-path gathers.  The result equals two
// single steps up to the order of the float32 sums.
#include <algorithm>

#include "common.h"

namespace sped {
namespace {

constexpr int kMaxThreads = 1024;
constexpr int kMaxRowsPerGroup = 8;
constexpr size_t kMaxLds = 160 * 1024;

struct Coef2 {
  float a, b, g;
};

typedef int32_t i4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

// 4 consecutive (col, val) entries from position q on (16-byte loads; the
// arrays' last entries one by one; entries at or past nnz read as 0).
__device__ inline void load_entries4(const int32_t *__restrict__ col, const float *__restrict__ val, int64_t q,
                                     int64_t nnz, i4u &c4, f4u &v4) {
  if (q + 3 < nnz) {
    c4 = *reinterpret_cast<const i4u *>(col + q);
    v4 = *reinterpret_cast<const f4u *>(val + q);
  } else {
    c4 = i4u{0, 0, 0, 0};
    v4 = f4u{0.f, 0.f, 0.f, 0.f};
    for (int i = 0; i < 4; ++i)
      if (q + i < nnz) {
        c4[i] = col[q + i];
        v4[i] = val[q + i];
      }
  }
}

__device__ inline void load4(const float *p, float (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4 *>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}

// Sum over the entries [beg, end) of a row of S_rj F(j) for this lane's 4
// columns.  `where(j)` returns the LDS offset of neighbour row j's 4 values
// when row j is in the block, -1 when it must be read from global memory at
// `gsrc + j * ldg`, and -2 to drop the term.  The G lanes of the group share
// each chunk of 4G entries (two 16-byte loads per lane, broadcast by
// shuffle).  Each batch of 8 issues 8 LDS reads unconditionally (an entry
// outside the block or past the row's end reads the group's own row) and the
// rare global reads under a branch; dropped terms are masked off bitwise.
template <typename Where>
__device__ inline void row_sum(const float *lds, int own_off, const float *__restrict__ gsrc, int64_t ldg, int c0,
                               const int32_t *__restrict__ col, const float *__restrict__ val, int64_t beg,
                               int64_t end, int64_t nnz, int G, int lig, Where where, float (&acc)[4]) {
  const int C = 4 * G;
  for (int64_t p = beg; p < end; p += C) {
    i4u c4;
    f4u v4;
    load_entries4(col, val, p + 4 * lig, nnz, c4, v4);
    const int cnt = int(min<int64_t>(C, end - p));
    for (int t = 0; t < cnt; t += 8) {
      int off[8];
      int32_t j[8];
      float sv[8];
      bool any_global = false;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int src = ((t + u) >> 2) & (G - 1);
        j[u] = __shfl(c4[u & 3], src, G);
        sv[u] = __shfl(v4[u & 3], src, G);
        off[u] = t + u < cnt ? where(j[u]) : -2;
        any_global |= off[u] == -1;
      }
      float x[8][4];
#pragma unroll
      for (int u = 0; u < 8; ++u) load4(lds + (off[u] >= 0 ? off[u] : own_off), x[u]);
      if (any_global) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (off[u] == -1) load4(gsrc + int64_t(j[u]) * ldg + c0, x[u]);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t km = off[u] != -2 ? 0xffffffffu : 0u;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          acc[v] = fmaf(__uint_as_float(__float_as_uint(sv[u]) & km), __uint_as_float(__float_as_uint(x[u][v]) & km),
                        acc[v]);
      }
    }
  }
}

// Global-only form of row_sum for the recomputed neighbours outside the block.
__device__ inline void row_sum_global(const int32_t *__restrict__ col, const float *__restrict__ val, int64_t beg,
                                      int64_t end, int64_t nnz, int G, int lig, const float *__restrict__ U,
                                      int64_t ldu, int c0, float (&acc)[4]) {
  const int C = 4 * G;
  for (int64_t p = beg; p < end; p += C) {
    i4u c4;
    f4u v4;
    load_entries4(col, val, p + 4 * lig, nnz, c4, v4);
    const int cnt = int(min<int64_t>(C, end - p));
    for (int t = 0; t < cnt; t += 8) {
      int32_t j[8];
      float sv[8];
      uint32_t km[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int src = ((t + u) >> 2) & (G - 1);
        j[u] = __shfl(c4[u & 3], src, G);
        sv[u] = __shfl(v4[u & 3], src, G);
        km[u] = t + u < cnt ? 0xffffffffu : 0u;
      }
      float x[8][4];
#pragma unroll
      for (int u = 0; u < 8; ++u) load4(U + int64_t(t + u < cnt ? j[u] : j[0]) * ldu + c0, x[u]);
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          acc[v] = fmaf(__uint_as_float(__float_as_uint(sv[u]) & km[u]),
                        __uint_as_float(__float_as_uint(x[u][v]) & km[u]), acc[v]);
    }
  }
}

template <int kThreads, int kRows>
__global__ __launch_bounds__(kThreads) void two_steps_kernel(
    int64_t n, int B, int k, int G, int lgG, int64_t nnz, const int64_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const float *__restrict__ val, const float *__restrict__ diag,
    const float *__restrict__ U, int64_t ldu, const float *__restrict__ X, int64_t ldx, float *__restrict__ O,
    int64_t ldo, Coef2 c1, Coef2 c2) {
  extern __shared__ float lds[];  // B x k: U of the block, then U1
  const int64_t base = int64_t(blockIdx.x) * B;
  const int rows = int(min<int64_t>(B, n - base));
  // coalesced load of the block's rows of U
  const int k4 = k >> 2;
  for (int i = threadIdx.x; i < rows * k4; i += kThreads) {
    const int r = i / k4, c = (i - r * k4) * 4;
    *reinterpret_cast<float4 *>(lds + r * k + c) = *reinterpret_cast<const float4 *>(U + (base + r) * ldu + c);
  }
  __syncthreads();
  const int lig = threadIdx.x & (G - 1);
  const int grp = threadIdx.x >> lgG;
  const int groups = kThreads >> lgG;
  const int c0 = lig * 4;
  auto dg_of = [&](int64_t r, int64_t b, int64_t e) { return diag ? diag[r] : (e > b ? 1.f : 0.f); };
  // neighbour rows of U: LDS inside the block, global memory outside
  auto fetch_u = [&](int32_t j) -> int {
    const int64_t jl = int64_t(j) - base;
    return (jl >= 0 && jl < rows) ? int(jl) * k + c0 : -1;
  };
  // step 1 for this group's rows, kept in registers
  float u1[kRows][4];
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const int rl = grp + i * groups;
    if (rl < rows) {
      const int64_t r = base + rl;
      const int64_t beg = rowptr[r], end = rowptr[r + 1];
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
      row_sum(lds, rl * k + c0, U, ldu, c0, col, val, beg, end, nnz, G, lig, fetch_u, acc);
      float u[4], x[4] = {0.f, 0.f, 0.f, 0.f};
      load4(lds + rl * k + c0, u);
      if (c1.g != 0.f) load4(X + r * ldx + c0, x);
      const float dg = dg_of(r, beg, end);
#pragma unroll
      for (int v = 0; v < 4; ++v) u1[i][v] = fmaf(c1.g, x[v], c1.a * (dg * u[v] - acc[v]) + c1.b * u[v]);
    }
  }
  __syncthreads();  // every group has read U from LDS
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const int rl = grp + i * groups;
    if (rl < rows) *reinterpret_cast<float4 *>(lds + rl * k + c0) = make_float4(u1[i][0], u1[i][1], u1[i][2], u1[i][3]);
  }
  __syncthreads();
  // neighbour rows of U1 inside the block (LDS); outside terms are dropped here
  auto fetch_u1_in = [&](int32_t j) -> int {
    const int64_t jl = int64_t(j) - base;
    return (jl >= 0 && jl < rows) ? int(jl) * k + c0 : -2;  // outside: dropped here
  };
#pragma unroll 1
  for (int i = 0; i < kRows; ++i) {
    const int rl = grp + i * groups;
    if (rl >= rows) continue;
    const int64_t r = base + rl;
    const int64_t beg = rowptr[r], end = rowptr[r + 1];
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    row_sum(lds, rl * k + c0, U, ldu, c0, col, val, beg, end, nnz, G, lig, fetch_u1_in, acc);
    // neighbours outside the block: U1[j] recomputed from U
    const int C = 4 * G;
    for (int64_t p = beg; p < end; p += C) {
      i4u c4;
      f4u v4;
      load_entries4(col, val, p + 4 * lig, nnz, c4, v4);
      const int cnt = int(min<int64_t>(C, end - p));
      for (int t = 0; t < cnt; ++t) {
        const int src = (t >> 2) & (G - 1);
        int32_t c4t = c4[0];
        float v4t = v4[0];
        switch (t & 3) {  // component t % 4 of lane t / 4
          case 1: c4t = c4[1]; v4t = v4[1]; break;
          case 2: c4t = c4[2]; v4t = v4[2]; break;
          case 3: c4t = c4[3]; v4t = v4[3]; break;
          default: break;
        }
        const int32_t j = __shfl(c4t, src, G);
        const float s = __shfl(v4t, src, G);
        const int64_t jl = int64_t(j) - base;
        if (jl >= 0 && jl < rows) continue;  // uniform over the group
        const int64_t jb = rowptr[j], je = rowptr[int64_t(j) + 1];
        float hacc[4] = {0.f, 0.f, 0.f, 0.f};
        row_sum_global(col, val, jb, je, nnz, G, lig, U, ldu, c0, hacc);
        float uj[4], xj[4] = {0.f, 0.f, 0.f, 0.f};
        load4(U + int64_t(j) * ldu + c0, uj);
        if (c1.g != 0.f) load4(X + int64_t(j) * ldx + c0, xj);
        const float dgj = dg_of(j, jb, je);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const float u1j = fmaf(c1.g, xj[w], c1.a * (dgj * uj[w] - hacc[w]) + c1.b * uj[w]);
          acc[w] = fmaf(s, u1j, acc[w]);
        }
      }
    }
    float u[4], x[4] = {0.f, 0.f, 0.f, 0.f};
    load4(lds + rl * k + c0, u);
    if (c2.g != 0.f) load4(X + r * ldx + c0, x);
    const float dg = dg_of(r, beg, end);
    float o[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) o[v] = fmaf(c2.g, x[v], c2.a * (dg * u[v] - acc[v]) + c2.b * u[v]);
    *reinterpret_cast<float4 *>(O + r * ldo + c0) = make_float4(o[0], o[1], o[2], o[3]);
  }
}

// Coefficients of step i (1-based) of the chain for p (as in the single-step
// chain: Horner for the monomial form, one factor per step for the limit form).
Coef2 step_coef(const sped_poly *p, int i) {
  const int ell = p->degree;
  if (p->kind == SPED_POLY_LIMIT) return Coef2{float(-1.0 / ell), 1.f, 0.f};
  const double *c = p->coeffs;
  const double tau = p->scale, sig = p->shift;
  if (i == 1) return Coef2{float(c[ell] / tau), float(c[ell - 1] - c[ell] * sig / tau), 0.f};
  return Coef2{float(1.0 / tau), float(-sig / tau), float(c[ell - i])};
}

}  // namespace
}  // namespace sped

using namespace sped;

extern "C" sped_status sped_apply_poly_blocked(const sped_csr *L, const sped_poly *p, int64_t block_rows,
                                               int64_t k, const void *X, int64_t ldx, int32_t xdt, void *Y,
                                               int64_t ldy, int32_t ydt, void *ws, size_t *ws_bytes,
                                               sped_stream_t stream) {
  clear_error();
  SPED_TRY(validate_csr(L));
  SPED_TRY(validate_poly(p));
  if (xdt != SPED_F32 || ydt != SPED_F32) return fail(SPED_E_UNSUPPORTED, "blocked chain: X and Y must be F32");
  if (k != 4 && k != 8 && k != 16 && k != 32 && k != 64)
    return fail(SPED_E_UNSUPPORTED, "blocked chain: k must be 4, 8, 16, 32 or 64");
  if (ldx < k || ldy < k || (ldx & 3) || (ldy & 3)) return fail(SPED_E_INVALID, "leading dimension");
  const int G = int(k / 4), lgG = ilog2(G);
  const int groups = kMaxThreads / G;
  if (block_rows < 1 || block_rows > int64_t(kMaxRowsPerGroup) * groups ||
      size_t(block_rows) * size_t(k) * sizeof(float) > kMaxLds)
    return fail(SPED_E_INVALID, "block_rows outside [1, min(8 x 4096 / k, 160 KiB / (4 k))]");
  if (L->n > 0 && (!X || !Y)) return fail(SPED_E_INVALID, "X or Y NULL");
  if ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) & 15)
    return fail(SPED_E_INVALID, "X and Y must be 16-byte aligned");
  const int ell = p->degree;
  const int nbuf = ell >= 3 ? 2 : ell - 1;
  Carver c(ws);
  float *buf[2] = {nbuf >= 1 ? c.take<float>(size_t(L->n) * k) : nullptr,
                   nbuf >= 2 ? c.take<float>(size_t(L->n) * k) : nullptr};
  const size_t sw = spmm_step_ws_bytes(L, k);
  void *step_ws = sw ? c.take<char>(sw) : nullptr;
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, c.bytes(), &query));
  if (query || L->n == 0) return SPED_OK;
  const char *xb = static_cast<const char *>(X), *yb = static_cast<const char *>(Y);
  size_t xs = size_t((L->n - 1) * ldx + k) * 4, ys = size_t((L->n - 1) * ldy + k) * 4;
  if (xb < yb + ys && yb < xb + xs) return fail(SPED_E_INVALID, "X and Y overlap");
  hipStream_t s = as_stream(stream);
  const size_t lds = size_t(block_rows) * size_t(k) * sizeof(float);
  // 256 threads when they hold the block (more workgroups per CU), else 1024;
  // rows per lane group 4 when that suffices (fewer registers)
  const int variant = block_rows <= int64_t(4) * (256 / G) ? 0 : block_rows <= int64_t(8) * (256 / G) ? 1 : 2;
  SPED_TRY(variant == 0   ? set_max_lds(two_steps_kernel<256, 4>, lds)
           : variant == 1 ? set_max_lds(two_steps_kernel<256, 8>, lds)
                          : set_max_lds(two_steps_kernel<1024, 8>, lds));
  const float *diag = L->kind == SPED_LAP_SYM_NORMALIZED ? nullptr : L->diag;
  const float *in = static_cast<const float *>(X);
  int64_t ldin = ldx;
  int next = 0;
  int i = 1;
  for (; i + 1 <= ell; i += 2) {  // steps i and i + 1 in one launch
    float *out;
    int64_t ldout;
    if (i + 1 == ell) {
      out = static_cast<float *>(Y);
      ldout = ldy;
    } else {
      out = buf[next];
      ldout = k;
      next ^= 1;
    }
    const unsigned grid = unsigned((L->n + block_rows - 1) / block_rows);
#define SPED_TWO(T_, R_)                                                                                      \
  hipLaunchKernelGGL((two_steps_kernel<T_, R_>), dim3(grid), dim3(T_), lds, s, L->n, int(block_rows), int(k), G, \
                     lgG, L->nnz, L->rowptr, L->col, L->val, diag, in, ldin, static_cast<const float *>(X), ldx,  \
                     out, ldout, step_coef(p, i), step_coef(p, i + 1))
    if (variant == 0) SPED_TWO(256, 4);
    else if (variant == 1) SPED_TWO(256, 8);
    else SPED_TWO(1024, 8);
#undef SPED_TWO
    SPED_CHECK_HIP(hipGetLastError());
    in = out;
    ldin = ldout;
  }
  if (i == ell) {  // odd degree: the last step alone
    const Coef2 cf = step_coef(p, i);
    StepArgs a{};
    a.heavy_ws = step_ws;
    a.U = in; a.ldu = ldin; a.tu = SPED_F32;
    a.V = X; a.ldv = ldx; a.tv = SPED_F32;
    a.O = Y; a.ldo = ldy; a.to = SPED_F32;
    a.a = cf.a; a.b = cf.b; a.g = cf.g;
    SPED_TRY(launch_spmm_step(L, k, a, s));
  }
  return SPED_OK;
}
