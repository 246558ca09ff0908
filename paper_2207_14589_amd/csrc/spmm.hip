// Fused sparse-Laplacian x block step (the inner operation of p(L)V, Sec. 4.2):
//     O = a (L U) + b U + g V,   L U = diag .* U - S U
// over the split CSR of sped.h.  One step of Horner's rule (a = 1/scale,
// b = -shift/scale, g = c_i), one factor of the limit product (a = -1/l, b = 1,
// g = 0) or a plain product (a = 1, b = g = 0) is one launch set.  Optionally
// the inner product <O, W> is accumulated in float64 (coefficient gradients).
//
// Rows are binned by their number of stored entries d:
//   light   d <= SPED_LIGHT_MAX : a group of G lanes per row, 256/G rows per block
//   medium  d <= SPED_MEDIUM_MAX: one 64-lane wavefront per row, 64/G lane groups
//           split the entries, partial sums meet by cross-lane xor shuffles
//   heavy   d >  SPED_MEDIUM_MAX: the row is cut into pieces of kPiece entries;
//           each piece is one 256-thread block (LDS reduction) that writes its
//           partial sum to the step workspace, and a second kernel adds a
//           row's partials in piece order and applies the epilogue, so a hub
//           row spreads over many CUs and the result is deterministic
// Each lane owns VEC consecutive columns; G = next_pow2(k / VEC) lanes cover
// a row of the block (columns beyond 64 VEC are tiled over blockIdx.y).  The
// G lanes of a group load 4G consecutive (col, val) pairs with two 16-byte
// loads per lane, broadcast them by shuffle, and issue 8 neighbour-row gathers
// before consuming any, so each lane keeps 8 row gathers in flight.
#include <algorithm>
#include <type_traits>

#include "common.h"

namespace sped {
namespace {

constexpr int kBlock = 256;

struct Coef {
  float a, b, g;
};

template <typename TU, typename TV, typename TO, int VEC, bool DOT>
struct Step {
  // 4 consecutive entries of each index array from entry a on, as one 16-byte
  // load each (dword alignment suffices); entries at or past nnz read as 0.
  typedef int32_t i4u __attribute__((ext_vector_type(4), aligned(4)));
  typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
  __device__ static void load_idx4(const int32_t *__restrict__ col, const float *__restrict__ val, int64_t a,
                                   int64_t nnz, i4u &c4, f4u &v4) {
    if (a + 3 < nnz) {
      c4 = __builtin_nontemporal_load(reinterpret_cast<const i4u *>(col + a));
      v4 = __builtin_nontemporal_load(reinterpret_cast<const f4u *>(val + a));
    } else {
      c4 = i4u{0, 0, 0, 0};
      v4 = f4u{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (a + i < nnz) {
          c4[i] = col[a + i];
          v4[i] = val[a + i];
        }
    }
  }

  // Accumulate sum_p S_rp U[col_p, c0 .. c0+VEC) over entries [beg, end),
  // handled by the G lanes of one group (lane `lig`) in chunks of C = 4G
  // entries that start at beg + first*C and advance by stride*C.  Each lane
  // loads 4 consecutive entries of each index array with one 16-byte load
  // (dword-aligned; the last 3 entries of the arrays are read one by one), so a
  // chunk of 4G entries costs two index loads instead of eight.  A load
  // instruction occupies the texture path for about the same time whatever
  // its width or lane mask, so fewer index loads leave more of it to the
  // neighbour-row gathers.  Entry e of a chunk sits in lane e / 4, component
  // e % 4 (a compile-time constant below, since batches start at multiples
  // of 8).  With PREFETCH the next chunk's indices load during this chunk's
  // gathers (long rows); without it the registers stay fewer (light rows,
  // mostly a single chunk).
  template <bool PREFETCH>
  __device__ static void gather4(const int32_t *__restrict__ col, const float *__restrict__ val,
                                 const TU *__restrict__ U, int64_t ldu, int64_t beg, int64_t end, int64_t nnz,
                                 int G, int lig, int first, int stride, int c0, bool col_ok, float (&acc)[VEC]) {
    const int C = 4 * G;
    auto load4 = [&](int64_t q, i4u &c4, f4u &v4) { load_idx4(col, val, q + 4 * lig, nnz, c4, v4); };
    int64_t p = beg + int64_t(first) * C;
    if (p >= end) return;
    i4u c4, nc4 = {0, 0, 0, 0};
    f4u v4, nv4 = {0.f, 0.f, 0.f, 0.f};
    load4(p, c4, v4);
    for (; p < end; p += int64_t(stride) * C) {
      const int cnt = int(min<int64_t>(C, end - p));
      const int64_t pn = p + int64_t(stride) * C;
      if (PREFETCH && pn < end) load4(pn, nc4, nv4);
      for (int t = 0; t < cnt; t += 8) {
        int32_t j[8];
        float sv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int src = ((t + u) >> 2) & (G - 1);
          j[u] = __shfl(c4[u & 3], src, G);
          sv[u] = (t + u < cnt) ? __shfl(v4[u & 3], src, G) : 0.f;
        }
        if (col_ok) {
          RawRow<TU, VEC> x[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (t + u < cnt) x[u].load(U + int64_t(j[u]) * ldu + c0);
            else x[u].zero();
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] = fmaf(sv[u], x[u].get(v), acc[v]);
        }
      }
      if (PREFETCH) {
        c4 = nc4;
        v4 = nv4;
      } else if (pn < end) {
        load4(pn, c4, v4);
      }
    }
  }

  // The same sum as gather4 with every neighbour-row load unconditional (no
  // exec-mask branches): the entries of a partial batch of 8 re-read the
  // batch's first row and their terms are masked off bitwise (index entries
  // past the row's end are other rows' valid columns, or 0 past the arrays'
  // end, so every load stays in bounds).  Faster with 16 or more lanes per row
  // (k >= 61 at 4 columns per lane: 12-17% on bf16 k = 64 blocks), slower
  // with 8 (5-7% at k = 32).
  template <bool PREFETCH>
  __device__ static void gather_straight(const int32_t *__restrict__ col, const float *__restrict__ val,
                                         const TU *__restrict__ U, int64_t ldu, int64_t beg, int64_t end,
                                         int64_t nnz, int G, int lig, int first, int stride, int c0, bool col_ok,
                                         float (&acc)[VEC]) {
    const int C = 4 * G;
    auto load4 = [&](int64_t q, i4u &c4, f4u &v4) { load_idx4(col, val, q + 4 * lig, nnz, c4, v4); };
    int64_t p = beg + int64_t(first) * C;
    if (p >= end) return;
    i4u c4, nc4 = {0, 0, 0, 0};
    f4u v4, nv4 = {0.f, 0.f, 0.f, 0.f};
    load4(p, c4, v4);
    for (; p < end; p += int64_t(stride) * C) {
      const int cnt = int(min<int64_t>(C, end - p));
      const int64_t pn = p + int64_t(stride) * C;
      if (PREFETCH && pn < end) load4(pn, nc4, nv4);
      for (int t = 0; t < cnt; t += 8) {
        int32_t j[8];
        float sv[8];
        uint32_t keep[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int src = ((t + u) >> 2) & (G - 1);
          j[u] = __shfl(c4[u & 3], src, G);
          sv[u] = __shfl(v4[u & 3], src, G);
          keep[u] = (t + u < cnt) ? 0xffffffffu : 0u;
        }
        if (col_ok) {
          RawRow<TU, VEC> x[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int32_t jj = (t + u < cnt) ? j[u] : j[0];
            x[u].load(U + int64_t(jj) * ldu + c0);
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int v = 0; v < VEC; ++v)
              acc[v] = fmaf(__uint_as_float(__float_as_uint(sv[u]) & keep[u]),
                            __uint_as_float(__float_as_uint(x[u].get(v)) & keep[u]), acc[v]);
        }
      }
      if (PREFETCH) {
        c4 = nc4;
        v4 = nv4;
      } else if (pn < end) {
        load4(pn, c4, v4);
      }
    }
  }

  // O[row] = a (dg U[row] - acc) + b U[row] + g V[row] with dg = L_row,row;
  // returns <O[row], W[row]> over this lane's columns when DOT.
  __device__ static double epilogue(int64_t row, int c0, float dg, const TU *__restrict__ U, int64_t ldu,
                                    const TV *__restrict__ V, int64_t ldv, TO *__restrict__ O, int64_t ldo,
                                    Coef cf, const float *__restrict__ W, int64_t ldw, const float (&acc)[VEC]) {
    float u[VEC], o[VEC];
    VecIO<TU, VEC>::load(U + row * ldu + c0, u);
#pragma unroll
    for (int v = 0; v < VEC; ++v) o[v] = cf.a * (dg * u[v] - acc[v]) + cf.b * u[v];
    if (cf.g != 0.f) {
      float x[VEC];
      VecIO<TV, VEC>::load(V + row * ldv + c0, x);
#pragma unroll
      for (int v = 0; v < VEC; ++v) o[v] = fmaf(cf.g, x[v], o[v]);
    }
    VecNT<TO, VEC>::store(O + row * ldo + c0, o);
    double d = 0.0;
    if (DOT) {
      float w[VEC];
      VecIO<float, VEC>::load(W + row * ldw + c0, w);
      // the stored (rounded) value is what the next step consumes
#pragma unroll
      for (int v = 0; v < VEC; ++v) d += double(to_f32<TO>(from_f32<TO>(o[v]))) * double(w[v]);
    }
    return d;
  }
};

__device__ inline double block_sum_double(double v, double *lds) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < int(blockDim.x >> 6); ++w) t += lds[w];
  return t;
}

// Row ranges of the 8 XCDs: XCD x owns rows [r[x], r[x+1]).
struct XcdRows {
  int64_t r[kXcds + 1];
};

// Blocks are dealt to the XCDs round-robin (block b runs on XCD b % 8), so
// block b takes the (b / 8)-th run of 256/G rows inside XCD (b % 8)'s range:
// each die walks a contiguous stretch of rows (neighbour rows of nearby nodes
// share its L2) and the ranges carry equal work.
template <typename TU, typename TV, typename TO, int VEC, bool DOT, bool STRAIGHT>
__global__ __launch_bounds__(kBlock) void spmm_light(
    XcdRows xr, int64_t nnz, int k, int G, int lgG, const int64_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const float *__restrict__ val, const float *__restrict__ diag,
    const TU *__restrict__ U, int64_t ldu, const TV *__restrict__ V, int64_t ldv, TO *__restrict__ O,
    int64_t ldo, Coef cf, const float *__restrict__ W, int64_t ldw, double *__restrict__ partials) {
  using S = Step<TU, TV, TO, VEC, DOT>;
  const int x = blockIdx.x % kXcds;
  const int64_t row0 = xr.r[x] + int64_t(blockIdx.x / kXcds) * (kBlock >> lgG);
  const int64_t rend = xr.r[x + 1];
  if (!DOT && row0 >= rend) return;  // past this XCD's range (uniform over the block)
  const int lig = threadIdx.x & (G - 1);
  const int grp = threadIdx.x >> lgG;
  const int64_t row = row0 + grp;
  const int c0 = blockIdx.y * 64 * VEC + lig * VEC;
  const bool col_ok = c0 < k;
  double dsum = 0.0;
  if (row < rend) {
    const int64_t beg = rowptr[row], end = rowptr[row + 1];
    if (end - beg <= SPED_LIGHT_MAX) {
      float acc[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[v] = 0.f;
      if (STRAIGHT)
        S::template gather_straight<false>(col, val, U, ldu, beg, end, nnz, G, lig, 0, 1, c0, col_ok, acc);
      else S::template gather4<false>(col, val, U, ldu, beg, end, nnz, G, lig, 0, 1, c0, col_ok, acc);
      // diag == NULL: the normalised Laplacian, whose diagonal is 1 on rows
      // with entries and 0 on isolated rows
      const float dg = diag ? diag[row] : (end > beg ? 1.f : 0.f);
      if (col_ok) dsum = S::epilogue(row, c0, dg, U, ldu, V, ldv, O, ldo, cf, W, ldw, acc);
    }
  }
  if (DOT) {
    __shared__ double red[kBlock / 64];
    double t = block_sum_double(dsum, red);
    if (threadIdx.x == 0) partials[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = t;
  }
}

// Medium rows run in chunks of `chunk` consecutive logical blocks, chunk c on
// XCD c % 8 (blocks are dispatched to the XCDs round-robin): neighbouring
// medium rows, which on a community-ordered graph gather from the same rows,
// share one XCD's L2, while a degree-sorted row list stays spread over the
// XCDs.  The grid is a multiple of 8 * chunk, so the map is a bijection.
__device__ inline int64_t medium_logical_block(int64_t chunk) {
  const int64_t b = blockIdx.x;
  const int64_t x = b % kXcds, i = b / kXcds;
  return ((i / chunk) * kXcds + x) * chunk + (i % chunk);
}

template <typename TU, typename TV, typename TO, int VEC, bool DOT, bool STRAIGHT>
__global__ __launch_bounds__(kBlock) void spmm_medium(
    int64_t n_rows, int64_t chunk, const int32_t *__restrict__ rows, int64_t nnz, int k, int G, int lgG,
    const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    const float *__restrict__ val, const float *__restrict__ diag, const TU *__restrict__ U,
    int64_t ldu, const TV *__restrict__ V, int64_t ldv, TO *__restrict__ O, int64_t ldo, Coef cf,
    const float *__restrict__ W, int64_t ldw, double *__restrict__ partials) {
  using S = Step<TU, TV, TO, VEC, DOT>;
  const int lane = threadIdx.x & 63;
  const int lig = lane & (G - 1);
  const int sub = lane >> lgG;
  const int nsub = 64 >> lgG;
  const int64_t lb = medium_logical_block(chunk);
  const int64_t ri = lb * (kBlock / 64) + (threadIdx.x >> 6);
  const int c0 = blockIdx.y * 64 * VEC + lig * VEC;
  const bool col_ok = c0 < k;
  double dsum = 0.0;
  if (ri < n_rows) {
    const int64_t row = rows[ri];
    const int64_t beg = rowptr[row], end = rowptr[row + 1];
    float acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = 0.f;
    if (STRAIGHT)
      S::template gather_straight<true>(col, val, U, ldu, beg, end, nnz, G, lig, sub, nsub, c0, col_ok, acc);
    else S::template gather4<true>(col, val, U, ldu, beg, end, nnz, G, lig, sub, nsub, c0, col_ok, acc);
    for (int off = G; off < 64; off <<= 1)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[v] += __shfl_xor(acc[v], off, 64);
    if (sub == 0 && col_ok)
      dsum = S::epilogue(row, c0, diag ? diag[row] : 1.f, U, ldu, V, ldv, O, ldo, cf, W, ldw, acc);
  }
  if (DOT) {
    __shared__ double red[kBlock / 64];
    double t = block_sum_double(dsum, red);
    if (threadIdx.x == 0) partials[int64_t(blockIdx.y) * gridDim.x + lb] = t;  // logical order
  }
}

// Pieces of the heavy rows: hp[h] = sum over heavy rows h' < h of
// ceil(d_h' / kPiece), h = 0 .. n_heavy (hp[n_heavy] = the piece count).  One
// block: each thread counts a contiguous run of rows, then an exclusive scan
// over the threads' counts.
constexpr int64_t kPiece = SPED_MEDIUM_MAX;

__global__ __launch_bounds__(1024) void heavy_plan_kernel(int64_t n_heavy, const int32_t *__restrict__ rows,
                                                          const int64_t *__restrict__ rowptr,
                                                          int64_t *__restrict__ hp) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n_heavy + 1023) / 1024;
  const int64_t lo = min(n_heavy, per * t), hi = min(n_heavy, lo + per);
  int64_t cnt = 0;
  for (int64_t h = lo; h < hi; ++h) {
    const int64_t r = rows[h];
    cnt += (rowptr[r + 1] - rowptr[r] + kPiece - 1) / kPiece;
  }
  part[t] = cnt;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - cnt;
  for (int64_t h = lo; h < hi; ++h) {
    hp[h] = run;
    const int64_t r = rows[h];
    run += (rowptr[r + 1] - rowptr[r] + kPiece - 1) / kPiece;
  }
  if (t == 1023) hp[n_heavy] = part[1023];
}

// One block per piece (blocks loop over the pieces): the piece's entries are
// shared by the block's lane groups as in a medium row, the groups' sums meet
// in LDS in a fixed order and the block writes the piece's partial row (float32,
// the block's columns) to part[piece * k + c].
template <typename TU, int VEC, bool STRAIGHT>
__global__ __launch_bounds__(kBlock) void spmm_heavy_pieces(
    int64_t n_heavy, const int32_t *__restrict__ rows, const int64_t *__restrict__ hp, int64_t nnz, int k, int G,
    int lgG, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col, const float *__restrict__ val,
    const TU *__restrict__ U, int64_t ldu, float *__restrict__ part) {
  using S = Step<TU, float, float, VEC, false>;
  __shared__ float red[kBlock * VEC];
  const int lig = threadIdx.x & (G - 1);
  const int sub = threadIdx.x >> lgG;
  const int nsub = kBlock >> lgG;
  const int c0 = blockIdx.y * 64 * VEC + lig * VEC;
  const bool col_ok = c0 < k;
  const int64_t total = hp[n_heavy];
  for (int64_t pc = blockIdx.x; pc < total; pc += gridDim.x) {
    // the heavy row holding piece pc: largest h with hp[h] <= pc
    int64_t lo = 0, hi = n_heavy - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (hp[mid] <= pc) lo = mid;
      else hi = mid - 1;
    }
    const int64_t row = rows[lo];
    const int64_t beg = rowptr[row] + (pc - hp[lo]) * kPiece;
    const int64_t end = min(rowptr[row + 1], beg + kPiece);
    float acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = 0.f;
    if (STRAIGHT)
      S::template gather_straight<true>(col, val, U, ldu, beg, end, nnz, G, lig, sub, nsub, c0, col_ok, acc);
    else S::template gather4<true>(col, val, U, ldu, beg, end, nnz, G, lig, sub, nsub, c0, col_ok, acc);
#pragma unroll
    for (int v = 0; v < VEC; ++v) red[threadIdx.x * VEC + v] = acc[v];
    __syncthreads();
    if (sub == 0 && col_ok) {
      for (int sidx = 1; sidx < nsub; ++sidx)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] += red[(sidx * G + lig) * VEC + v];
      VecIO<float, VEC>::store(part + pc * k + c0, acc);
    }
    __syncthreads();  // red is reused by the next piece
  }
}

// One lane group per heavy row: the row's piece partials added in piece
// order, then the epilogue.
template <typename TU, typename TV, typename TO, int VEC, bool DOT>
__global__ __launch_bounds__(kBlock) void spmm_heavy_finish(
    int64_t n_heavy, const int32_t *__restrict__ rows, const int64_t *__restrict__ hp, int k, int G, int lgG,
    const float *__restrict__ diag, const TU *__restrict__ U, int64_t ldu, const TV *__restrict__ V, int64_t ldv,
    TO *__restrict__ O, int64_t ldo, Coef cf, const float *__restrict__ W, int64_t ldw,
    const float *__restrict__ part, double *__restrict__ partials) {
  using S = Step<TU, TV, TO, VEC, DOT>;
  const int lig = threadIdx.x & (G - 1);
  const int64_t h = int64_t(blockIdx.x) * (kBlock >> lgG) + (threadIdx.x >> lgG);
  const int c0 = blockIdx.y * 64 * VEC + lig * VEC;
  double dsum = 0.0;
  if (h < n_heavy && c0 < k) {
    float acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = 0.f;
    for (int64_t pc = hp[h]; pc < hp[h + 1]; ++pc) {
      float x[VEC];
      VecIO<float, VEC>::load(part + pc * k + c0, x);
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[v] += x[v];
    }
    const int64_t row = rows[h];
    dsum = S::epilogue(row, c0, diag ? diag[row] : 1.f, U, ldu, V, ldv, O, ldo, cf, W, ldw, acc);
  }
  if (DOT) {
    __shared__ double red[kBlock / 64];
    double t = block_sum_double(dsum, red);
    if (threadIdx.x == 0) partials[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kBlock) void reduce_partials_kernel(const double *__restrict__ p,
                                                                  int64_t count, double *out) {
  __shared__ double red[kBlock];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += kBlock) s += p[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// The piece prefix hp[0 .. n_heavy], rounded up to 256 bytes.
size_t heavy_plan_bytes(const sped_csr *L) { return (size_t(L->n_heavy + 1) * sizeof(int64_t) + 255) / 256 * 256; }

struct Geometry {
  int vec, G, lgG, ytiles;
  XcdRows xr;
  int64_t light_blocks, medium_blocks, heavy_blocks;
  int64_t medium_chunk;  // consecutive medium blocks per XCD turn
};

bool valid_xcd_rows(const sped_csr *L) {
  if (L->xcd_rows[0] != 0 || L->xcd_rows[kXcds] != L->n) return false;
  for (int x = 0; x < kXcds; ++x)
    if (L->xcd_rows[x + 1] < L->xcd_rows[x]) return false;
  return true;
}

// Medium blocks per XCD turn (0: one contiguous range per XCD).  On the
// 4e6-node power-law graph numbered by label propagation the 64-column bf16
// step takes 809 us with 1 (plain round-robin), 795 with 4, 774 with 16 and
// 768 with 64; on the generator's degree-sorted ids, 1139, 1133, 1139 and
// 1167 us, and 1685 with one range per XCD (the heaviest rows all on XCD 0).
constexpr int64_t kMediumChunk = 16;

Geometry geometry(const sped_csr *L, int64_t k, int vec) {
  Geometry g;
  g.vec = vec;
  int lanes = int((k + vec - 1) / vec);
  g.ytiles = (lanes + 63) / 64;
  g.G = lanes >= 64 ? 64 : next_pow2(lanes);
  g.lgG = ilog2(g.G);
  const int64_t rpb = kBlock >> g.lgG;
  if (L->n > 0 && valid_xcd_rows(L)) {
    for (int x = 0; x <= kXcds; ++x) g.xr.r[x] = L->xcd_rows[x];
  } else {  // even split in whole blocks
    const int64_t per = ((L->n + rpb - 1) / rpb + kXcds - 1) / kXcds * rpb;
    for (int x = 0; x <= kXcds; ++x) g.xr.r[x] = std::min<int64_t>(L->n, per * x);
  }
  int64_t most = 0;
  for (int x = 0; x < kXcds; ++x) most = std::max(most, (g.xr.r[x + 1] - g.xr.r[x] + rpb - 1) / rpb);
  g.light_blocks = most * kXcds;
  const int64_t mb = (L->n_medium + 3) / 4;
  g.medium_chunk = std::max<int64_t>(1, kMediumChunk > 0 ? kMediumChunk : (mb + kXcds - 1) / kXcds);
  g.medium_blocks = mb > 0 ? (mb + kXcds * g.medium_chunk - 1) / (kXcds * g.medium_chunk) * (kXcds * g.medium_chunk) : 0;
  g.heavy_blocks = (L->n_heavy + rpb - 1) / rpb;  // finishing blocks, one lane group per heavy row
  return g;
}

int64_t partial_count(const Geometry &g) {
  return (g.light_blocks + g.medium_blocks + g.heavy_blocks) * g.ytiles;
}

// Upper bound on the pieces of the heavy rows: ceil(d / kPiece) <= d / kPiece + 1
// and the heavy rows hold at most nnz entries, so the total is at most
// ceil(nnz / kPiece) + n_heavy.
int64_t max_pieces(const sped_csr *L) {
  return L->n_heavy > 0 ? (L->nnz + kPiece - 1) / kPiece + L->n_heavy : 0;
}

// Blocks of the piece kernel: enough to fill the chip several times over,
// each looping over pieces.
constexpr int64_t kPieceBlocks = 2048;

template <typename TU, typename TV, typename TO, int VEC, bool DOT>
sped_status launch_typed(const sped_csr *L, int64_t k, const StepArgs &a, const Geometry &g,
                         hipStream_t s) {
  Coef cf{a.a, a.b, a.g};
  // the normalised Laplacian's diagonal follows from the row pointers
  const float *dgp = L->kind == SPED_LAP_SYM_NORMALIZED ? nullptr : L->diag;
  const TU *U = static_cast<const TU *>(a.U);
  const TV *V = static_cast<const TV *>(a.V);
  TO *O = static_cast<TO *>(a.O);
  double *part = a.dot_partials;
  // unconditional gathers pay off with 16 or more lanes per row
  const bool straight = VEC == 4 && g.G >= 16;
  if (g.light_blocks > 0) {
    const dim3 grid = dim3(unsigned(g.light_blocks), unsigned(g.ytiles));
    if constexpr (VEC == 4) {
      if (straight)
        hipLaunchKernelGGL((spmm_light<TU, TV, TO, VEC, DOT, true>), grid, dim3(kBlock), 0, s, g.xr, L->nnz, int(k),
                           g.G, g.lgG, L->rowptr, L->col, L->val, dgp, U, a.ldu, V, a.ldv, O, a.ldo,
                           cf, a.dotw, a.lddw, part);
    }
    if (!straight)
      hipLaunchKernelGGL((spmm_light<TU, TV, TO, VEC, DOT, false>), grid, dim3(kBlock), 0, s, g.xr, L->nnz, int(k),
                         g.G, g.lgG, L->rowptr, L->col, L->val, dgp, U, a.ldu, V, a.ldv, O, a.ldo,
                         cf, a.dotw, a.lddw, part);
    SPED_CHECK_HIP(hipGetLastError());
    if (DOT) part += g.light_blocks * g.ytiles;
  }
  if (g.medium_blocks > 0) {
    const dim3 grid = dim3(unsigned(g.medium_blocks), unsigned(g.ytiles));
#define SPED_MEDIUM(ST)                                                                                    \
  hipLaunchKernelGGL((spmm_medium<TU, TV, TO, VEC, DOT, ST>), grid, dim3(kBlock), 0, s, L->n_medium,      \
                     g.medium_chunk, L->bins, L->nnz, int(k), g.G, g.lgG, L->rowptr, L->col, L->val, dgp, U, a.ldu,     \
                     V, a.ldv, O, a.ldo, cf, a.dotw, a.lddw, part)
    if constexpr (VEC == 4) {
      if (straight) SPED_MEDIUM(true);
    }
    if (!straight) SPED_MEDIUM(false);
#undef SPED_MEDIUM
    SPED_CHECK_HIP(hipGetLastError());
    if (DOT) part += g.medium_blocks * g.ytiles;
  }
  if (L->n_heavy > 0) {
    if (!a.heavy_ws) return fail(SPED_E_WORKSPACE, "heavy rows need the step workspace");
    const int32_t *hrows = L->bins + L->n_medium;
    int64_t *hp = static_cast<int64_t *>(a.heavy_ws);
    float *hpart = reinterpret_cast<float *>(static_cast<char *>(a.heavy_ws) + heavy_plan_bytes(L));
    hipLaunchKernelGGL(heavy_plan_kernel, dim3(1), dim3(1024), 0, s, L->n_heavy, hrows, L->rowptr, hp);
    SPED_CHECK_HIP(hipGetLastError());
    const dim3 pgrid = dim3(unsigned(std::min<int64_t>(max_pieces(L), kPieceBlocks)), unsigned(g.ytiles));
#define SPED_PIECES(ST)                                                                                     \
  hipLaunchKernelGGL((spmm_heavy_pieces<TU, VEC, ST>), pgrid, dim3(kBlock), 0, s, L->n_heavy, hrows, hp,    \
                     L->nnz, int(k), g.G, g.lgG, L->rowptr, L->col, L->val, U, a.ldu, hpart)
    if constexpr (VEC == 4) {
      if (straight) SPED_PIECES(true);
    }
    if (!straight) SPED_PIECES(false);
#undef SPED_PIECES
    SPED_CHECK_HIP(hipGetLastError());
    const dim3 grid = dim3(unsigned(g.heavy_blocks), unsigned(g.ytiles));
    hipLaunchKernelGGL((spmm_heavy_finish<TU, TV, TO, VEC, DOT>), grid, dim3(kBlock), 0, s, L->n_heavy, hrows, hp,
                       int(k), g.G, g.lgG, dgp, U, a.ldu, V, a.ldv, O, a.ldo, cf, a.dotw, a.lddw, hpart, part);
    SPED_CHECK_HIP(hipGetLastError());
  }
  return SPED_OK;
}

template <int VEC, bool DOT>
sped_status dispatch_types(const sped_csr *L, int64_t k, const StepArgs &a, const Geometry &g,
                           hipStream_t s) {
  const bool u32 = a.tu == SPED_F32, v32 = a.tv == SPED_F32, o32 = a.to == SPED_F32;
#define SPED_CASE(TU_, TV_, TO_)                                                      \
  if (u32 == std::is_same<TU_, float>::value && v32 == std::is_same<TV_, float>::value && \
      o32 == std::is_same<TO_, float>::value)                                         \
    return launch_typed<TU_, TV_, TO_, VEC, DOT>(L, k, a, g, s);
  SPED_CASE(float, float, float)
  SPED_CASE(float, bf16_t, float)
  SPED_CASE(float, float, bf16_t)
  SPED_CASE(float, bf16_t, bf16_t)
  SPED_CASE(bf16_t, bf16_t, float)
  SPED_CASE(bf16_t, bf16_t, bf16_t)
  SPED_CASE(bf16_t, float, float)
  SPED_CASE(bf16_t, float, bf16_t)
#undef SPED_CASE
  return fail(SPED_E_UNSUPPORTED, "spmm dtype combination");
}

// 8 columns per lane for a bf16 gathered block (one 16-byte load per lane and
// row): half the lanes per row, so a wavefront keeps twice the rows in flight.
sped_status dispatch_bf16_vec8(const sped_csr *L, int64_t k, const StepArgs &a, const Geometry &g,
                               hipStream_t s) {
  const bool v32 = a.tv == SPED_F32, o32 = a.to == SPED_F32;
  if (!v32 && !o32) return launch_typed<bf16_t, bf16_t, bf16_t, 8, false>(L, k, a, g, s);
  if (!v32 && o32) return launch_typed<bf16_t, bf16_t, float, 8, false>(L, k, a, g, s);
  if (v32 && o32) return launch_typed<bf16_t, float, float, 8, false>(L, k, a, g, s);
  return launch_typed<bf16_t, float, bf16_t, 8, false>(L, k, a, g, s);
}

bool vec8_ok(int64_t k, std::initializer_list<int64_t> lds, std::initializer_list<const void *> ptrs) {
  if (k % 8) return false;
  for (int64_t ld : lds)
    if (ld % 8) return false;
  for (const void *p : ptrs)
    if (p && (reinterpret_cast<uintptr_t>(p) & 15)) return false;
  return true;
}

}  // namespace

size_t spmm_step_ws_bytes(const sped_csr *L, int64_t k) {
  if (L->n_heavy <= 0) return 0;
  return heavy_plan_bytes(L) + size_t(max_pieces(L)) * size_t(k) * sizeof(float);
}

int64_t spmm_partials(const sped_csr *L, int64_t k) {
  return partial_count(geometry(L, k, 1));  // upper bound: vec = 1 gives the most blocks
}

sped_status launch_spmm_step(const sped_csr *L, int64_t k, const StepArgs &a, hipStream_t s,
                             int64_t *partials_written) {
  if (a.tu == SPED_F64 || a.tv == SPED_F64 || a.to == SPED_F64)
    return fail(SPED_E_UNSUPPORTED, "float64 blocks are not supported by the sparse step");
  const void *V = a.g != 0.f ? a.V : a.U;
  int64_t ldv = a.g != 0.f ? a.ldv : a.ldu;
  int vec = pick_vec(k, {a.ldu, ldv, a.ldo, a.dotw ? a.lddw : k}, {a.U, V, a.O, a.dotw},
                     {int(dtype_size(a.tu)), int(dtype_size(a.g != 0.f ? a.tv : a.tu)),
                      int(dtype_size(a.to)), 4});
  StepArgs b = a;
  if (a.g == 0.f) {
    b.V = a.U;
    b.ldv = a.ldu;
    b.tv = a.tu;
  }
  const bool dot = a.dotw != nullptr;
  if (vec == 4 && !dot && a.tu == SPED_BF16 && vec8_ok(k, {a.ldu, b.ldv, a.ldo}, {a.U, b.V, a.O})) {
    if (partials_written) *partials_written = 0;
    return dispatch_bf16_vec8(L, k, b, geometry(L, k, 8), s);
  }
  Geometry g = geometry(L, k, vec);
  if (partials_written) *partials_written = dot ? partial_count(g) : 0;
  if (vec == 4) return dot ? dispatch_types<4, true>(L, k, b, g, s) : dispatch_types<4, false>(L, k, b, g, s);
  if (vec == 2) return dot ? dispatch_types<2, true>(L, k, b, g, s) : dispatch_types<2, false>(L, k, b, g, s);
  return dot ? dispatch_types<1, true>(L, k, b, g, s) : dispatch_types<1, false>(L, k, b, g, s);
}

sped_status launch_reduce_partials(const double *partials, int64_t count, double *out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kBlock), 0, s, partials, count, out);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

}  // namespace sped
