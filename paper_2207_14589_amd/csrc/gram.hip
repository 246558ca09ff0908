// Tall-skinny dense kernels of the block solver:
//   gram   G = A^T B in float64 on the float64 matrix cores
//          (v_mfma_f64_16x16x4f64), one 16x16 output tile per MFMA chain;
//   tsmm   O = X T for a small k_in x k_out matrix T (float64 in memory, float
//          in LDS), one lane group per row like the sparse step;
//   resid  R^T R for R = Z - Q diag(theta) formed on the fly (same Gram
//          kernels), column norms and an upper bound on ||R||_2.
// Split over rows, every block writes its own partial; a second pass adds the
// partials in a fixed order, so results are bitwise reproducible.
#include "common.h"

namespace sped {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxK = 128;        // ka, kb <= kMaxK
constexpr int kGramBlocks = 512;

typedef double double4_t __attribute__((ext_vector_type(4)));

template <typename T>
__device__ inline double load_as_double(const T *p);
template <>
__device__ inline double load_as_double<float>(const float *p) { return double(*p); }
template <>
__device__ inline double load_as_double<bf16_t>(const bf16_t *p) { return double(bf16_to_f32(*p)); }

// Operand loaders of the Gram kernels: element (row, c) of the left and right
// factors, converted to float64.
template <typename T1, typename T2>
struct PlainLoad {
  const T1 *A;
  int64_t lda;
  const T2 *B;
  int64_t ldb;
  __device__ double a(int64_t r, int c) const { return load_as_double(A + r * lda + c); }
  __device__ double b(int64_t r, int c) const { return load_as_double(B + r * ldb + c); }
};

// Residual block R = Z - Q diag(theta) formed on the fly (both factors are R).
template <typename TQ>
struct ResidLoad {
  const float *Z;
  const TQ *Q;
  int64_t ld;
  const double *theta;
  __device__ double a(int64_t r, int c) const {
    return double(Z[r * ld + c]) - theta[c] * load_as_double(Q + r * ld + c);
  }
  __device__ double b(int64_t r, int c) const { return a(r, c); }
};

// Each wavefront streams its rows straight from global memory (16 rows per
// round: lane (li, lk) reads element [row + 4u + lk][16 tile + li], u = 0..3)
// into float64 MFMA operands; no LDS and no barriers.  With few output tiles
// (ROWSPLIT) every wavefront forms all tiles over its own quarter of the
// block's rows and writes its own partial; otherwise the tiles are dealt
// round-robin to the 4 wavefronts, which all read the block's rows (their
// shared lines come from L1) and write disjoint tiles of one partial.  With
// SYM (A == B) only tiles p <= q are formed and mirrored on output.
template <typename LD, int MAXT, bool SYM, bool ROWSPLIT>
__global__ __launch_bounds__(kBlock) void gram_kernel(int64_t n, int ka, int kb, LD ld,
                                                      int64_t rows_per_block, double *__restrict__ partials) {
  constexpr int KU = MAXT <= 4 ? 4 : 1;
  const int TA = (ka + 15) / 16, TB = (kb + 15) / 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;

  int tp[MAXT], tq[MAXT];
  int nt = 0;
  {
    int idx = 0;
    for (int p = 0; p < TA; ++p)
      for (int q = SYM ? p : 0; q < TB; ++q) {
        if ((ROWSPLIT || idx % 4 == wave) && nt < MAXT) {
          tp[nt] = p;
          tq[nt] = q;
          ++nt;
        }
        ++idx;
      }
  }
  double4_t acc[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) acc[t] = double4_t{0.0, 0.0, 0.0, 0.0};

  const int64_t r_begin = int64_t(blockIdx.x) * rows_per_block;
  const int64_t r_end = min(n, r_begin + rows_per_block);
  const int64_t first = r_begin + (ROWSPLIT ? 4 * KU * wave : 0);
  const int64_t stride = ROWSPLIT ? 16 * KU : 4 * KU;
  for (int64_t r = first; r < r_end; r += stride) {
    double a[KU][MAXT], b[KU][MAXT];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int64_t row = r + 4 * u + lk;
      const bool rok = row < r_end;
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        a[u][t] = b[u][t] = 0.0;
        if (t < nt && rok) {
          const int ca = tp[t] * 16 + li, cb = tq[t] * 16 + li;
          if (ca < ka) a[u][t] = ld.a(row, ca);
          if (cb < kb) b[u][t] = ld.b(row, cb);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int t = 0; t < MAXT; ++t)
        if (t < nt) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][t], b[u][t], acc[t], 0, 0, 0);
  }
  // Which (row, column) of the 16x16 tile each of this lane's 4 accumulator
  // slots holds is read off the matrix core itself: with A[i][0] = i,
  // B[0][j] = 1 (other k = 0) the product is D[i][j] = i, and with A[i][0] = 1,
  // B[0][j] = j it is D[i][j] = j.  Only the operand layout (lane l holds
  // A[l % 16][l / 16] and B[l / 16][l % 16]) is assumed.
  const double4_t zero4 = double4_t{0.0, 0.0, 0.0, 0.0};
  const double4_t rowid = __builtin_amdgcn_mfma_f64_16x16x4f64(lk == 0 ? double(li) : 0.0, lk == 0 ? 1.0 : 0.0,
                                                               zero4, 0, 0, 0);
  const double4_t colid = __builtin_amdgcn_mfma_f64_16x16x4f64(lk == 0 ? 1.0 : 0.0, lk == 0 ? double(li) : 0.0,
                                                               zero4, 0, 0, 0);
  const int64_t slot = ROWSPLIT ? int64_t(blockIdx.x) * 4 + wave : int64_t(blockIdx.x);
  double *out = partials + slot * ka * kb;
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    if (t < nt) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int i = tp[t] * 16 + int(rowid[r]);
        int j = tq[t] * 16 + int(colid[r]);
        if (i < ka && j < kb) out[i * kb + j] = acc[t][r];
        if (SYM && tp[t] != tq[t] && j < ka && i < kb) out[j * kb + i] = acc[t][r];
      }
    }
  }
}

// Narrow Gram (both widths <= 32): 16 wavefronts per block, each streams its
// own interleaved 16-row chunks of the block's rows and forms all TA x TB tiles
// (operand fragments loaded once per row group and reused across tiles).  The
// wavefronts then add their tiles into one LDS copy in wavefront order (fixed
// order: deterministic) and the block writes one partial.
constexpr int kNarrowBlock = 1024;
template <typename LD, int TA, int TB, bool SYM>
__global__ __launch_bounds__(kNarrowBlock) void gram_narrow_kernel(int64_t n, int ka, int kb, LD ld,
                                                                   int64_t rows_per_block,
                                                                   double *__restrict__ partials) {
  constexpr int KU = 4;
  constexpr int NW = kNarrowBlock / 64;
  __shared__ double red[TA * 16 * TB * 16];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  double4_t acc[TA][TB];
#pragma unroll
  for (int p = 0; p < TA; ++p)
#pragma unroll
    for (int q = 0; q < TB; ++q) acc[p][q] = double4_t{0.0, 0.0, 0.0, 0.0};
  const int64_t r_begin = int64_t(blockIdx.x) * rows_per_block;
  const int64_t r_end = min(n, r_begin + rows_per_block);
  for (int64_t r = r_begin + 4 * KU * wave; r < r_end; r += 4 * KU * NW) {
    double fa[KU][TA], fb[KU][TB];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int64_t row = r + 4 * u + lk;
      const bool rok = row < r_end;
#pragma unroll
      for (int p = 0; p < TA; ++p) {
        const int c = p * 16 + li;
        fa[u][p] = (rok && c < ka) ? ld.a(row, c) : 0.0;
      }
      if (!SYM) {
#pragma unroll
        for (int q = 0; q < TB; ++q) {
          const int c = q * 16 + li;
          fb[u][q] = (rok && c < kb) ? ld.b(row, c) : 0.0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int p = 0; p < TA; ++p)
#pragma unroll
        for (int q = 0; q < TB; ++q)
          if (!SYM || p <= q)
            acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[u][p], SYM ? fa[u][q] : fb[u][q], acc[p][q], 0, 0, 0);
  }
  const double4_t zero4 = double4_t{0.0, 0.0, 0.0, 0.0};
  const double4_t rowid = __builtin_amdgcn_mfma_f64_16x16x4f64(lk == 0 ? double(li) : 0.0, lk == 0 ? 1.0 : 0.0,
                                                               zero4, 0, 0, 0);
  const double4_t colid = __builtin_amdgcn_mfma_f64_16x16x4f64(lk == 0 ? 1.0 : 0.0, lk == 0 ? double(li) : 0.0,
                                                               zero4, 0, 0, 0);
  constexpr int W = TB * 16;
  for (int w = 0; w < NW; ++w) {
    if (wave == w) {
#pragma unroll
      for (int p = 0; p < TA; ++p)
#pragma unroll
        for (int q = 0; q < TB; ++q)
          if (!SYM || p <= q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = p * 16 + int(rowid[r]), j = q * 16 + int(colid[r]);
              red[i * W + j] = (w == 0 ? 0.0 : red[i * W + j]) + acc[p][q][r];
            }
    }
    __syncthreads();
  }
  double *out = partials + int64_t(blockIdx.x) * ka * kb;
  for (int idx = threadIdx.x; idx < ka * kb; idx += kNarrowBlock) {
    const int i = idx / kb, j = idx - i * kb;
    const int pi = i / 16, qj = j / 16;
    out[idx] = (SYM && pi > qj) ? red[j * W + i] : red[i * W + j];
  }
}

// One wavefront per output entry: lane l adds partials l, l + 64, ... and the
// lanes meet in a fixed xor tree (deterministic).
__global__ __launch_bounds__(kBlock) void sum_partials_kernel(const double *__restrict__ partials, int nparts,
                                                               int64_t count, double *__restrict__ out,
                                                               int take_sqrt) {
  const int64_t i = int64_t(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= count) return;  // uniform per wavefront
  double s = 0.0;
  for (int p = lane; p < nparts; p += 64) s += partials[int64_t(p) * count + i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) out[i] = take_sqrt ? sqrt(s) : s;
}

sped_status launch_sum_partials(const double *partials, int nparts, int64_t count, double *out, bool take_sqrt,
                                hipStream_t s) {
  const int64_t blocks = (count + kBlock / 64 - 1) / (kBlock / 64);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(unsigned(blocks)), dim3(kBlock), 0, s, partials, nparts, count, out,
                     int(take_sqrt));
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

// O[r, :] = X[r, :] T, T kin x kout float64 -> float in LDS.
template <typename TX, typename TO, int VEC>
__global__ __launch_bounds__(kBlock) void tsmm_kernel(int64_t n, int kin, int kout, int G, int lgG,
                                                      const TX *__restrict__ X, int64_t ldx,
                                                      const double *__restrict__ T, TO *__restrict__ O,
                                                      int64_t ldo) {
  extern __shared__ float sT[];
  const int kop = (kout + 3) & ~3;
  for (int i = threadIdx.x; i < kin * kop; i += kBlock) {
    int r = i / kop, c = i - r * kop;
    sT[i] = c < kout ? float(T[r * kout + c]) : 0.f;
  }
  __syncthreads();
  const int lig = threadIdx.x & (G - 1);
  const int64_t row = int64_t(blockIdx.x) * (kBlock >> lgG) + (threadIdx.x >> lgG);
  const int c0 = blockIdx.y * 64 * VEC + lig * VEC;
  if (row >= n || c0 >= kout) return;
  float o[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) o[v] = 0.f;
  const TX *xr = X + row * ldx;
  for (int j = 0; j < kin; ++j) {
    float x = to_f32<TX>(xr[j]);
#pragma unroll
    for (int v = 0; v < VEC; ++v) o[v] = fmaf(x, sT[j * kop + c0 + v], o[v]);
  }
  VecIO<TO, VEC>::store(O + row * ldo + c0, o);
}


struct GramPlan {
  int nblocks, nparts, maxt;
  bool rowsplit, narrow;
  int64_t rows_per_block;
};

GramPlan gram_plan(int64_t n, int ka, int kb, bool sym) {
  const int TA = (ka + 15) / 16, TB = (kb + 15) / 16;
  const int tiles = sym ? TA * (TA + 1) / 2 : TA * TB;
  GramPlan p;
  p.rowsplit = tiles <= 4;
  const int per_wave = p.rowsplit ? tiles : (tiles + 3) / 4;
  p.maxt = per_wave <= 1 ? 1 : per_wave <= 2 ? 2 : per_wave <= 4 ? 4 : per_wave <= 8 ? 8 : 16;
  int64_t blocks = (n + 255) / 256;
  p.nblocks = int(blocks < kGramBlocks ? (blocks > 0 ? blocks : 1) : kGramBlocks);
  int64_t rpb = (n + p.nblocks - 1) / p.nblocks;
  p.rows_per_block = (rpb + 63) / 64 * 64;
  p.nparts = p.rowsplit ? 4 * p.nblocks : p.nblocks;
  p.narrow = TA <= 2 && TB <= 2;
  if (p.narrow) {
    int64_t nb = (n + 1023) / 1024;
    p.nblocks = int(nb < kGramBlocks ? (nb > 0 ? nb : 1) : kGramBlocks);
    int64_t r = (n + p.nblocks - 1) / p.nblocks;
    p.rows_per_block = (r + 255) / 256 * 256;
    p.nparts = p.nblocks;
  }
  return p;
}

template <typename LD, int MAXT, bool SYM, bool RS>
sped_status launch_gram_t(int64_t n, int ka, int kb, const LD &ld, double *partials, const GramPlan &p,
                          hipStream_t s) {
  hipLaunchKernelGGL((gram_kernel<LD, MAXT, SYM, RS>), dim3(p.nblocks), dim3(kBlock), 0, s, n, ka, kb, ld,
                     p.rows_per_block, partials);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

template <typename LD, int TA, int TB, bool SYM>
sped_status launch_gram_narrow_t(int64_t n, int ka, int kb, const LD &ld, double *partials, const GramPlan &p,
                                 hipStream_t s) {
  hipLaunchKernelGGL((gram_narrow_kernel<LD, TA, TB, SYM>), dim3(p.nblocks), dim3(kNarrowBlock), 0, s, n, ka, kb,
                     ld, p.rows_per_block, partials);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

template <typename LD, bool SYM>
sped_status launch_gram_maxt(int64_t n, int ka, int kb, const LD &ld, double *partials, const GramPlan &p,
                             hipStream_t s) {
  if (p.narrow) {
    const int TA = (ka + 15) / 16, TB = (kb + 15) / 16;
    if (TA == 1 && TB == 1) return launch_gram_narrow_t<LD, 1, 1, SYM>(n, ka, kb, ld, partials, p, s);
    if (TA == 1 && TB == 2) return launch_gram_narrow_t<LD, 1, 2, SYM>(n, ka, kb, ld, partials, p, s);
    if (TA == 2 && TB == 1) return launch_gram_narrow_t<LD, 2, 1, SYM>(n, ka, kb, ld, partials, p, s);
    return launch_gram_narrow_t<LD, 2, 2, SYM>(n, ka, kb, ld, partials, p, s);
  }
  if (p.rowsplit) {
    if (p.maxt <= 1) return launch_gram_t<LD, 1, SYM, true>(n, ka, kb, ld, partials, p, s);
    if (p.maxt <= 2) return launch_gram_t<LD, 2, SYM, true>(n, ka, kb, ld, partials, p, s);
    return launch_gram_t<LD, 4, SYM, true>(n, ka, kb, ld, partials, p, s);
  }
  if (p.maxt <= 2) return launch_gram_t<LD, 2, SYM, false>(n, ka, kb, ld, partials, p, s);
  if (p.maxt <= 4) return launch_gram_t<LD, 4, SYM, false>(n, ka, kb, ld, partials, p, s);
  if (p.maxt <= 8) return launch_gram_t<LD, 8, SYM, false>(n, ka, kb, ld, partials, p, s);
  return launch_gram_t<LD, 16, SYM, false>(n, ka, kb, ld, partials, p, s);
}

template <typename T1, typename T2, bool SYM>
sped_status launch_gram_plain(int64_t n, int ka, int kb, const void *A, int64_t lda, const void *B, int64_t ldb,
                              double *partials, const GramPlan &p, hipStream_t s) {
  PlainLoad<T1, T2> ld{static_cast<const T1 *>(A), lda, static_cast<const T2 *>(B), ldb};
  return launch_gram_maxt<PlainLoad<T1, T2>, SYM>(n, ka, kb, ld, partials, p, s);
}

// From G = R^T R (k x k): resid[i] = sqrt(G_ii) for i < k, and
// *norm2 = sqrt(min(max_{i<kn} sum_{j<kn} |G_ij|, sum_{i<kn} G_ii)), an upper
// bound on the spectral norm of the first kn columns of R (the largest
// eigenvalue of their Gram block is at most both its infinity norm and its
// trace).
__global__ void resid_norms_kernel(int k, int kn, const double *__restrict__ G, double *__restrict__ resid,
                                   double *__restrict__ norm2) {
  __shared__ double rs[kBlock];
  double best = 0.0;
  for (int i = threadIdx.x; i < k; i += kBlock) {
    resid[i] = sqrt(fmax(G[i * k + i], 0.0));
    if (i < kn) {
      double sum = 0.0;
      for (int j = 0; j < kn; ++j) sum += fabs(G[i * k + j]);
      best = fmax(best, sum);
    }
  }
  rs[threadIdx.x] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0, tr = 0.0;
    for (int i = 0; i < kBlock; ++i) m = fmax(m, rs[i]);
    for (int i = 0; i < kn; ++i) tr += fmax(G[i * k + i], 0.0);
    *norm2 = sqrt(fmin(m, tr));
  }
}

template <typename TX, typename TO>
sped_status launch_tsmm_t(int64_t n, int kin, int kout, const void *X, int64_t ldx, const double *T, void *O,
                          int64_t ldo, hipStream_t s) {
  int vec = pick_vec(kout, {ldo}, {O}, {int(sizeof(TO))});
  int lanes = (kout + vec - 1) / vec;
  int ytiles = (lanes + 63) / 64;
  int G = lanes >= 64 ? 64 : next_pow2(lanes);
  int lgG = ilog2(G);
  int64_t blocks = (n + (kBlock >> lgG) - 1) / (kBlock >> lgG);
  size_t shm = size_t(kin) * ((kout + 3) & ~3) * sizeof(float);
  const dim3 grid = dim3(unsigned(blocks), unsigned(ytiles));
  SPED_TRY(set_max_lds(tsmm_kernel<TX, TO, 4>, shm));
  SPED_TRY(set_max_lds(tsmm_kernel<TX, TO, 2>, shm));
  SPED_TRY(set_max_lds(tsmm_kernel<TX, TO, 1>, shm));
#define SPED_TSMM(V)                                                                          \
  hipLaunchKernelGGL((tsmm_kernel<TX, TO, V>), grid, dim3(kBlock), shm, s, n, kin, kout, G, lgG, \
                     static_cast<const TX *>(X), ldx, T, static_cast<TO *>(O), ldo)
  if (vec == 4) SPED_TSMM(4);
  else if (vec == 2) SPED_TSMM(2);
  else SPED_TSMM(1);
#undef SPED_TSMM
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

}  // namespace

size_t gram_ws_doubles(int64_t n, int64_t ka, int64_t kb) {
  // the larger of the symmetric and general plans
  GramPlan a = gram_plan(n, int(ka), int(kb), false), b = gram_plan(n, int(ka), int(kb), ka == kb);
  return size_t(a.nparts > b.nparts ? a.nparts : b.nparts) * ka * kb;
}

sped_status launch_gram(int64_t n, int ka, int kb, const void *A, int64_t lda, int ta, const void *B, int64_t ldb,
                        int tb, double *G, double *partials, hipStream_t s) {
  if (ka < 1 || kb < 1 || ka > kMaxK || kb > kMaxK) return fail(SPED_E_UNSUPPORTED, "gram width outside [1, 128]");
  const bool sym = (A == B) && (lda == ldb) && (ka == kb) && (ta == tb);
  const GramPlan plan = gram_plan(n, ka, kb, sym);
  sped_status st;
  const bool a32 = ta == SPED_F32, b32 = tb == SPED_F32;
  if ((ta != SPED_F32 && ta != SPED_BF16) || (tb != SPED_F32 && tb != SPED_BF16))
    return fail(SPED_E_UNSUPPORTED, "gram dtype");
  if (sym)
    st = a32 ? launch_gram_plain<float, float, true>(n, ka, kb, A, lda, B, ldb, partials, plan, s)
             : launch_gram_plain<bf16_t, bf16_t, true>(n, ka, kb, A, lda, B, ldb, partials, plan, s);
  else if (a32 && b32)
    st = launch_gram_plain<float, float, false>(n, ka, kb, A, lda, B, ldb, partials, plan, s);
  else if (!a32 && !b32)
    st = launch_gram_plain<bf16_t, bf16_t, false>(n, ka, kb, A, lda, B, ldb, partials, plan, s);
  else if (!a32 && b32)
    st = launch_gram_plain<bf16_t, float, false>(n, ka, kb, A, lda, B, ldb, partials, plan, s);
  else
    st = launch_gram_plain<float, bf16_t, false>(n, ka, kb, A, lda, B, ldb, partials, plan, s);
  if (st != SPED_OK) return st;
  return launch_sum_partials(partials, plan.nparts, int64_t(ka) * kb, G, false, s);
}

sped_status launch_tsmm(int64_t n, int kin, int kout, const void *X, int64_t ldx, int tx, const double *T,
                        void *O, int64_t ldo, int to, hipStream_t s) {
  if (n == 0) return SPED_OK;
  if (tx == SPED_F32 && to == SPED_F32) return launch_tsmm_t<float, float>(n, kin, kout, X, ldx, T, O, ldo, s);
  if (tx == SPED_F32 && to == SPED_BF16) return launch_tsmm_t<float, bf16_t>(n, kin, kout, X, ldx, T, O, ldo, s);
  if (tx == SPED_BF16 && to == SPED_F32) return launch_tsmm_t<bf16_t, float>(n, kin, kout, X, ldx, T, O, ldo, s);
  if (tx == SPED_BF16 && to == SPED_BF16) return launch_tsmm_t<bf16_t, bf16_t>(n, kin, kout, X, ldx, T, O, ldo, s);
  return fail(SPED_E_UNSUPPORTED, "tsmm dtype");
}


sped_status launch_resid(int64_t n, int k, int kn, const float *Z, const void *Q, int64_t ld, int tq,
                         const double *theta, double *G, double *resid, double *norm2, double *partials,
                         hipStream_t s) {
  if (k < 1 || k > kMaxK || kn < 1 || kn > k) return fail(SPED_E_UNSUPPORTED, "resid width outside [1, 128]");
  const GramPlan plan = gram_plan(n, k, k, true);
  sped_status st;
  if (tq == SPED_F32) {
    ResidLoad<float> ld_{Z, static_cast<const float *>(Q), ld, theta};
    st = launch_gram_maxt<ResidLoad<float>, true>(n, k, k, ld_, partials, plan, s);
  } else {
    ResidLoad<bf16_t> ld_{Z, static_cast<const bf16_t *>(Q), ld, theta};
    st = launch_gram_maxt<ResidLoad<bf16_t>, true>(n, k, k, ld_, partials, plan, s);
  }
  if (st != SPED_OK) return st;
  SPED_TRY(launch_sum_partials(partials, plan.nparts, int64_t(k) * k, G, false, s));
  hipLaunchKernelGGL(resid_norms_kernel, dim3(1), dim3(kBlock), 0, s, k, kn, G, resid, norm2);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

}  // namespace sped

using namespace sped;

extern "C" sped_status sped_gram(int64_t n, int64_t ka, int64_t kb, const void *A, int64_t lda, const void *B,
                                 int64_t ldb, int32_t dt, double *G, void *ws, size_t *ws_bytes,
                                 sped_stream_t stream) {
  clear_error();
  if (n < 0 || ka < 1 || kb < 1) return fail(SPED_E_INVALID, "gram shape");
  if (ka > kMaxK || kb > kMaxK) return fail(SPED_E_UNSUPPORTED, "gram width > 128");
  if (lda < ka || ldb < kb) return fail(SPED_E_INVALID, "gram leading dimension");
  if (dt != SPED_F32 && dt != SPED_BF16) return fail(SPED_E_UNSUPPORTED, "gram dtype");
  if ((n > 0 && (!A || !B)) || !G) return fail(SPED_E_INVALID, "gram NULL pointer");
  Carver c(ws);
  double *partials = c.take<double>(gram_ws_doubles(n, ka, kb));
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, c.bytes(), &query));
  if (query) return SPED_OK;
  return launch_gram(n, int(ka), int(kb), A, lda, dt, B, ldb, dt, G, partials, as_stream(stream));
}
