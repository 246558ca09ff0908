// Tall-skinny dense kernels of the block solver:
//   gram   G = A^T B in float64 on the float64 matrix cores
//          (v_mfma_f64_16x16x4f64), one 16x16 output tile per MFMA chain;
//   tsmm   O = X T for a small k_in x k_out matrix T (float64 in memory, float
//          in LDS) on the float32 matrix cores (v_mfma_f32_16x16x4f32);
//   resid  R^T R for R = Z - Q diag(theta) formed on the fly (same Gram
//          kernels), column norms and an upper bound on ||R||_2.
// Split over rows, every block writes its own partial; a second pass adds the
// partials in a fixed order, so results are bitwise reproducible.
#include "common.h"

namespace sped {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxK = 128;        // ka, kb <= kMaxK
constexpr int kGramBlocks = 512;   // narrow Gram
constexpr int kWideBlocks = 1024;  // wide Gram

typedef double double4_t __attribute__((ext_vector_type(4)));

template <typename T>
__device__ inline double load_as_double(const T *p);
template <>
__device__ inline double load_as_double<float>(const float *p) { return double(*p); }
template <>
__device__ inline double load_as_double<bf16_t>(const bf16_t *p) { return double(bf16_to_f32(*p)); }

// Elements c and c + 1 with one load (p aligned to two elements).
template <typename T>
__device__ inline void load2_as_double(const T *p, double &x0, double &x1);
template <>
__device__ inline void load2_as_double<float>(const float *p, double &x0, double &x1) {
  const float2 v = *reinterpret_cast<const float2 *>(p);
  x0 = double(v.x);
  x1 = double(v.y);
}
template <>
__device__ inline void load2_as_double<bf16_t>(const bf16_t *p, double &x0, double &x1) {
  const uint32_t v = *reinterpret_cast<const uint32_t *>(p);
  x0 = double(bf16_to_f32(bf16_t(v & 0xffffu)));
  x1 = double(bf16_to_f32(bf16_t(v >> 16)));
}

// Operand loaders of the Gram kernels: element (row, c) of the left and right
// factors, converted to float64; a2/b2 give elements c and c + 1 (c even,
// rows aligned to two elements).
// kPairWaves: wavefronts per block of the column-pair Gram.  With 512 blocks
// a plain loader is fastest at 4 (the fixed-order LDS merge is 4 steps), the
// residual loader, whose two operand streams want more loads in flight, at 8
// (1e6 x 32 float32: 53 us against 62 at 16 and 90 at 4).
template <typename T1, typename T2>
struct PlainLoad {
  static constexpr int kPairWaves = 4;
  const T1 *A;
  int64_t lda;
  const T2 *B;
  int64_t ldb;
  __device__ double a(int64_t r, int c) const { return load_as_double(A + r * lda + c); }
  __device__ double b(int64_t r, int c) const { return load_as_double(B + r * ldb + c); }
  __device__ void a2(int64_t r, int c, double &x0, double &x1) const { load2_as_double(A + r * lda + c, x0, x1); }
  __device__ void b2(int64_t r, int c, double &x0, double &x1) const { load2_as_double(B + r * ldb + c, x0, x1); }
};

// Residual block R = Z - Q diag(theta) formed on the fly (both factors are R).
template <typename TQ>
struct ResidLoad {
  static constexpr int kPairWaves = 8;
  const float *Z;
  const TQ *Q;
  int64_t ld;
  const double *theta;
  __device__ double a(int64_t r, int c) const {
    return double(Z[r * ld + c]) - theta[c] * load_as_double(Q + r * ld + c);
  }
  __device__ double b(int64_t r, int c) const { return a(r, c); }
  __device__ void a2(int64_t r, int c, double &x0, double &x1) const {
    double z0, z1, q0, q1;
    load2_as_double(Z + r * ld + c, z0, z1);
    load2_as_double(Q + r * ld + c, q0, q1);
    x0 = z0 - theta[c] * q0;
    x1 = z1 - theta[c + 1] * q1;
  }
  __device__ void b2(int64_t r, int c, double &x0, double &x1) const { a2(r, c, x0, x1); }
};

// Wide Gram (a width above 32, both <= 128; symmetric only above 80).  The
// block has NW wavefronts;
// wavefront p owns the 16-row output block p (waves past the last block exit
// at once) and forms its tiles (p, q) for every q < TB (q >= p when SYM) over
// all of the block's rows, 4 KU rows per round: lane (li, lk) holds element
// [row + 4u + lk][16 block + li] of each operand fragment (the float64 MFMA
// operand layout).  Every load is unconditional: column indices are clamped
// into range (a padded column only feeds output entries that are never
// written) and rows past the end are clamped to the block's first row and
// scaled by zero, so no branch separates the loads of a round.  Two fragment
// buffers alternate, the next round's loads being issued before the current
// round's MFMAs.  Wavefronts write disjoint tiles of the block's partial; with
// SYM the tiles above the diagonal are mirrored.
template <typename LD, int TBM, int NW, bool SYM>
__global__ __launch_bounds__(64 * NW) void gram_wide_kernel(int64_t n, int ka, int kb, LD ld,
                                                            int64_t rows_per_block, double *__restrict__ partials) {
  constexpr int KU = TBM <= 4 ? 4 : 2;
  constexpr int STEP = 4 * KU;
  const int TA = (ka + 15) / 16, TB = (kb + 15) / 16;
  // wave-uniform (read from lane 0), so the tile tests below are scalar branches
  const int pb = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (pb >= TA) return;  // no barriers in this kernel
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t r_begin = int64_t(blockIdx.x) * rows_per_block;
  const int64_t r_end = min(n, r_begin + rows_per_block);
  const int ca = min(pb * 16 + li, ka - 1);
  int cb[TBM];
#pragma unroll
  for (int q = 0; q < TBM; ++q) cb[q] = min(q * 16 + li, kb - 1);
  double4_t acc[TBM];
#pragma unroll
  for (int q = 0; q < TBM; ++q) acc[q] = double4_t{0.0, 0.0, 0.0, 0.0};

  struct Frag {
    double a[KU], b[KU][TBM];
  };
  auto load = [&](int64_t r, Frag &f) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int64_t row = r + 4 * u + lk;
      const bool rok = row < r_end;
      const int64_t rc = rok ? row : r_begin;
      const double rm = rok ? 1.0 : 0.0;
      f.a[u] = ld.a(rc, ca) * rm;
#pragma unroll
      for (int q = 0; q < TBM; ++q) f.b[u][q] = ld.b(rc, cb[q]) * rm;
    }
  };
  auto mma = [&](const Frag &f) {
#pragma unroll
    for (int q = 0; q < TBM; ++q)
      if (q < TB && (!SYM || q >= pb))
#pragma unroll
        for (int u = 0; u < KU; ++u) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.a[u], f.b[u][q], acc[q], 0, 0, 0);
  };

  if (r_begin < r_end) {
    Frag f0, f1;
    load(r_begin, f0);
    for (int64_t r = r_begin; r < r_end; r += 2 * STEP) {
      load(r + STEP, f1);  // rows past the end load as zeros
      mma(f0);
      load(r + 2 * STEP, f0);
      mma(f1);
    }
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
  double *out = partials + int64_t(blockIdx.x) * ka * kb;
#pragma unroll
  for (int q = 0; q < TBM; ++q) {
    if (q < TB && (!SYM || q >= pb)) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = pb * 16 + int(rowid[r]);
        const int jj = q * 16 + int(colid[r]);
        if (ii < ka && jj < kb) out[ii * kb + jj] = acc[q][r];
        if (SYM && pb != q && jj < ka && ii < kb) out[jj * kb + ii] = acc[q][r];
      }
    }
  }
}

// Narrow Gram (both widths <= 32, or a symmetric Gram up to 80 columns): 4
// wavefronts per block, each streams its own interleaved 16-row chunks of the
// block's rows and forms all TA x TB tiles (operand fragments loaded once per
// row group and reused across tiles).  The
// wavefronts then add their tiles into one LDS copy in wavefront order (fixed
// order: deterministic) and the block writes one partial.
constexpr int kNarrowBlock = 256;
template <typename LD, int TA, int TB, bool SYM>
__global__ __launch_bounds__(kNarrowBlock) void gram_narrow_kernel(int64_t n, int ka, int kb, LD ld,
                                                                   int64_t rows_per_block,
                                                                   double *__restrict__ partials) {
  constexpr int KU = 4;
  constexpr int NW = kNarrowBlock / 64;
  __shared__ double red[TA * 16 * TB * 16];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  double4_t acc[TA][TB];
#pragma unroll
  for (int p = 0; p < TA; ++p)
#pragma unroll
    for (int q = 0; q < TB; ++q) acc[p][q] = double4_t{0.0, 0.0, 0.0, 0.0};
  const int64_t r_begin = int64_t(blockIdx.x) * rows_per_block;
  const int64_t r_end = min(n, r_begin + rows_per_block);
  // Loads are unconditional (clamped columns feed only output entries that are
  // never written; rows past the end re-read the block's first row, scaled by
  // zero), and two fragment buffers alternate so that the next chunk's loads
  // are in flight during the current chunk's MFMAs.
  int ca[TA], cb[TB];
#pragma unroll
  for (int p = 0; p < TA; ++p) ca[p] = min(p * 16 + li, ka - 1);
#pragma unroll
  for (int q = 0; q < TB; ++q) cb[q] = min(q * 16 + li, kb - 1);
  struct Frag {
    double a[KU][TA], b[KU][TB];
  };
  auto load = [&](int64_t r, Frag &f) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int64_t row = r + 4 * u + lk;
      const bool rok = row < r_end;
      const int64_t rc = rok ? row : r_begin;
      const double rm = rok ? 1.0 : 0.0;
#pragma unroll
      for (int p = 0; p < TA; ++p) f.a[u][p] = ld.a(rc, ca[p]) * rm;
      if (!SYM)
#pragma unroll
        for (int q = 0; q < TB; ++q) f.b[u][q] = ld.b(rc, cb[q]) * rm;
    }
  };
  auto mma = [&](const Frag &f) {
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int p = 0; p < TA; ++p)
#pragma unroll
        for (int q = 0; q < TB; ++q)
          if (!SYM || p <= q)
            acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.a[u][p], SYM ? f.a[u][q] : f.b[u][q], acc[p][q], 0,
                                                             0, 0);
  };
  constexpr int64_t STRIDE = 4 * KU * NW;
  const int64_t first = r_begin + 4 * KU * wave;
  if (first < r_end) {
    Frag f0, f1;
    load(first, f0);
    for (int64_t r = first; r < r_end; r += 2 * STRIDE) {
      load(r + STRIDE, f1);  // rows past the end load as zeros
      mma(f0);
      load(r + 2 * STRIDE, f0);
      mma(f1);
    }
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

// Narrow Gram with column pairs (both widths even and in (16, 32], rows
// aligned to two elements): lane (li, lk) loads columns 2li and 2li + 1 of row
// row + 4u + lk with one load, so 16 lanes read a whole row and a load
// instruction covers 4 rows (half the instructions of the one-column form).
// Component v of the pair feeds MFMA operand v: the tile of MFMA pair
// (v1, v2) holds G[2i + v1][2j + v2] (i, j the tile's row and column), the
// four tiles together the whole 32 x 32 block.  With SYM the tile (1, 0) is
// the transpose of (0, 1) and is not formed.  Otherwise as the one-column
// form: unconditional loads, two alternating fragment buffers, the
// wavefronts adding their tiles into LDS in wavefront order, one partial per
// block.  Blocks of LD::kPairWaves wavefronts: with plain loads 4 against
// 16 took the symmetric 1e6 x 32 float32 Gram from 48.9 to 36.8 us and A^T B
// from 81.1 to 51.9 us.
template <typename LD, bool SYM>
__global__ __launch_bounds__(64 * LD::kPairWaves) void gram_pair_kernel(int64_t n, int ka, int kb, LD ld,
                                                                        int64_t rows_per_block,
                                                                        double *__restrict__ partials) {
  constexpr int KU = 4;
  constexpr int NW = LD::kPairWaves;
  constexpr int W = 32;
  __shared__ double red[W * W];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  double4_t acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = double4_t{0.0, 0.0, 0.0, 0.0};
  const int64_t r_begin = int64_t(blockIdx.x) * rows_per_block;
  const int64_t r_end = min(n, r_begin + rows_per_block);
  // pairs past the width re-read the last pair (they feed only output entries
  // that are never written)
  const int ca = 2 * min(li, ka / 2 - 1), cb = 2 * min(li, kb / 2 - 1);
  struct Frag {
    double a[KU][2], b[KU][2];
  };
  auto load = [&](int64_t r, Frag &f) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int64_t row = r + 4 * u + lk;
      const bool rok = row < r_end;
      const int64_t rc = rok ? row : r_begin;
      const double rm = rok ? 1.0 : 0.0;
      ld.a2(rc, ca, f.a[u][0], f.a[u][1]);
      f.a[u][0] *= rm;
      f.a[u][1] *= rm;
      if (!SYM) {
        ld.b2(rc, cb, f.b[u][0], f.b[u][1]);
        f.b[u][0] *= rm;
        f.b[u][1] *= rm;
      }
    }
  };
  auto mma = [&](const Frag &f) {
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          if (!SYM || p <= q)
            acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.a[u][p], SYM ? f.a[u][q] : f.b[u][q], acc[p][q], 0,
                                                             0, 0);
  };
  constexpr int64_t STRIDE = 4 * KU * NW;
  const int64_t first = r_begin + 4 * KU * wave;
  if (first < r_end) {
    Frag f0, f1;
    load(first, f0);
    for (int64_t r = first; r < r_end; r += 2 * STRIDE) {
      load(r + STRIDE, f1);  // rows past the end load as zeros
      mma(f0);
      load(r + 2 * STRIDE, f0);
      mma(f1);
    }
  }
  // accumulator slot -> (row, column) of the tile, read off the matrix core
  const double4_t zero4 = double4_t{0.0, 0.0, 0.0, 0.0};
  const double4_t rowid = __builtin_amdgcn_mfma_f64_16x16x4f64(lk == 0 ? double(li) : 0.0, lk == 0 ? 1.0 : 0.0,
                                                               zero4, 0, 0, 0);
  const double4_t colid = __builtin_amdgcn_mfma_f64_16x16x4f64(lk == 0 ? 1.0 : 0.0, lk == 0 ? double(li) : 0.0,
                                                               zero4, 0, 0, 0);
  for (int w = 0; w < NW; ++w) {
    if (wave == w) {
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          if (!SYM || p <= q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = 2 * int(rowid[r]) + p, j = 2 * int(colid[r]) + q;
              red[i * W + j] = (w == 0 ? 0.0 : red[i * W + j]) + acc[p][q][r];
            }
    }
    __syncthreads();
  }
  double *out = partials + int64_t(blockIdx.x) * ka * kb;
  for (int idx = threadIdx.x; idx < ka * kb; idx += 64 * NW) {
    const int i = idx / kb, j = idx - i * kb;
    out[idx] = (SYM && (i & 1) && !(j & 1)) ? red[j * W + i] : red[i * W + j];
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

// O = X T for a small kin x kout T on the float32 matrix cores
// (v_mfma_f32_16x16x4f32).  T (float64 in memory) is staged as float in LDS,
// zero-padded to a multiple of 16 rows, with a row stride of 16 mod 64 floats
// so that the four k-rows a wavefront reads at once fall in distinct banks.
// Each wavefront forms 16-row strips of O (all TBO 16-column tiles at once),
// striding over the strips of the grid; lane (li, lk) streams X[row + li][k +
// lk], four k-steps per batch.  Rows past n are clamped (their outputs are not
// stored); columns past kin are clamped and zeroed bitwise, so non-finite
// data never meets the zero padding of T.  A strip's inputs are all read
// before its outputs are written, so O may alias X.  With ADD the stored value
// is X T + beta Y (Y read element by element just before the store, so O may
// alias Y as well).
typedef float float4_t __attribute__((ext_vector_type(4)));

inline int tsmm_lds_stride(int w) { return ((w - 16 + 63) / 64) * 64 + 16; }

template <typename TX, typename TO, int TBO, bool ADD>
__global__ __launch_bounds__(kBlock) void tsmm_kernel(int64_t n, int kin, int kout, const TX *__restrict__ X,
                                                      int64_t ldx, const double *__restrict__ T, TO *O,
                                                      int64_t ldo, const TO *Y, int64_t ldy, float beta) {
  extern __shared__ float sT[];
  const int S = ((16 * TBO - 16 + 63) / 64) * 64 + 16;
  const int kin16 = (kin + 15) & ~15;
  for (int i = threadIdx.x; i < kin16 * 16 * TBO; i += kBlock) {
    const int r = i / (16 * TBO), c = i - r * (16 * TBO);
    sT[r * S + c] = (r < kin && c < kout) ? float(T[r * kout + c]) : 0.f;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const float4_t zero4 = float4_t{0.f, 0.f, 0.f, 0.f};
  // output slot layout read off the matrix core (as for the float64 Gram)
  const float4_t rowid =
      __builtin_amdgcn_mfma_f32_16x16x4f32(lk == 0 ? float(li) : 0.f, lk == 0 ? 1.f : 0.f, zero4, 0, 0, 0);
  const float4_t colid =
      __builtin_amdgcn_mfma_f32_16x16x4f32(lk == 0 ? 1.f : 0.f, lk == 0 ? float(li) : 0.f, zero4, 0, 0, 0);
  const int64_t strips = (n + 15) / 16;
  for (int64_t st = int64_t(blockIdx.x) * 4 + wave; st < strips; st += int64_t(gridDim.x) * 4) {
    const int64_t row0 = st * 16;
    const int64_t row = min(row0 + li, n - 1);
    const TX *xr = X + row * ldx;
    float4_t acc[TBO];
#pragma unroll
    for (int q = 0; q < TBO; ++q) acc[q] = zero4;
    for (int k0 = 0; k0 < kin16; k0 += 16) {
      float x[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int kk = k0 + 4 * j + lk;
        const float v = to_f32<TX>(xr[min(kk, kin - 1)]);
        x[j] = __uint_as_float(__float_as_uint(v) & (kk < kin ? 0xffffffffu : 0u));
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int q = 0; q < TBO; ++q)
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[j], sT[(k0 + 4 * j + lk) * S + q * 16 + li], acc[q], 0,
                                                        0, 0);
    }
#pragma unroll
    for (int q = 0; q < TBO; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t orow = row0 + int(rowid[r]);
        const int oc = q * 16 + int(colid[r]);
        if (orow < n && oc < kout) {
          float v = acc[q][r];
          if (ADD) v = fmaf(beta, to_f32<TO>(Y[orow * ldy + oc]), v);
          O[orow * ldo + oc] = from_f32<TO>(v);
        }
      }
  }
}

// The same product with 4-wide row loads, for kin a multiple of 4 and rows
// aligned to 4 elements.  The contraction index is permuted inside each
// 16-column chunk: lane (li, lk) loads columns 16c + 4lk .. 16c + 4lk + 3 of
// its row as one vector and feeds the j-th of them to the j-th MFMA of the
// chunk, and reads the matching row 16c + 4lk + j of T.  T's LDS row stride
// is 4 mod 64 floats, so those four rows (4 apart) fall in distinct banks.
// Each wavefront loads its next strip before the current strip's MFMAs.
inline int tsmm4_lds_stride(int w) { return ((w + 63) / 64) * 64 + 4; }

template <typename TX, typename TO, int TB, bool ADD>
__global__ __launch_bounds__(kBlock) void tsmm4_kernel(int64_t n, int kin, int kout, const TX *__restrict__ X,
                                                       int64_t ldx, const double *__restrict__ T, TO *O,
                                                       int64_t ldo, const TO *Y, int64_t ldy, float beta) {
  extern __shared__ float sT[];
  const int S = ((16 * TB + 63) / 64) * 64 + 4;
  const int kc = (kin + 15) >> 4;  // chunks of 16 input columns, <= TB
  for (int i = threadIdx.x; i < kc * 16 * 16 * TB; i += kBlock) {
    const int r = i / (16 * TB), c = i - r * (16 * TB);
    sT[r * S + c] = (r < kin && c < kout) ? float(T[r * kout + c]) : 0.f;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const float4_t zero4 = float4_t{0.f, 0.f, 0.f, 0.f};
  const float4_t rowid =
      __builtin_amdgcn_mfma_f32_16x16x4f32(lk == 0 ? float(li) : 0.f, lk == 0 ? 1.f : 0.f, zero4, 0, 0, 0);
  const float4_t colid =
      __builtin_amdgcn_mfma_f32_16x16x4f32(lk == 0 ? 1.f : 0.f, lk == 0 ? float(li) : 0.f, zero4, 0, 0, 0);
  const int64_t strips = (n + 15) / 16;
  const int64_t step = int64_t(gridDim.x) * 4;
  // lane's columns in chunk c: 16c + 4lk .. +3, all inside [0, kin) or all
  // outside (then columns 0..3 are loaded, which exist since kin >= 4, and zeroed)
  auto load_strip = [&](int64_t st, float (&xs)[TB][4]) {
    const int64_t row = min(st * 16 + li, n - 1);
    const TX *xr = X + row * ldx;
#pragma unroll
    for (int c = 0; c < TB; ++c) {
      const int col = 16 * c + 4 * lk;
      VecIO<TX, 4>::load(xr + (col < kin ? col : 0), xs[c]);
      const uint32_t keep = col < kin ? 0xffffffffu : 0u;
#pragma unroll
      for (int j = 0; j < 4; ++j) xs[c][j] = __uint_as_float(__float_as_uint(xs[c][j]) & keep);
    }
  };
  int64_t st = int64_t(blockIdx.x) * 4 + wave;
  if (st >= strips) return;
  float xa[TB][4];
  load_strip(st, xa);
  for (; st < strips; st += step) {
    float xb[TB][4];
    const int64_t nx = st + step;
    if (nx < strips) load_strip(nx, xb);
    float4_t acc[TB];
#pragma unroll
    for (int q = 0; q < TB; ++q) acc[q] = zero4;
#pragma unroll
    for (int c = 0; c < TB; ++c) {
      if (c < kc) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int q = 0; q < TB; ++q)
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[c][j], sT[(16 * c + 4 * lk + j) * S + q * 16 + li],
                                                          acc[q], 0, 0, 0);
      }
    }
    const int64_t row0 = st * 16;
#pragma unroll
    for (int q = 0; q < TB; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t orow = row0 + int(rowid[r]);
        const int oc = q * 16 + int(colid[r]);
        if (orow < n && oc < kout) {
          float v = acc[q][r];
          if (ADD) v = fmaf(beta, to_f32<TO>(Y[orow * ldy + oc]), v);
          O[orow * ldo + oc] = from_f32<TO>(v);
        }
      }
#pragma unroll
    for (int c = 0; c < TB; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) xa[c][j] = xb[c][j];
  }
}

template <typename TX, typename TO, bool ADD>
sped_status launch_tsmm_t(int64_t n, int kin, int kout, const void *X, int64_t ldx, const double *T, void *O,
                          int64_t ldo, const void *Y, int64_t ldy, float beta, hipStream_t s) {
  const uintptr_t xa = reinterpret_cast<uintptr_t>(X);
  const bool vec4 = kin % 4 == 0 && ldx % 4 == 0 && xa % (4 * sizeof(TX)) == 0;
  if (vec4) {
    const int kmax = kin > kout ? kin : kout;
    // 16-column tiles; 5 and 6 are instantiated so that widths of 65..96 (the
    // solver's 64 + guard) do not pay for 8 tiles of matrix-core work
    const int TB = kmax <= 16 ? 1 : kmax <= 32 ? 2 : kmax <= 64 ? 4 : kmax <= 80 ? 5 : kmax <= 96 ? 6 : 8;
    const size_t shm = size_t((kin + 15) & ~15) * tsmm4_lds_stride(16 * TB) * sizeof(float);
    const int64_t strips = (n + 15) / 16;
    const int64_t want = (strips + 15) / 16;  // about 4 strips per wavefront
    const unsigned blocks = unsigned(want < 1 ? 1 : (want > 4096 ? 4096 : want));
#define SPED_TSMM4(B)                                                                                     \
  {                                                                                                       \
    SPED_TRY(set_max_lds(tsmm4_kernel<TX, TO, B, ADD>, shm));                                             \
    hipLaunchKernelGGL((tsmm4_kernel<TX, TO, B, ADD>), dim3(blocks), dim3(kBlock), shm, s, n, kin, kout,  \
                       static_cast<const TX *>(X), ldx, T, static_cast<TO *>(O), ldo,                     \
                       static_cast<const TO *>(Y), ldy, beta);                                            \
  }
    if (TB == 1) SPED_TSMM4(1)
    else if (TB == 2) SPED_TSMM4(2)
    else if (TB == 4) SPED_TSMM4(4)
    else if (TB == 5) SPED_TSMM4(5)
    else if (TB == 6) SPED_TSMM4(6)
    else SPED_TSMM4(8)
#undef SPED_TSMM4
    SPED_CHECK_HIP(hipGetLastError());
    return SPED_OK;
  }
  const int TBO = (kout + 15) / 16;
  const size_t shm = size_t((kin + 15) & ~15) * tsmm_lds_stride(16 * TBO) * sizeof(float);
  const int64_t strips = (n + 15) / 16;
  const int64_t want = (strips + 31) / 32;  // about 8 strips per wavefront
  const unsigned blocks = unsigned(want < 1 ? 1 : (want > 2048 ? 2048 : want));
#define SPED_TSMM(B)                                                                                     \
  {                                                                                                      \
    SPED_TRY(set_max_lds(tsmm_kernel<TX, TO, B, ADD>, shm));                                             \
    hipLaunchKernelGGL((tsmm_kernel<TX, TO, B, ADD>), dim3(blocks), dim3(kBlock), shm, s, n, kin, kout,  \
                       static_cast<const TX *>(X), ldx, T, static_cast<TO *>(O), ldo,                    \
                       static_cast<const TO *>(Y), ldy, beta);                                           \
  }
  if (TBO <= 1) SPED_TSMM(1)
  else if (TBO <= 2) SPED_TSMM(2)
  else if (TBO <= 4) SPED_TSMM(4)
  else if (TBO == 5) SPED_TSMM(5)
  else if (TBO == 6) SPED_TSMM(6)
  else SPED_TSMM(8)
#undef SPED_TSMM
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

struct GramPlan {
  int nblocks, nparts;
  bool narrow;
  int64_t rows_per_block;
};

GramPlan gram_plan(int64_t n, int ka, int kb, bool sym) {
  const int TA = (ka + 15) / 16, TB = (kb + 15) / 16;
  GramPlan p;
  p.narrow = (TA <= 2 && TB <= 2) || (sym && TA <= 5 && TB <= 5);
  // rows per block at least: one 64-row pass per wavefront keeps small
  // Grams from walking many chunks in sequence on a few blocks (2,000 x 14:
  // residual Gram 19.9 -> 7.7 us, symmetric 7.7 -> 4.3 us against 1024 rows)
  const int64_t unit = p.narrow ? 256 : 128;
  const int64_t align = p.narrow ? 256 : 64;
  const int64_t cap = p.narrow ? kGramBlocks : kWideBlocks;
  int64_t nb = (n + unit - 1) / unit;
  p.nblocks = int(nb < cap ? (nb > 0 ? nb : 1) : cap);
  int64_t r = (n + p.nblocks - 1) / p.nblocks;
  p.rows_per_block = (r + align - 1) / align * align;
  p.nparts = p.nblocks;
  return p;
}

template <typename LD, int TBM, int NW, bool SYM>
sped_status launch_gram_wide_t(int64_t n, int ka, int kb, const LD &ld, double *partials, const GramPlan &p,
                               hipStream_t s) {
  hipLaunchKernelGGL((gram_wide_kernel<LD, TBM, NW, SYM>), dim3(p.nblocks), dim3(64 * NW), 0, s, n, ka, kb, ld,
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
                             hipStream_t s, bool pairs) {
  const int TA = (ka + 15) / 16, TB = (kb + 15) / 16;
  // column pairs fill the four 16 x 16 tiles only when both widths are in (16, 32]
  if (p.narrow && pairs && TA == 2 && TB == 2 && ka % 2 == 0 && kb % 2 == 0 && ka > 16 && kb > 16) {
    hipLaunchKernelGGL((gram_pair_kernel<LD, SYM>), dim3(p.nblocks), dim3(64 * LD::kPairWaves), 0, s, n, ka, kb,
                       ld, p.rows_per_block, partials);
    SPED_CHECK_HIP(hipGetLastError());
    return SPED_OK;
  }
  if (p.narrow) {
    if (TA == 1 && TB == 1) return launch_gram_narrow_t<LD, 1, 1, SYM>(n, ka, kb, ld, partials, p, s);
    if (TA == 1 && TB == 2) return launch_gram_narrow_t<LD, 1, 2, SYM>(n, ka, kb, ld, partials, p, s);
    if (TA == 2 && TB == 1) return launch_gram_narrow_t<LD, 2, 1, SYM>(n, ka, kb, ld, partials, p, s);
    if (TA == 2 && TB == 2) return launch_gram_narrow_t<LD, 2, 2, SYM>(n, ka, kb, ld, partials, p, s);
    // A symmetric Gram up to 80 columns (the plan's 512 blocks): each
    // wavefront forms all of its rows' tiles, so no row is loaded twice.
    // Against the wide kernel, whose wavefronts each reload whole rows: 1e6 x
    // 56 float32 177.8 -> 101.5 us (residual Gram 234.6 -> 123.5 us), 1e6 x 72
    // float32 268.3 -> 174.5 us (residual 377.9 -> 209.5 us), 4e6 x 64 bf16
    // 598.5 -> 366.3 us.  For A^T B (two operands, twice the fragment
    // registers, one wavefront per SIMD) the wide kernel stays ahead in
    // float32, so the plan keeps those wide.
    if (SYM && TA == 3) return launch_gram_narrow_t<LD, 3, 3, SYM>(n, ka, kb, ld, partials, p, s);
    if (SYM && TA == 4) return launch_gram_narrow_t<LD, 4, 4, SYM>(n, ka, kb, ld, partials, p, s);
    if (SYM && TA == 5) return launch_gram_narrow_t<LD, 5, 5, SYM>(n, ka, kb, ld, partials, p, s);
    return fail(SPED_E_UNSUPPORTED, "gram: no narrow kernel for this width");
  }
  // TBM = TB where instantiated: column tiles past TB would still be loaded
  // (clamped) by every lane, and the wide kernel is bound by its load
  // instructions
  if (TA <= 4) {
    if (TB <= 4) return launch_gram_wide_t<LD, 4, 4, SYM>(n, ka, kb, ld, partials, p, s);
    if (TB == 5) return launch_gram_wide_t<LD, 5, 4, SYM>(n, ka, kb, ld, partials, p, s);
    if (TB == 6) return launch_gram_wide_t<LD, 6, 4, SYM>(n, ka, kb, ld, partials, p, s);
    return launch_gram_wide_t<LD, 8, 4, SYM>(n, ka, kb, ld, partials, p, s);
  }
  if (TB == 5) return launch_gram_wide_t<LD, 5, 8, SYM>(n, ka, kb, ld, partials, p, s);
  if (TB == 6) return launch_gram_wide_t<LD, 6, 8, SYM>(n, ka, kb, ld, partials, p, s);
  return launch_gram_wide_t<LD, 8, 8, SYM>(n, ka, kb, ld, partials, p, s);
}

template <typename T1, typename T2, bool SYM>
sped_status launch_gram_plain(int64_t n, int ka, int kb, const void *A, int64_t lda, const void *B, int64_t ldb,
                              double *partials, const GramPlan &p, hipStream_t s) {
  PlainLoad<T1, T2> ld{static_cast<const T1 *>(A), lda, static_cast<const T2 *>(B), ldb};
  // column pairs need every row to start on a two-element boundary
  const bool pairs = lda % 2 == 0 && ldb % 2 == 0 && reinterpret_cast<uintptr_t>(A) % (2 * sizeof(T1)) == 0 &&
                     reinterpret_cast<uintptr_t>(B) % (2 * sizeof(T2)) == 0;
  return launch_gram_maxt<PlainLoad<T1, T2>, SYM>(n, ka, kb, ld, partials, p, s, pairs);
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
                        void *O, int64_t ldo, int to, hipStream_t s, const void *Y, int64_t ldy, float beta) {
  if (kin < 1 || kout < 1 || kin > kMaxK || kout > kMaxK) return fail(SPED_E_UNSUPPORTED, "tsmm width outside [1, 128]");
  if (n == 0) return SPED_OK;
  if (Y && to != SPED_F32) return fail(SPED_E_UNSUPPORTED, "tsmm addend needs a float32 output");
  if (Y) {
    if (tx == SPED_F32) return launch_tsmm_t<float, float, true>(n, kin, kout, X, ldx, T, O, ldo, Y, ldy, beta, s);
    if (tx == SPED_BF16) return launch_tsmm_t<bf16_t, float, true>(n, kin, kout, X, ldx, T, O, ldo, Y, ldy, beta, s);
    return fail(SPED_E_UNSUPPORTED, "tsmm dtype");
  }
  if (tx == SPED_F32 && to == SPED_F32)
    return launch_tsmm_t<float, float, false>(n, kin, kout, X, ldx, T, O, ldo, nullptr, 0, 0.f, s);
  if (tx == SPED_F32 && to == SPED_BF16)
    return launch_tsmm_t<float, bf16_t, false>(n, kin, kout, X, ldx, T, O, ldo, nullptr, 0, 0.f, s);
  if (tx == SPED_BF16 && to == SPED_F32)
    return launch_tsmm_t<bf16_t, float, false>(n, kin, kout, X, ldx, T, O, ldo, nullptr, 0, 0.f, s);
  if (tx == SPED_BF16 && to == SPED_BF16)
    return launch_tsmm_t<bf16_t, bf16_t, false>(n, kin, kout, X, ldx, T, O, ldo, nullptr, 0, 0.f, s);
  return fail(SPED_E_UNSUPPORTED, "tsmm dtype");
}


sped_status launch_resid(int64_t n, int k, int kn, const float *Z, const void *Q, int64_t ld, int tq,
                         const double *theta, double *G, double *resid, double *norm2, double *partials,
                         hipStream_t s) {
  if (k < 1 || k > kMaxK || kn < 1 || kn > k) return fail(SPED_E_UNSUPPORTED, "resid width outside [1, 128]");
  const GramPlan plan = gram_plan(n, k, k, true);
  const size_t qsize = tq == SPED_F32 ? sizeof(float) : sizeof(bf16_t);
  const bool pairs = ld % 2 == 0 && reinterpret_cast<uintptr_t>(Z) % (2 * sizeof(float)) == 0 &&
                     reinterpret_cast<uintptr_t>(Q) % (2 * qsize) == 0;
  sped_status st;
  if (tq == SPED_F32) {
    ResidLoad<float> ld_{Z, static_cast<const float *>(Q), ld, theta};
    st = launch_gram_maxt<ResidLoad<float>, true>(n, k, k, ld_, partials, plan, s, pairs);
  } else {
    ResidLoad<bf16_t> ld_{Z, static_cast<const bf16_t *>(Q), ld, theta};
    st = launch_gram_maxt<ResidLoad<bf16_t>, true>(n, k, k, ld_, partials, plan, s, pairs);
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
