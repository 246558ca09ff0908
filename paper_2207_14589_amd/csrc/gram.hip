// Tall-skinny dense kernels of the block solver:
//   gram   G = A^T B in float64 on the float64 matrix cores
//          (v_mfma_f64_16x16x4f64), one 16x16 output tile per MFMA chain;
//   tsmm   O = X T for a small k_in x k_out matrix T (float64 in memory, float
//          in LDS), one lane group per row like the sparse step;
//   resid  per-column ||Z_i - theta_i Q_i||_2 in float64.
// Split over rows, every block writes its own partial; a second pass adds the
// partials in a fixed order, so results are bitwise reproducible.
#include "common.h"

namespace sped {
namespace {

constexpr int kBlock = 256;
constexpr int kChunk = 64;        // rows staged in LDS per round
constexpr int kMaxK = 128;        // ka, kb <= kMaxK
constexpr int kGramBlocks = 512;

typedef double double4_t __attribute__((ext_vector_type(4)));

template <typename T>
__device__ inline double load_as_double(const T *p);
template <>
__device__ inline double load_as_double<float>(const float *p) { return double(*p); }
template <>
__device__ inline double load_as_double<bf16_t>(const bf16_t *p) { return double(bf16_to_f32(*p)); }

// Tiles of the ka x kb output are assigned round-robin to the 4 waves; a wave
// holds at most MAXT tiles.  With SYM (A == B) only tiles p <= q are formed.
template <typename T, int MAXT, bool SYM>
__global__ __launch_bounds__(kBlock) void gram_kernel(int64_t n, int ka, int kb, const T *__restrict__ A,
                                                      int64_t lda, const T *__restrict__ B, int64_t ldb,
                                                      double *__restrict__ partials) {
  extern __shared__ double lds[];
  const int TA = (ka + 15) / 16, TB = (kb + 15) / 16;
  const int pa = TA * 16 + 1, pb = TB * 16 + 1;  // padded LDS row strides
  double *sA = lds;
  double *sB = SYM ? lds : lds + kChunk * pa;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;

  // tile list of this wave
  int tp[MAXT], tq[MAXT];
  int nt = 0;
  {
    int idx = 0;
    for (int p = 0; p < TA; ++p)
      for (int q = SYM ? p : 0; q < TB; ++q) {
        if (idx % 4 == wave && nt < MAXT) {
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

  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const int64_t r0 = ch * kChunk;
    __syncthreads();
    for (int i = threadIdx.x; i < kChunk * TA * 16; i += kBlock) {
      int r = i / (TA * 16), c = i - r * (TA * 16);
      int64_t gr = r0 + r;
      sA[r * pa + c] = (gr < n && c < ka) ? load_as_double(A + gr * lda + c) : 0.0;
    }
    if (!SYM)
      for (int i = threadIdx.x; i < kChunk * TB * 16; i += kBlock) {
        int r = i / (TB * 16), c = i - r * (TB * 16);
        int64_t gr = r0 + r;
        sB[r * pb + c] = (gr < n && c < kb) ? load_as_double(B + gr * ldb + c) : 0.0;
      }
    __syncthreads();
    const int sbs = SYM ? pa : pb;
#pragma unroll 4
    for (int kk = 0; kk < kChunk; kk += 4) {
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        if (t < nt) {
          double a = sA[(kk + lk) * pa + tp[t] * 16 + li];
          double b = sB[(kk + lk) * sbs + tq[t] * 16 + li];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
        }
      }
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

__global__ __launch_bounds__(kBlock) void sum_partials_kernel(const double *__restrict__ partials, int nparts,
                                                               int64_t count, double *__restrict__ out) {
  int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= count) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += partials[int64_t(p) * count + i];
  out[i] = s;
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

// partial[b][c] = sum over this block's rows of (Z[r,c] - theta[c] Q[r,c])^2
__global__ __launch_bounds__(kBlock) void resid_kernel(int64_t n, int k, const float *__restrict__ Z, int64_t ldz,
                                                        const float *__restrict__ Q, int64_t ldq,
                                                        const double *__restrict__ theta,
                                                        double *__restrict__ partials) {
  // thread layout: column c = threadIdx.x % kc, row lane = threadIdx.x / kc
  const int kc = k <= kBlock ? k : kBlock;
  const int rl = threadIdx.x / kc, nrl = kBlock / kc;
  const int c = threadIdx.x - rl * kc;
  __shared__ double red[kBlock];
  double s = 0.0;
  if (rl < nrl) {
    const double th = theta[c];
    for (int64_t r = int64_t(blockIdx.x) * nrl + rl; r < n; r += int64_t(gridDim.x) * nrl) {
      double d = double(Z[r * ldz + c]) - th * double(Q[r * ldq + c]);
      s += d * d;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < kc) {
    double t = 0.0;
    for (int i = 0; i < nrl; ++i) t += red[i * kc + threadIdx.x];
    partials[int64_t(blockIdx.x) * k + threadIdx.x] = t;
  }
}

__global__ void sqrt_sum_kernel(const double *__restrict__ partials, int nparts, int k, double *__restrict__ out) {
  int c = threadIdx.x;
  if (c >= k) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += partials[int64_t(p) * k + c];
  out[c] = sqrt(s);
}

constexpr int kResidBlocks = 512;

template <typename T, int MAXT, bool SYM>
sped_status launch_gram_t(int64_t n, int ka, int kb, const void *A, int64_t lda, const void *B, int64_t ldb,
                          double *partials, int nblocks, hipStream_t s) {
  const int TA = (ka + 15) / 16, TB = (kb + 15) / 16;
  size_t shm = size_t(kChunk) * (TA * 16 + 1) * sizeof(double);
  if (!SYM) shm += size_t(kChunk) * (TB * 16 + 1) * sizeof(double);
  SPED_TRY(set_max_lds(gram_kernel<T, MAXT, SYM>, shm));
  hipLaunchKernelGGL((gram_kernel<T, MAXT, SYM>), dim3(nblocks), dim3(kBlock), shm, s, n, ka, kb,
                     static_cast<const T *>(A), lda, static_cast<const T *>(B), ldb, partials);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

template <typename T, bool SYM>
sped_status launch_gram_maxt(int64_t n, int ka, int kb, const void *A, int64_t lda, const void *B,
                             int64_t ldb, double *partials, int nblocks, hipStream_t s) {
  const int TA = (ka + 15) / 16, TB = (kb + 15) / 16;
  int tiles = SYM ? TA * (TA + 1) / 2 : TA * TB;
  int per_wave = (tiles + 3) / 4;
  if (per_wave <= 1) return launch_gram_t<T, 1, SYM>(n, ka, kb, A, lda, B, ldb, partials, nblocks, s);
  if (per_wave <= 2) return launch_gram_t<T, 2, SYM>(n, ka, kb, A, lda, B, ldb, partials, nblocks, s);
  if (per_wave <= 4) return launch_gram_t<T, 4, SYM>(n, ka, kb, A, lda, B, ldb, partials, nblocks, s);
  if (per_wave <= 8) return launch_gram_t<T, 8, SYM>(n, ka, kb, A, lda, B, ldb, partials, nblocks, s);
  return launch_gram_t<T, 16, SYM>(n, ka, kb, A, lda, B, ldb, partials, nblocks, s);
}

int gram_blocks(int64_t n) {
  int64_t chunks = (n + kChunk - 1) / kChunk;
  return int(chunks < kGramBlocks ? (chunks > 0 ? chunks : 1) : kGramBlocks);
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

size_t gram_ws_doubles(int64_t n, int64_t ka, int64_t kb) { return size_t(gram_blocks(n)) * ka * kb; }

sped_status launch_gram(int64_t n, int ka, int kb, const void *A, int64_t lda, const void *B, int64_t ldb,
                        int dt, double *G, double *partials, hipStream_t s) {
  if (ka < 1 || kb < 1 || ka > kMaxK || kb > kMaxK) return fail(SPED_E_UNSUPPORTED, "gram width outside [1, 128]");
  const int nb = gram_blocks(n);
  const bool sym = (A == B) && (lda == ldb) && (ka == kb);
  sped_status st;
  if (dt == SPED_F32)
    st = sym ? launch_gram_maxt<float, true>(n, ka, kb, A, lda, B, ldb, partials, nb, s)
             : launch_gram_maxt<float, false>(n, ka, kb, A, lda, B, ldb, partials, nb, s);
  else if (dt == SPED_BF16)
    st = sym ? launch_gram_maxt<bf16_t, true>(n, ka, kb, A, lda, B, ldb, partials, nb, s)
             : launch_gram_maxt<bf16_t, false>(n, ka, kb, A, lda, B, ldb, partials, nb, s);
  else
    return fail(SPED_E_UNSUPPORTED, "gram dtype");
  if (st != SPED_OK) return st;
  int64_t count = int64_t(ka) * kb;
  hipLaunchKernelGGL(sum_partials_kernel, dim3(unsigned((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     partials, nb, count, G);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
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

size_t resid_ws_doubles(int64_t k) { return size_t(kResidBlocks) * k; }

sped_status launch_resid(int64_t n, int k, const float *Z, int64_t ldz, const float *Q, int64_t ldq,
                         const double *theta, double *resid, double *partials, hipStream_t s) {
  if (k > kBlock) return fail(SPED_E_UNSUPPORTED, "resid width > 256");
  hipLaunchKernelGGL(resid_kernel, dim3(kResidBlocks), dim3(kBlock), 0, s, n, k, Z, ldz, Q, ldq, theta, partials);
  SPED_CHECK_HIP(hipGetLastError());
  hipLaunchKernelGGL(sqrt_sum_kernel, dim3(1), dim3(kBlock), 0, s, partials, kResidBlocks, k, resid);
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
  return launch_gram(n, int(ka), int(kb), A, lda, B, ldb, dt, G, partials, as_stream(stream));
}
