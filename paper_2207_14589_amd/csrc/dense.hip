// Small dense float64 factorisations for the block solver, each on one
// workgroup with the matrix in LDS (k <= 96):
//   chol_inv  G = R^T R (Cholesky, upper R) and T = R^{-1} in one sweep; on a pivot
//             breakdown G is shifted by s I, s = 1e-12 trace(G) growing x100
//             per retry (shifted Cholesky QR), counted in flags[0];
//   jacobi    H = S diag(theta) S^T by cyclic two-sided Jacobi with the
//             round-robin (circle) ordering: the k/2 rotations of a round act
//             on disjoint index pairs and are applied together as 2x2 block
//             updates; eigenvalues sorted ascending.
#include <cmath>

#include "common.h"

namespace sped {
namespace {

constexpr int kBlock = 1024;
constexpr int kMaxDense = 96;

// Cholesky G = R^T R, upper R, right-looking, with the inverse formed in the
// same sweep: the row operations that reduce G to R (subtract f_r times pivot
// row j from each row r > j, f_r = A_jr / A_jj, then scale row j by
// 1 / sqrt(A_jj)) applied to the identity give M = R^{-T}, so T = R^{-1} = M^T
// needs no back substitution.  Step j reads the pivot (every thread, so the
// breakdown test is uniform), keeps 1 / sqrt(pivot) in LDS, and updates the
// trailing upper triangle of A and rows r > j of M (columns c <= j; M is
// lower triangular); rows j of A and M are only read in step j, so one
// barrier per step suffices.  Rows j of A and M are final after step j, so R
// and T are written once, after the last step: no global store is pending at
// the barriers (14 columns: 12.4 -> 11.3 us).  Threads form a 32 x 32 grid over
// (row, column) offsets.
__global__ __launch_bounds__(kBlock) void chol_inv_kernel(int k, const double *__restrict__ G,
                                                          double *__restrict__ T, double *__restrict__ R_out,
                                                          int *__restrict__ flags) {
  extern __shared__ double sm[];
  double *A = sm;              // k x k working copy (upper triangle used)
  double *M = sm + k * k;      // R^{-T}, built row by row
  double *inv = sm + 2 * k * k;  // 1 / sqrt(pivot j); 0 for steps not reached
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  double trace = 0.0;
  for (int i = 0; i < k; ++i) trace += G[i * k + i];
  double shift = 0.0;
  bool broke = true;
  for (int attempt = 0; attempt < 6 && broke; ++attempt) {
    if (attempt > 0) {
      shift = (shift == 0.0 ? 1e-12 * (trace > 0 ? trace : 1.0) : shift * 100.0);
      if (threadIdx.x == 0) atomicAdd(flags, 1);
    }
    for (int i = threadIdx.x; i < k * k; i += kBlock) {
      const int r = i / k, c = i - r * k;
      A[i] = 0.5 * (G[r * k + c] + G[c * k + r]) + (r == c ? shift : 0.0);
      M[i] = (r == c) ? 1.0 : 0.0;
    }
    for (int i = threadIdx.x; i < k; i += kBlock) inv[i] = 0.0;
    __syncthreads();
    broke = false;
    for (int j = 0; j < k; ++j) {
      const double piv = A[j * k + j];
      if (!(piv > 1e-300) || !isfinite(piv)) {
        broke = true;
        break;
      }
      if (threadIdx.x == 0) inv[j] = 1.0 / sqrt(piv);
      for (int r = j + 1 + ty; r < k; r += 32) {
        const double f = A[j * k + r] / piv;
        for (int c = r + tx; c < k; c += 32) A[r * k + c] -= f * A[j * k + c];
        for (int c = tx; c <= j; c += 32) M[r * k + c] -= f * M[j * k + c];
      }
      __syncthreads();
    }
    __syncthreads();
  }
  // row j of R and column j of T from the final rows j of A and M
  for (int i = threadIdx.x; i < k * k; i += kBlock) {
    const int j = i / k, c = i - j * k;
    T[c * k + j] = M[j * k + c] * inv[j];
    if (R_out) R_out[j * k + c] = c >= j ? A[j * k + c] * inv[j] : 0.0;
  }
  if (broke && threadIdx.x == 0) atomicAdd(flags + 1, 1);
}

__device__ inline int rr_player(int pos, int round, int m) {
  if (pos == 0) return 0;
  int x = pos - 1 + round;
  if (x >= m - 1) x -= m - 1;
  return x + 1;
}

constexpr int kMaxPairs = kMaxDense / 2;
constexpr int kBlkItems = (kMaxPairs * kMaxPairs + kBlock - 1) / kBlock;   // 2x2 blocks per thread
constexpr int kVItems = (kMaxDense * kMaxPairs + kBlock - 1) / kBlock;     // V row pairs per thread

// Cyclic two-sided Jacobi on the m x m matrix (m = k rounded up to even; an
// odd k gets a zero row and column that no rotation ever touches).  A round's
// m/2 rotations act on disjoint index pairs (circle ordering); once they are
// known, A <- J^T A J is applied as independent 2x2 block updates (block
// (q1, q2) couples pairs q1 and q2; the diagonal blocks are set to their exact
// rotated form, off-diagonal entry zero) together with V <- V J, so a round
// costs two barriers.  Sweeps stop when the off-diagonal mass is below
// 1e-24 of the total (off-diagonal norm 1e-12 relative).  Eigenvalues are
// ranked ascending in parallel (ties by index).
__global__ __launch_bounds__(kBlock) void jacobi_kernel(int k, const double *__restrict__ H,
                                                        double *__restrict__ theta, double *__restrict__ S,
                                                        int *__restrict__ flags, double rel,
                                                        const double *__restrict__ rel_dev) {
  // stopping point: from device memory when given (set by a kernel launched
  // before this one, so a captured graph can reuse this launch)
  const double rel_used = rel_dev ? *rel_dev : rel;
  const double rel2 = rel_used * rel_used;
  // LDS rows are padded to ld = m + 1 doubles so that walking down a column
  // touches different banks.
  extern __shared__ double sm[];
  const int m = k + (k & 1);
  const int ld = m + 1;
  double *A = sm;
  double *V = sm + m * ld;
  __shared__ double cs[kMaxPairs][3];
  __shared__ int pp[kMaxPairs][2];
  __shared__ double red[2][kBlock / 64];
  __shared__ int perm[kMaxDense];
  const int npairs = m / 2;
  for (int i = threadIdx.x; i < m * m; i += kBlock) {
    const int r = i / m, c = i - r * m;
    A[r * ld + c] = (r < k && c < k) ? 0.5 * (H[r * k + c] + H[c * k + r]) : 0.0;
    V[r * ld + c] = (r == c) ? 1.0 : 0.0;
  }
  // this thread's 2x2 blocks and V row pairs (the same every round)
  int bq1[kBlkItems], bq2[kBlkItems], vq[kVItems], vrow[kVItems];
#pragma unroll
  for (int t = 0; t < kBlkItems; ++t) {
    const int i = threadIdx.x + t * kBlock;
    bq1[t] = i < npairs * npairs ? i / npairs : -1;
    bq2[t] = i < npairs * npairs ? i - (i / npairs) * npairs : -1;
  }
#pragma unroll
  for (int t = 0; t < kVItems; ++t) {
    const int i = threadIdx.x + t * kBlock;
    vq[t] = i < npairs * m ? i / m : -1;
    vrow[t] = i < npairs * m ? i - (i / m) * m : -1;
  }
  __syncthreads();
  int sweep = 0;
  for (; sweep < 60 && k > 1; ++sweep) {
    // squared norms of the off-diagonal part and of the whole matrix
    double o = 0.0, t2 = 0.0;
    for (int i = threadIdx.x; i < m * m; i += kBlock) {
      const int r = i / m, c = i - r * m;
      const double x = A[r * ld + c];
      t2 += x * x;
      if (r != c) o += x * x;
    }
    for (int off = 32; off > 0; off >>= 1) {
      o += __shfl_xor(o, off, 64);
      t2 += __shfl_xor(t2, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = o;
      red[1][threadIdx.x >> 6] = t2;
    }
    __syncthreads();
    double off2 = 0.0, tot2 = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      off2 += red[0][w];
      tot2 += red[1][w];
    }
    __syncthreads();  // red is rewritten next sweep
    if (!(off2 > rel2 * tot2) || !(tot2 > 0.0)) break;
    for (int round = 0; round < m - 1; ++round) {
      if (threadIdx.x < npairs) {
        const int q = threadIdx.x;
        const int a = rr_player(q, round, m), b = rr_player(m - 1 - q, round, m);
        const int p = a < b ? a : b, r = a < b ? b : a;
        double c = 1.0, s = 0.0, t = 0.0;
        const double apq = A[p * ld + r];
        if (apq != 0.0) {
          const double tau = (A[r * ld + r] - A[p * ld + p]) / (2.0 * apq);
          t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        pp[q][0] = p;
        pp[q][1] = r;
        cs[q][0] = c;
        cs[q][1] = s;
        cs[q][2] = t;
      }
      __syncthreads();
#pragma unroll
      for (int it = 0; it < kBlkItems; ++it) {
        const int q1 = bq1[it], q2 = bq2[it];
        if (q1 < 0) continue;
        const int p1 = pp[q1][0], r1 = pp[q1][1], p2 = pp[q2][0], r2 = pp[q2][1];
        if (q1 == q2) {
          const double t = cs[q1][2], apr = A[p1 * ld + r1];
          A[p1 * ld + p1] -= t * apr;
          A[r1 * ld + r1] += t * apr;
          A[p1 * ld + r1] = 0.0;
          A[r1 * ld + p1] = 0.0;
        } else {
          const double c1 = cs[q1][0], s1 = cs[q1][1], c2 = cs[q2][0], s2 = cs[q2][1];
          const double app = A[p1 * ld + p2], apr = A[p1 * ld + r2];
          const double arp = A[r1 * ld + p2], arr = A[r1 * ld + r2];
          // columns (pair q2), then rows (pair q1)
          const double xpp = c2 * app - s2 * apr, xpr = s2 * app + c2 * apr;
          const double xrp = c2 * arp - s2 * arr, xrr = s2 * arp + c2 * arr;
          A[p1 * ld + p2] = c1 * xpp - s1 * xrp;
          A[r1 * ld + p2] = s1 * xpp + c1 * xrp;
          A[p1 * ld + r2] = c1 * xpr - s1 * xrr;
          A[r1 * ld + r2] = s1 * xpr + c1 * xrr;
        }
      }
#pragma unroll
      for (int it = 0; it < kVItems; ++it) {
        const int q = vq[it], row = vrow[it];
        if (q < 0) continue;
        const int p = pp[q][0], r = pp[q][1];
        const double c = cs[q][0], s = cs[q][1];
        const double vp = V[row * ld + p], vr = V[row * ld + r];
        V[row * ld + p] = c * vp - s * vr;
        V[row * ld + r] = s * vp + c * vr;
      }
      __syncthreads();
    }
  }
  // ascending rank of each eigenvalue (ties by index)
  for (int i = threadIdx.x; i < k; i += kBlock) {
    const double di = A[i * ld + i];
    int rank = 0;
    for (int j = 0; j < k; ++j) {
      const double dj = A[j * ld + j];
      rank += (dj < di || (dj == di && j < i)) ? 1 : 0;
    }
    perm[rank] = i;
  }
  if (threadIdx.x == 0 && sweep >= 60) atomicAdd(flags + 2, 1);
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += kBlock) theta[i] = A[perm[i] * ld + perm[i]];
  for (int i = threadIdx.x; i < k * k; i += kBlock) {
    const int r = i / k, c = i - r * k;
    S[i] = V[r * ld + perm[c]];
  }
}

}  // namespace

int dense_max_k() { return kMaxDense; }

sped_status launch_chol_inv(int k, const double *G, double *T, double *R_out, int *flags, hipStream_t s) {
  if (k < 1 || k > kMaxDense) return fail(SPED_E_UNSUPPORTED, "dense width outside [1, 96]");
  size_t shm = (size_t(2) * k * k + k) * sizeof(double);
  SPED_TRY(set_max_lds(chol_inv_kernel, shm));
  hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(kBlock), shm, s, k, G, T, R_out, flags);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

sped_status launch_jacobi(int k, const double *H, double *theta, double *S, int *flags, hipStream_t s,
                          double rel, const double *rel_dev) {
  if (k < 1 || k > kMaxDense) return fail(SPED_E_UNSUPPORTED, "dense width outside [1, 96]");
  const int m = k + (k & 1);
  size_t shm = size_t(2) * m * (m + 1) * sizeof(double);
  SPED_TRY(set_max_lds(jacobi_kernel, shm));
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(kBlock), shm, s, k, H, theta, S, flags, rel, rel_dev);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

}  // namespace sped
