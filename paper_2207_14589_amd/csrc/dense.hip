// Small dense float64 factorisations for the block solver, each on one
// workgroup with the matrix in LDS (k <= 96):
//   chol_inv  G = R^T R (Cholesky, upper R) and T = R^{-1}; on a pivot
//             breakdown G is shifted by s I, s = 1e-12 trace(G) growing x100
//             per retry (shifted Cholesky QR), counted in flags[0];
//   jacobi    H = S diag(theta) S^T by cyclic two-sided Jacobi with the
//             round-robin (circle) ordering: the k/2 rotations of a round act
//             on disjoint index pairs and are applied together, first to the
//             columns and then to the rows; eigenvalues sorted ascending.
#include <cmath>

#include "common.h"

namespace sped {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxDense = 96;

__global__ __launch_bounds__(kBlock) void chol_inv_kernel(int k, const double *__restrict__ G,
                                                          double *__restrict__ T, double *__restrict__ R_out,
                                                          int *__restrict__ flags) {
  extern __shared__ double sm[];
  double *A = sm;          // k x k working copy, upper triangle becomes R
  double *Rinv = sm + k * k;
  __shared__ double shift;
  __shared__ int broke;
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int i = 0; i < k; ++i) tr += G[i * k + i];
    shift = 0.0;
    broke = 0;
    Rinv[0] = tr;  // scratch: trace
  }
  __syncthreads();
  const double trace = Rinv[0];
  for (int attempt = 0; attempt < 6; ++attempt) {
    for (int i = threadIdx.x; i < k * k; i += kBlock) {
      int r = i / k, c = i - r * k;
      double g = 0.5 * (G[r * k + c] + G[c * k + r]);
      A[i] = g + (r == c ? shift : 0.0);
    }
    __syncthreads();
    for (int j = 0; j < k; ++j) {
      if (threadIdx.x == 0) {
        double piv = A[j * k + j];
        if (!(piv > 1e-300) || !isfinite(piv)) {
          broke = 1;
        } else {
          A[j * k + j] = sqrt(piv);
        }
      }
      __syncthreads();
      if (broke) break;
      const double rjj = A[j * k + j];
      for (int c = j + 1 + threadIdx.x; c < k; c += kBlock) A[j * k + c] /= rjj;
      __syncthreads();
      const int m = k - j - 1;
      for (int i = threadIdx.x; i < m * m; i += kBlock) {
        int r = j + 1 + i / m, c = j + 1 + i % m;
        if (c >= r) A[r * k + c] -= A[j * k + r] * A[j * k + c];
      }
      __syncthreads();
    }
    if (!broke) break;
    __syncthreads();
    if (threadIdx.x == 0) {
      shift = (shift == 0.0 ? 1e-12 * (trace > 0 ? trace : 1.0) : shift * 100.0);
      broke = 0;
      atomicAdd(flags, 1);
    }
    __syncthreads();
  }
  if (broke) {
    if (threadIdx.x == 0) atomicAdd(flags + 1, 1);
    return;
  }
  // T = R^{-1}: column c solves R t = e_c by back substitution (one thread per column)
  for (int c = threadIdx.x; c < k; c += kBlock) {
    for (int i = k - 1; i >= 0; --i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int j = i + 1; j <= c; ++j) s -= A[i * k + j] * Rinv[j * k + c];
      Rinv[i * k + c] = (i <= c) ? s / A[i * k + i] : 0.0;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k * k; i += kBlock) {
    int r = i / k, c = i - r * k;
    T[i] = Rinv[i];
    if (R_out) R_out[i] = (c >= r) ? A[i] : 0.0;
  }
}

__device__ inline int rr_player(int pos, int round, int m) {
  return pos == 0 ? 0 : ((pos - 1 + round) % (m - 1)) + 1;
}

__global__ __launch_bounds__(kBlock) void jacobi_kernel(int k, const double *__restrict__ H,
                                                        double *__restrict__ theta, double *__restrict__ S,
                                                        int *__restrict__ flags) {
  // LDS rows are padded to ld = k + 1 doubles so that walking down a column
  // (the column half of a rotation) touches different banks.
  extern __shared__ double sm[];
  const int ld = k + 1;
  double *A = sm;
  double *V = sm + k * ld;
  __shared__ double cs[kMaxDense / 2 + 1][2];
  __shared__ int pp[kMaxDense / 2 + 1][2];
  __shared__ double red[kBlock / 64];
  __shared__ double off2, tot2;
  __shared__ int perm[kMaxDense];
  const int m = k + (k & 1);  // players, with a bye when k is odd
  const int npairs = m / 2;
  for (int i = threadIdx.x; i < k * k; i += kBlock) {
    int r = i / k, c = i - r * k;
    A[r * ld + c] = 0.5 * (H[r * k + c] + H[c * k + r]);
    V[r * ld + c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  int sweep = 0;
  for (; sweep < 60 && k > 1; ++sweep) {
    // squared norms of the off-diagonal part and of the whole matrix
    double o = 0.0, t = 0.0;
    for (int i = threadIdx.x; i < k * k; i += kBlock) {
      int r = i / k, c = i - r * k;
      double x = A[r * ld + c];
      t += x * x;
      if (r != c) o += x * x;
    }
    for (int off = 32; off > 0; off >>= 1) {
      o += __shfl_xor(o, off, 64);
      t += __shfl_xor(t, off, 64);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = o;
    __syncthreads();
    if (threadIdx.x == 0) {
      off2 = red[0] + red[1] + red[2] + red[3];
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) tot2 = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    if (!(off2 > 1e-30 * tot2) || !(tot2 > 0.0)) break;
    for (int round = 0; round < m - 1; ++round) {
      for (int q = threadIdx.x; q < npairs; q += kBlock) {
        int a = rr_player(q, round, m), b = rr_player(m - 1 - q, round, m);
        int p = a < b ? a : b, r = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (r < k) {
          double apq = A[p * ld + r];
          if (apq != 0.0) {
            double tau = (A[r * ld + r] - A[p * ld + p]) / (2.0 * apq);
            double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        pp[q][0] = p;
        pp[q][1] = r < k ? r : -1;
        cs[q][0] = c;
        cs[q][1] = s;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J  (consecutive threads walk down a column)
      for (int i = threadIdx.x; i < k * npairs; i += kBlock) {
        int q = i / k, row = i - q * k;
        int p = pp[q][0], r = pp[q][1];
        if (r < 0) continue;
        double c = cs[q][0], s = cs[q][1];
        double ap = A[row * ld + p], ar = A[row * ld + r];
        A[row * ld + p] = c * ap - s * ar;
        A[row * ld + r] = s * ap + c * ar;
        double vp = V[row * ld + p], vr = V[row * ld + r];
        V[row * ld + p] = c * vp - s * vr;
        V[row * ld + r] = s * vp + c * vr;
      }
      __syncthreads();
      // rows: A <- J^T A  (consecutive threads walk along a row)
      for (int i = threadIdx.x; i < k * npairs; i += kBlock) {
        int q = i / k, col = i - q * k;
        int p = pp[q][0], r = pp[q][1];
        if (r < 0) continue;
        double c = cs[q][0], s = cs[q][1];
        double ap = A[p * ld + col], ar = A[r * ld + col];
        A[p * ld + col] = c * ap - s * ar;
        A[r * ld + col] = s * ap + c * ar;
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    for (int i = 0; i < k; ++i) perm[i] = i;
    for (int i = 0; i < k; ++i) {
      int best = i;
      for (int j = i + 1; j < k; ++j)
        if (A[perm[j] * ld + perm[j]] < A[perm[best] * ld + perm[best]]) best = j;
      int t = perm[i];
      perm[i] = perm[best];
      perm[best] = t;
    }
    if (sweep >= 60) atomicAdd(flags + 2, 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += kBlock) theta[i] = A[perm[i] * ld + perm[i]];
  for (int i = threadIdx.x; i < k * k; i += kBlock) {
    int r = i / k, c = i - r * k;
    S[i] = V[r * ld + perm[c]];
  }
}

}  // namespace

int dense_max_k() { return kMaxDense; }

sped_status launch_chol_inv(int k, const double *G, double *T, double *R_out, int *flags, hipStream_t s) {
  if (k < 1 || k > kMaxDense) return fail(SPED_E_UNSUPPORTED, "dense width outside [1, 96]");
  size_t shm = size_t(2) * k * k * sizeof(double);
  SPED_TRY(set_max_lds(chol_inv_kernel, shm));
  hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(kBlock), shm, s, k, G, T, R_out, flags);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

sped_status launch_jacobi(int k, const double *H, double *theta, double *S, int *flags, hipStream_t s) {
  if (k < 1 || k > kMaxDense) return fail(SPED_E_UNSUPPORTED, "dense width outside [1, 96]");
  size_t shm = size_t(2) * k * (k + 1) * sizeof(double);
  SPED_TRY(set_max_lds(jacobi_kernel, shm));
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(kBlock), shm, s, k, H, theta, S, flags);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

}  // namespace sped
