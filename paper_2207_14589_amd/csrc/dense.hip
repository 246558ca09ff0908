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
  extern __shared__ double sm[];
  double *A = sm;
  double *V = sm + k * k;
  __shared__ double cs[kMaxDense / 2 + 1][2];
  __shared__ int pp[kMaxDense / 2 + 1][2];
  __shared__ double off2, tot2;
  __shared__ int perm[kMaxDense];
  const int m = k + (k & 1);  // players, with a bye when k is odd
  for (int i = threadIdx.x; i < k * k; i += kBlock) {
    int r = i / k, c = i - r * k;
    A[i] = 0.5 * (H[r * k + c] + H[c * k + r]);
    V[i] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < k * k; ++i) t += A[i] * A[i];
    tot2 = t;
  }
  __syncthreads();
  int sweep = 0;
  for (; sweep < 60 && k > 1; ++sweep) {
    if (threadIdx.x == 0) {
      double o = 0.0;
      for (int r = 0; r < k; ++r)
        for (int c = r + 1; c < k; ++c) o += 2.0 * A[r * k + c] * A[r * k + c];
      off2 = o;
    }
    __syncthreads();
    if (!(off2 > 1e-30 * tot2) || !(tot2 > 0.0)) break;
    for (int round = 0; round < m - 1; ++round) {
      const int npairs = m / 2;
      for (int q = threadIdx.x; q < npairs; q += kBlock) {
        int a = rr_player(q, round, m), b = rr_player(m - 1 - q, round, m);
        int p = a < b ? a : b, r = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (r < k) {
          double apq = A[p * k + r];
          if (apq != 0.0) {
            double tau = (A[r * k + r] - A[p * k + p]) / (2.0 * apq);
            double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        pp[q][0] = p;
        pp[q][1] = r < k ? r : -1;
        cs[q][0] = c;
        cs[q][1] = s;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int i = threadIdx.x; i < k * npairs; i += kBlock) {
        int row = i / npairs, q = i - row * npairs;
        int p = pp[q][0], r = pp[q][1];
        if (r < 0) continue;
        double c = cs[q][0], s = cs[q][1];
        double ap = A[row * k + p], ar = A[row * k + r];
        A[row * k + p] = c * ap - s * ar;
        A[row * k + r] = s * ap + c * ar;
        double vp = V[row * k + p], vr = V[row * k + r];
        V[row * k + p] = c * vp - s * vr;
        V[row * k + r] = s * vp + c * vr;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int i = threadIdx.x; i < k * npairs; i += kBlock) {
        int col = i / npairs, q = i - col * npairs;
        int p = pp[q][0], r = pp[q][1];
        if (r < 0) continue;
        double c = cs[q][0], s = cs[q][1];
        double ap = A[p * k + col], ar = A[r * k + col];
        A[p * k + col] = c * ap - s * ar;
        A[r * k + col] = s * ap + c * ar;
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    for (int i = 0; i < k; ++i) perm[i] = i;
    for (int i = 0; i < k; ++i) {
      int best = i;
      for (int j = i + 1; j < k; ++j)
        if (A[perm[j] * k + perm[j]] < A[perm[best] * k + perm[best]]) best = j;
      int t = perm[i];
      perm[i] = perm[best];
      perm[best] = t;
    }
    if (sweep >= 60) atomicAdd(flags + 2, 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += kBlock) theta[i] = A[perm[i] * k + perm[i]];
  for (int i = threadIdx.x; i < k * k; i += kBlock) {
    int r = i / k, c = i - r * k;
    S[i] = V[r * k + perm[c]];
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
  size_t shm = size_t(2) * k * k * sizeof(double);
  SPED_TRY(set_max_lds(jacobi_kernel, shm));
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(kBlock), shm, s, k, H, theta, S, flags);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

}  // namespace sped
