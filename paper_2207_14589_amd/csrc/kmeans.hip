// k-means on the spectral embedding (Sec. 1: the bottom-k eigenvectors embed
// the nodes and k-means yields the hard clusters; Sec. 2.1: k = 2 on the
// Fiedler vector).  Float64 throughout: rows are converted (and optionally
// scaled to unit length) once; k-means++ seeding draws Philox uniforms; Lloyd
// rounds alternate centroid means and nearest-centre assignment (ties go to
// the lower centre index) until no label changes.
#include <hipcub/hipcub.hpp>

#include <cmath>

#include "common.h"

namespace sped {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxClusters = 256;
constexpr int kMaxK = 128;

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > 65536) b = 65536;
  return unsigned(b > 0 ? b : 1);
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < (n); i += int64_t(gridDim.x) * kBlock)

template <typename T>
__global__ void to_double_rows(int64_t n, int k, const T *__restrict__ V, int64_t ldv, int normalize,
                               double *__restrict__ X) {
  GRID_STRIDE(r, n) {
    double nrm = 0.0;
    for (int c = 0; c < k; ++c) {
      double x = double(to_f32<T>(V[r * ldv + c]));
      X[r * k + c] = x;
      nrm += x * x;
    }
    if (normalize) {
      double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
      for (int c = 0; c < k; ++c) X[r * k + c] = nrm > 0.0 ? X[r * k + c] * inv : 0.0;
    }
  }
}

__global__ void fill_double(int64_t n, double *p, double v) {
  GRID_STRIDE(i, n) p[i] = v;
}

// d2[i] = min(d2[i], ||X_i - C_c||^2)
__global__ void update_mind2(int64_t n, int k, const double *__restrict__ X, const double *__restrict__ C, int c,
                             double *__restrict__ d2) {
  GRID_STRIDE(i, n) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) {
      double d = X[i * k + j] - C[c * k + j];
      s += d * d;
    }
    if (s < d2[i]) d2[i] = s;
  }
}

// choose the first index whose inclusive prefix exceeds u * total; copy it to C[c]
__global__ void pick_center(int64_t n, int k, const double *__restrict__ X, const double *__restrict__ prefix,
                            uint32_t k0, uint32_t k1, int c, double *__restrict__ C) {
  __shared__ int64_t idx;
  if (threadIdx.x == 0) {
    double u = uniform53(k0, k1, uint32_t(c), 0u, 0u, 0u);
    double total = prefix ? prefix[n - 1] : 0.0;
    int64_t pick;
    if (!(total > 0.0)) {
      pick = int64_t(u * double(n));
    } else {
      double target = u * total;
      int64_t lo = 0, hi = n - 1;
      while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (prefix[mid] > target) hi = mid;
        else lo = mid + 1;
      }
      pick = lo;
    }
    idx = pick < n ? pick : n - 1;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += kBlock) C[c * k + j] = X[idx * k + j];
}

__global__ void assign_kernel(int64_t n, int k, int nc, const double *__restrict__ X, const double *__restrict__ C,
                              int32_t *__restrict__ labels, double *__restrict__ d2, int *__restrict__ changed) {
  extern __shared__ double sC[];
  for (int i = threadIdx.x; i < nc * k; i += kBlock) sC[i] = C[i];
  __syncthreads();
  GRID_STRIDE(i, n) {
    double best = INFINITY;
    int bi = 0;
    for (int c = 0; c < nc; ++c) {
      double s = 0.0;
      for (int j = 0; j < k; ++j) {
        double d = X[i * k + j] - sC[c * k + j];
        s += d * d;
      }
      if (s < best) {
        best = s;
        bi = c;
      }
    }
    if (labels[i] != bi) {
      labels[i] = bi;
      atomicOr(changed, 1);
    }
    d2[i] = best;
  }
}

__global__ void accumulate_kernel(int64_t n, int k, const double *__restrict__ X, const int32_t *__restrict__ labels,
                                  double *__restrict__ sums, unsigned long long *__restrict__ counts) {
  GRID_STRIDE(i, n) {
    int c = labels[i];
    atomicAdd(&counts[c], 1ull);
    for (int j = 0; j < k; ++j) atomicAdd(&sums[c * k + j], X[i * k + j]);
  }
}

__global__ void update_centroids(int nc, int k, const double *__restrict__ sums,
                                 const unsigned long long *__restrict__ counts, double *__restrict__ C) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nc * k) return;
  int c = i / k;
  if (counts[c] > 0) C[i] = sums[i] / double(counts[c]);
}

__global__ void zero_kernel(int64_t n, unsigned long long *p) {
  GRID_STRIDE(i, n) p[i] = 0ull;
}

__global__ void neg_labels(int64_t n, int32_t *labels) {
  GRID_STRIDE(i, n) labels[i] = -1;
}

}  // namespace
}  // namespace sped

using namespace sped;

extern "C" sped_status sped_cluster_embed(const void *V, int64_t n, int64_t k, int64_t ldv, int32_t vdt,
                                          int32_t n_clusters, int32_t row_normalize, uint64_t seed, int32_t max_iters,
                                          const double *init, int32_t *labels, double *centroids, double *inertia,
                                          int32_t *iters, void *ws, size_t *ws_bytes, sped_stream_t stream) {
  clear_error();
  if (n < 1 || k < 1 || k > kMaxK) return fail(SPED_E_INVALID, "cluster shape (k in [1, 128])");
  if (n_clusters < 1 || n_clusters > kMaxClusters || n_clusters > n)
    return fail(SPED_E_INVALID, "n_clusters outside [1, min(256, n)]");
  if (ldv < k) return fail(SPED_E_INVALID, "ldv < k");
  if (vdt != SPED_F32 && vdt != SPED_BF16) return fail(SPED_E_UNSUPPORTED, "dtype");
  if (!V || !labels || !centroids) return fail(SPED_E_INVALID, "NULL pointer");
  if (max_iters < 0) return fail(SPED_E_INVALID, "max_iters < 0");
  if (int64_t(n_clusters) * k > 16384) return fail(SPED_E_UNSUPPORTED, "n_clusters * k > 16384");
  const int nc = n_clusters;
  Carver cv(ws);
  double *X = cv.take<double>(size_t(n) * k);
  double *d2 = cv.take<double>(size_t(n));
  double *prefix = cv.take<double>(size_t(n));
  double *sums = cv.take<double>(size_t(nc) * k);
  unsigned long long *counts = cv.take<unsigned long long>(nc);
  int *changed = cv.take<int>(1);
  size_t scan_bytes = 0, red_bytes = 0;
  hipcub::DeviceScan::InclusiveSum(nullptr, scan_bytes, (double *)nullptr, (double *)nullptr, n);
  hipcub::DeviceReduce::Sum(nullptr, red_bytes, (double *)nullptr, (double *)nullptr, n);
  size_t tbytes = scan_bytes > red_bytes ? scan_bytes : red_bytes;
  void *temp = cv.take<char>(tbytes);
  double *dsum = cv.take<double>(1);
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, cv.bytes(), &query));
  if (query) return SPED_OK;
  hipStream_t s = as_stream(stream);
  if (vdt == SPED_F32)
    hipLaunchKernelGGL(to_double_rows<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, int(k),
                       static_cast<const float *>(V), ldv, row_normalize, X);
  else
    hipLaunchKernelGGL(to_double_rows<bf16_t>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, int(k),
                       static_cast<const bf16_t *>(V), ldv, row_normalize, X);
  SPED_CHECK_HIP(hipGetLastError());
  const uint32_t k0 = uint32_t(seed & 0xffffffffu), k1 = uint32_t(seed >> 32);
  if (init) {
    SPED_CHECK_HIP(hipMemcpyAsync(centroids, init, sizeof(double) * nc * k, hipMemcpyDeviceToDevice, s));
  } else {
    hipLaunchKernelGGL(pick_center, dim3(1), dim3(kBlock), 0, s, n, int(k), X, (const double *)nullptr, k0, k1, 0,
                       centroids);
    hipLaunchKernelGGL(fill_double, dim3(grid_for(n)), dim3(kBlock), 0, s, n, d2, INFINITY);
    SPED_CHECK_HIP(hipGetLastError());
    for (int c = 1; c < nc; ++c) {
      hipLaunchKernelGGL(update_mind2, dim3(grid_for(n)), dim3(kBlock), 0, s, n, int(k), X, centroids, c - 1, d2);
      size_t tb = tbytes;
      SPED_CHECK_HIP(hipcub::DeviceScan::InclusiveSum(temp, tb, d2, prefix, n, s));
      hipLaunchKernelGGL(pick_center, dim3(1), dim3(kBlock), 0, s, n, int(k), X, prefix, k0, k1, c, centroids);
      SPED_CHECK_HIP(hipGetLastError());
    }
  }
  const size_t shm = size_t(nc) * k * sizeof(double);
  SPED_TRY(set_max_lds(assign_kernel, shm));
  hipLaunchKernelGGL(neg_labels, dim3(grid_for(n)), dim3(kBlock), 0, s, n, labels);
  int hchanged = 0;
  SPED_CHECK_HIP(hipMemsetAsync(changed, 0, sizeof(int), s));
  hipLaunchKernelGGL(assign_kernel, dim3(grid_for(n)), dim3(kBlock), shm, s, n, int(k), nc, X, centroids, labels, d2,
                     changed);
  SPED_CHECK_HIP(hipGetLastError());
  int it = 0;
  for (it = 1; it <= max_iters; ++it) {
    hipLaunchKernelGGL(fill_double, dim3(grid_for(int64_t(nc) * k)), dim3(kBlock), 0, s, int64_t(nc) * k, sums, 0.0);
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(kBlock), 0, s, int64_t(nc), counts);
    hipLaunchKernelGGL(accumulate_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, int(k), X, labels, sums, counts);
    hipLaunchKernelGGL(update_centroids, dim3(unsigned((nc * k + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, nc,
                       int(k), sums, counts, centroids);
    SPED_CHECK_HIP(hipMemsetAsync(changed, 0, sizeof(int), s));
    hipLaunchKernelGGL(assign_kernel, dim3(grid_for(n)), dim3(kBlock), shm, s, n, int(k), nc, X, centroids, labels,
                       d2, changed);
    SPED_CHECK_HIP(hipGetLastError());
    SPED_CHECK_HIP(hipMemcpyAsync(&hchanged, changed, sizeof(int), hipMemcpyDeviceToHost, s));
    SPED_CHECK_HIP(hipStreamSynchronize(s));
    if (!hchanged) break;
  }
  if (it > max_iters) it = max_iters;
  size_t tb = tbytes;
  SPED_CHECK_HIP(hipcub::DeviceReduce::Sum(temp, tb, d2, dsum, n, s));
  double hin = 0.0;
  SPED_CHECK_HIP(hipMemcpyAsync(&hin, dsum, sizeof(double), hipMemcpyDeviceToHost, s));
  SPED_CHECK_HIP(hipStreamSynchronize(s));
  if (inertia) *inertia = hin;
  if (iters) *iters = it;
  return SPED_OK;
}
