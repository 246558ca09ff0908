// Laplacian products from edge batches, for graphs whose edge list is not
// resident on the device (the edge-minibatch setting of Sec. 3 and the
// conclusion).  L = sum_e x_e x_e^T (Sec. 2; Sec. 4.1 scales x_e by s_i at
// each endpoint), so a batch B of edges adds
//     x_e x_e^T X:  w s_i (s_i X_i - s_j X_j) to row i, -w s_j (s_i X_i - s_j X_j) to row j
// for each e = (i, j, w) in B (self-loops have x_e = 0).  One group of G lanes
// takes an edge (VEC columns per lane, columns beyond 64 VEC tiled over
// blockIdx.y), reads the two endpoint rows once and adds the two updates with
// float atomics (hardware adds in L2): the order in which edges meet in a row
// is not fixed, so results agree with the float64 sum to rounding.
//
// The streamed entry points copy a host edge list in batches into two device
// staging buffers (alternating, on a private copy stream ordered by events),
// so the copy of batch b + 1 overlaps the kernel of batch b.  The minibatch
// solver runs Oja steps (Sec. 5) on such batches: the reversed operator
// lambda I - L from one batch, or the limit polynomial (I - L/l)^l from l
// batches, one per factor, then Cholesky QR.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace sped {
namespace {

constexpr int kBlock = 256;

#define GRID_STRIDE(i, n) \
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < (n); i += int64_t(gridDim.x) * blockDim.x)

// One lane group walks a run of kEdgeRun consecutive edges.  The update of
// the source row is kept in registers while consecutive edges share their
// source and added with atomics once per run of equal sources (an edge list
// sorted by source, the usual layout, then pays about one source flush per
// node instead of one per edge); the destination row gets its atomics per
// edge.  Invalid edges are counted once each (first column tile, lane 0).
constexpr int kEdgeRun = 8;
template <typename TX, int VEC>
__global__ __launch_bounds__(kBlock) void edge_apply_kernel(int64_t m, const int32_t *__restrict__ src,
                                                            const int32_t *__restrict__ dst,
                                                            const float *__restrict__ w,
                                                            const float *__restrict__ scale, int64_t n, int k, int G,
                                                            int lgG, const TX *__restrict__ X, int64_t ldx,
                                                            float *__restrict__ Y, int64_t ldy, float alpha,
                                                            unsigned long long *__restrict__ invalid) {
  const int lig = threadIdx.x & (G - 1);
  const int64_t e0 = (int64_t(blockIdx.x) * (kBlock >> lgG) + (threadIdx.x >> lgG)) * kEdgeRun;
  if (e0 >= m) return;
  const int c0 = blockIdx.y * 64 * VEC + lig * VEC;
  const bool col_ok = c0 < k;
  int32_t cur = -1;  // source row held in acc (uniform over the lane group)
  float cur_s = 0.f, xc[VEC], acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = xc[v] = 0.f;
  auto flush = [&]() {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      unsafeAtomicAdd(Y + int64_t(cur) * ldy + c0 + v, acc[v]);
      acc[v] = 0.f;
    }
  };
  for (int r = 0; r < kEdgeRun; ++r) {
    const int64_t e = e0 + r;
    if (e >= m) break;
    const int32_t i = src[e], j = dst[e];
    const float wt = w ? w[e] : 1.f;
    if (i < 0 || i >= n || j < 0 || j >= n || !(wt > 0.f) || !isfinite(wt)) {
      if (lig == 0 && blockIdx.y == 0 && invalid) atomicAdd(invalid, 1ull);
      continue;
    }
    if (i == j || !col_ok) continue;
    if (i != cur) {
      if (cur >= 0) flush();
      cur = i;
      cur_s = scale ? scale[i] : 1.f;
      VecIO<TX, VEC>::load(X + int64_t(i) * ldx + c0, xc);
    }
    const float sj = scale ? scale[j] : 1.f;
    float xj[VEC];
    VecIO<TX, VEC>::load(X + int64_t(j) * ldx + c0, xj);
    const float fi = alpha * wt * cur_s, fj = -alpha * wt * sj;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const float d = cur_s * xc[v] - sj * xj[v];
      acc[v] = fmaf(fi, d, acc[v]);
      unsafeAtomicAdd(Y + int64_t(j) * ldy + c0 + v, fj * d);
    }
  }
  if (cur >= 0) flush();
}

// d_i += w for both endpoints of every non-loop edge (float64 atomics).  Each
// thread walks a run of kEdgeRun consecutive edges and adds a source's
// weights once per run of equal sources, as the product does.
__global__ __launch_bounds__(kBlock) void edge_degree_kernel(int64_t m, const int32_t *__restrict__ src,
                                                             const int32_t *__restrict__ dst,
                                                             const float *__restrict__ w, int64_t n,
                                                             double *__restrict__ degree,
                                                             unsigned long long *__restrict__ invalid) {
  const int64_t runs = (m + kEdgeRun - 1) / kEdgeRun;
  GRID_STRIDE(run, runs) {
    int32_t cur = -1;
    double acc = 0.0;
    for (int r = 0; r < kEdgeRun; ++r) {
      const int64_t e = run * kEdgeRun + r;
      if (e >= m) break;
      const int32_t i = src[e], j = dst[e];
      const float wt = w ? w[e] : 1.f;
      if (i < 0 || i >= n || j < 0 || j >= n || !(wt > 0.f) || !isfinite(wt)) {
        atomicAdd(invalid, 1ull);
        continue;
      }
      if (i == j) continue;
      if (i != cur) {
        if (cur >= 0) unsafeAtomicAdd(degree + cur, acc);
        cur = i;
        acc = 0.0;
      }
      acc += double(wt);
      unsafeAtomicAdd(degree + j, double(wt));
    }
    if (cur >= 0) unsafeAtomicAdd(degree + cur, acc);
  }
}

__global__ void node_scale_kernel(int64_t n, int kind, const double *__restrict__ degree, float *__restrict__ scale) {
  GRID_STRIDE(i, n) {
    const double d = degree[i];
    scale[i] = kind == SPED_LAP_COMBINATORIAL ? 1.f : (d > 0.0 ? float(1.0 / sqrt(d)) : 0.f);
  }
}

__global__ void fill_f32_kernel(int64_t n, int k, float *__restrict__ Y, int64_t ldy) {
  GRID_STRIDE(t, n * k) {
    const int64_t r = t / k;
    Y[r * ldy + (t - r * k)] = 0.f;
  }
}

__global__ void fill_f64_kernel(int64_t n, double *__restrict__ p) {
  GRID_STRIDE(t, n) p[t] = 0.0;
}

__global__ void zero_u64_kernel(unsigned long long *p) { *p = 0ull; }

// out = a in (n x k blocks)
__global__ void scale_copy_kernel(int64_t n, int k, const float *__restrict__ in, int64_t ldi, float *__restrict__ out,
                                  int64_t ldo, float a) {
  GRID_STRIDE(t, n * k) {
    const int64_t r = t / k, c = t - r * k;
    out[r * ldo + c] = a * in[r * ldi + c];
  }
}

// V += eta W (n x k blocks)
__global__ void axpy_block_kernel(int64_t n, int k, float *__restrict__ V, int64_t ldv, const float *__restrict__ W,
                                  int64_t ldw, float eta) {
  GRID_STRIDE(t, n * k) {
    const int64_t r = t / k, c = t - r * k;
    V[r * ldv + c] += eta * W[r * ldw + c];
  }
}

unsigned grid_blocks(int64_t work) {
  int64_t b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return unsigned(b);
}

struct EdgeGeom {
  int vec, G, lgG, ytiles;
};

EdgeGeom edge_geom(int64_t k, const void *X, int64_t ldx, int xdt, const float *Y, int64_t ldy) {
  EdgeGeom g;
  g.vec = pick_vec(k, {ldx, ldy}, {X, Y}, {int(dtype_size(xdt)), 4});
  const int lanes = int((k + g.vec - 1) / g.vec);
  g.ytiles = (lanes + 63) / 64;
  g.G = lanes >= 64 ? 64 : next_pow2(lanes);
  g.lgG = ilog2(g.G);
  return g;
}

template <typename TX>
sped_status launch_edge_apply_t(const EdgeGeom &g, int64_t m, const int32_t *src, const int32_t *dst,
                                const float *w, const float *scale, int64_t n, int64_t k, const void *X,
                                int64_t ldx, float *Y, int64_t ldy, float alpha, unsigned long long *invalid,
                                hipStream_t s) {
  const int64_t per_block = (kBlock >> g.lgG) * kEdgeRun;
  const int64_t blocks = (m + per_block - 1) / per_block;
  if (blocks > 0x7fffffff) return fail(SPED_E_UNSUPPORTED, "edge batch too large for one launch");
  const dim3 grid(unsigned(blocks), unsigned(g.ytiles));
#define SPED_EDGE(V)                                                                                     \
  hipLaunchKernelGGL((edge_apply_kernel<TX, V>), grid, dim3(kBlock), 0, s, m, src, dst, w, scale, n, int(k), \
                     g.G, g.lgG, static_cast<const TX *>(X), ldx, Y, ldy, alpha, invalid)
  if (g.vec == 4) SPED_EDGE(4);
  else if (g.vec == 2) SPED_EDGE(2);
  else SPED_EDGE(1);
#undef SPED_EDGE
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

sped_status launch_edge_apply(const EdgeGeom &g, int64_t m, const int32_t *src, const int32_t *dst, const float *w,
                              const float *scale, int64_t n, int64_t k, const void *X, int64_t ldx, int xdt,
                              float *Y, int64_t ldy, float alpha, unsigned long long *invalid, hipStream_t s) {
  if (m == 0) return SPED_OK;
  if (xdt == SPED_F32)
    return launch_edge_apply_t<float>(g, m, src, dst, w, scale, n, k, X, ldx, Y, ldy, alpha, invalid, s);
  return launch_edge_apply_t<bf16_t>(g, m, src, dst, w, scale, n, k, X, ldx, Y, ldy, alpha, invalid, s);
}

sped_status check_block_args(int64_t n, int64_t k, const void *X, int64_t ldx, int xdt, const float *Y,
                             int64_t ldy) {
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(SPED_E_INVALID, "n out of range");
  if (k < 1) return fail(SPED_E_INVALID, "k < 1");
  if (xdt != SPED_F32 && xdt != SPED_BF16) return fail(SPED_E_UNSUPPORTED, "X dtype (F32 or BF16)");
  if (ldx < k || ldy < k) return fail(SPED_E_INVALID, "leading dimension smaller than k");
  if (n > 0 && (!X || !Y)) return fail(SPED_E_INVALID, "X or Y NULL");
  return SPED_OK;
}

// Host edge list -> device batches on a private copy stream, two staging
// buffers alternating.  Batch j is seg(j) = up to two ranges of the host
// arrays (a batch may wrap around the end of the list), copied back to back
// into one staging buffer; `body(j, src, dst, w, count)` enqueues the batch's
// kernels on `s`.  Synchronises `s` before returning.
struct Segs {
  int64_t off[2], cnt[2];
};

template <typename SegFn, typename Body>
sped_status stream_segments(int64_t nbatches, const int32_t *src_h, const int32_t *dst_h, const float *w_h,
                            int32_t *stage_src[2], int32_t *stage_dst[2], float *stage_w[2], hipStream_t s,
                            SegFn seg, Body body) {
  hipStream_t cs = nullptr;
  hipEvent_t copied[2] = {nullptr, nullptr}, used[2] = {nullptr, nullptr};
  sped_status st = SPED_OK;
  auto hip_ok = [&](hipError_t e, const char *what) {
    if (e != hipSuccess && st == SPED_OK) st = fail(SPED_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return st == SPED_OK;
  };
  if (hip_ok(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreateWithFlags") &&
      hip_ok(hipEventCreateWithFlags(&copied[0], hipEventDisableTiming), "hipEventCreate") &&
      hip_ok(hipEventCreateWithFlags(&copied[1], hipEventDisableTiming), "hipEventCreate") &&
      hip_ok(hipEventCreateWithFlags(&used[0], hipEventDisableTiming), "hipEventCreate") &&
      hip_ok(hipEventCreateWithFlags(&used[1], hipEventDisableTiming), "hipEventCreate")) {
    // the copies must not start before work already queued on s that may
    // still read the staging buffers
    hip_ok(hipEventRecord(used[0], s), "hipEventRecord");
    hip_ok(hipEventRecord(used[1], s), "hipEventRecord");
    int64_t count[2] = {0, 0};
    // Enqueue batch j's copy into buffer j & 1 on the copy stream, after the
    // kernels that last read that buffer (batch j - 2's).
    auto issue_copy = [&](int64_t j) {
      const int buf = int(j & 1);
      const Segs g = seg(j);
      if (!hip_ok(hipStreamWaitEvent(cs, used[buf], 0), "hipStreamWaitEvent")) return;
      int64_t at = 0;
      for (int q = 0; q < 2 && st == SPED_OK; ++q) {
        if (g.cnt[q] == 0) continue;
        hip_ok(hipMemcpyAsync(stage_src[buf] + at, src_h + g.off[q], g.cnt[q] * sizeof(int32_t),
                              hipMemcpyHostToDevice, cs), "hipMemcpyAsync");
        hip_ok(hipMemcpyAsync(stage_dst[buf] + at, dst_h + g.off[q], g.cnt[q] * sizeof(int32_t),
                              hipMemcpyHostToDevice, cs), "hipMemcpyAsync");
        if (w_h)
          hip_ok(hipMemcpyAsync(stage_w[buf] + at, w_h + g.off[q], g.cnt[q] * sizeof(float), hipMemcpyHostToDevice,
                                cs), "hipMemcpyAsync");
        at += g.cnt[q];
      }
      count[buf] = at;
      hip_ok(hipEventRecord(copied[buf], cs), "hipEventRecord");
    };
    if (nbatches > 0) issue_copy(0);
    for (int64_t j = 0; j < nbatches && st == SPED_OK; ++j) {
      const int buf = int(j & 1);
      if (!hip_ok(hipStreamWaitEvent(s, copied[buf], 0), "hipStreamWaitEvent")) break;
      // One batch ahead: batch j + 1's copy is queued before batch j's
      // kernels, so it overlaps them even when the body synchronises.
      if (j + 1 < nbatches) issue_copy(j + 1);
      if (st != SPED_OK) break;
      const sped_status kst = body(j, stage_src[buf], stage_dst[buf], w_h ? stage_w[buf] : nullptr, count[buf]);
      if (kst != SPED_OK) {
        st = kst;
        break;
      }
      hip_ok(hipEventRecord(used[buf], s), "hipEventRecord");
    }
  }
  // drain both streams before the events, the copy stream and the caller's
  // host arrays can go away
  const hipError_t e1 = cs ? hipStreamSynchronize(cs) : hipSuccess;
  const hipError_t e2 = hipStreamSynchronize(s);
  hip_ok(e1, "hipStreamSynchronize");
  hip_ok(e2, "hipStreamSynchronize");
  for (hipEvent_t ev : {copied[0], copied[1], used[0], used[1]})
    if (ev) hipEventDestroy(ev);
  if (cs) hipStreamDestroy(cs);
  return st;
}

// The list [0, m) in consecutive batches of `batch` edges.
template <typename Body>
sped_status stream_batches(int64_t m, const int32_t *src_h, const int32_t *dst_h, const float *w_h, int64_t batch,
                           int32_t *stage_src[2], int32_t *stage_dst[2], float *stage_w[2], hipStream_t s,
                           Body body) {
  const int64_t nb = (m + batch - 1) / batch;
  return stream_segments(
      nb, src_h, dst_h, w_h, stage_src, stage_dst, stage_w, s,
      [&](int64_t j) {
        Segs g{{j * batch, 0}, {std::min(batch, m - j * batch), 0}};
        return g;
      },
      body);
}

struct StreamWs {
  int32_t *src[2], *dst[2];
  float *w[2];
  unsigned long long *invalid;
};

size_t carve_stream_ws(void *ws, int64_t batch, StreamWs *out) {
  Carver c(ws);
  for (int b = 0; b < 2; ++b) {
    out->src[b] = c.take<int32_t>(size_t(batch));
    out->dst[b] = c.take<int32_t>(size_t(batch));
    out->w[b] = c.take<float>(size_t(batch));
  }
  out->invalid = c.take<unsigned long long>(1);
  return c.bytes();
}

sped_status read_invalid(const unsigned long long *invalid, hipStream_t s) {
  unsigned long long h = 0;
  SPED_CHECK_HIP(hipMemcpyAsync(&h, invalid, sizeof(h), hipMemcpyDeviceToHost, s));
  SPED_CHECK_HIP(hipStreamSynchronize(s));
  if (h) return fail(SPED_E_INVALID, std::to_string(h) + " edges with an endpoint outside [0, n) or a weight not "
                                                        "finite and > 0 (skipped)");
  return SPED_OK;
}

}  // namespace
}  // namespace sped

using namespace sped;

extern "C" sped_status sped_edge_apply(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const float *w,
                                       const float *scale, int64_t k, const void *X, int64_t ldx, int32_t xdt,
                                       float *Y, int64_t ldy, float alpha, unsigned long long *invalid,
                                       sped_stream_t stream) {
  clear_error();
  SPED_TRY(check_block_args(n, k, X, ldx, xdt, Y, ldy));
  if (m < 0) return fail(SPED_E_INVALID, "m < 0");
  if (m > 0 && (!src || !dst)) return fail(SPED_E_INVALID, "src or dst NULL");
  if (!std::isfinite(alpha)) return fail(SPED_E_INVALID, "alpha not finite");
  if (n > 0 && static_cast<const void *>(Y) == X) return fail(SPED_E_INVALID, "Y must not be X");
  const EdgeGeom g = edge_geom(k, X, ldx, xdt, Y, ldy);
  return launch_edge_apply(g, m, src, dst, w, scale, n, k, X, ldx, xdt, Y, ldy, alpha, invalid, as_stream(stream));
}

extern "C" sped_status sped_stream_node_scales(int64_t n, int64_t m, const int32_t *src_h, const int32_t *dst_h,
                                               const float *w_h, int32_t kind, int64_t batch, double *degree,
                                               float *scale, void *ws, size_t *ws_bytes, sped_stream_t stream) {
  clear_error();
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(SPED_E_INVALID, "n out of range");
  if (m < 0) return fail(SPED_E_INVALID, "m < 0");
  if (batch < 1) return fail(SPED_E_INVALID, "batch < 1");
  if (kind != SPED_LAP_COMBINATORIAL && kind != SPED_LAP_SYM_NORMALIZED) return fail(SPED_E_INVALID, "kind");
  if (m > 0 && (!src_h || !dst_h)) return fail(SPED_E_INVALID, "src or dst NULL");
  if (n > 0 && (!degree || !scale)) return fail(SPED_E_INVALID, "degree or scale NULL");
  StreamWs w;
  const size_t need = carve_stream_ws(ws, std::min(batch, std::max<int64_t>(m, 1)), &w);
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, need, &query));
  if (query) return SPED_OK;
  hipStream_t s = as_stream(stream);
  if (n > 0) {
    hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_blocks(n)), dim3(kBlock), 0, s, n, degree);
    SPED_CHECK_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, w.invalid);
  SPED_CHECK_HIP(hipGetLastError());
  const int64_t bsz = std::min(batch, std::max<int64_t>(m, 1));
  SPED_TRY(stream_batches(m, src_h, dst_h, w_h, bsz, w.src, w.dst, w.w, s,
                          [&](int64_t, const int32_t *bs, const int32_t *bd, const float *bw, int64_t cnt) {
                            const unsigned blocks = grid_blocks((cnt + kEdgeRun - 1) / kEdgeRun);
                            hipLaunchKernelGGL(edge_degree_kernel, dim3(blocks), dim3(kBlock), 0, s, cnt, bs, bd, bw,
                                               n, degree, w.invalid);
                            SPED_CHECK_HIP(hipGetLastError());
                            return SPED_OK;
                          }));
  if (n > 0) {
    hipLaunchKernelGGL(node_scale_kernel, dim3(grid_blocks(n)), dim3(kBlock), 0, s, n, int(kind), degree, scale);
    SPED_CHECK_HIP(hipGetLastError());
  }
  return read_invalid(w.invalid, s);
}

extern "C" sped_status sped_stream_laplacian_apply(int64_t n, int64_t m, const int32_t *src_h, const int32_t *dst_h,
                                                   const float *w_h, const float *scale, int64_t k, const void *X,
                                                   int64_t ldx, int32_t xdt, float *Y, int64_t ldy, float alpha,
                                                   int32_t accumulate, int64_t batch, void *ws, size_t *ws_bytes,
                                                   sped_stream_t stream) {
  clear_error();
  SPED_TRY(check_block_args(n, k, X, ldx, xdt, Y, ldy));
  if (m < 0) return fail(SPED_E_INVALID, "m < 0");
  if (batch < 1) return fail(SPED_E_INVALID, "batch < 1");
  if (m > 0 && (!src_h || !dst_h)) return fail(SPED_E_INVALID, "src or dst NULL");
  if (!std::isfinite(alpha)) return fail(SPED_E_INVALID, "alpha not finite");
  if (n > 0 && static_cast<const void *>(Y) == X) return fail(SPED_E_INVALID, "Y must not be X");
  StreamWs w;
  const int64_t bsz = std::min(batch, std::max<int64_t>(m, 1));
  const size_t need = carve_stream_ws(ws, bsz, &w);
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, need, &query));
  if (query) return SPED_OK;
  hipStream_t s = as_stream(stream);
  if (!accumulate && n > 0) {
    hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_blocks(n * k)), dim3(kBlock), 0, s, n, int(k), Y, ldy);
    SPED_CHECK_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, w.invalid);
  SPED_CHECK_HIP(hipGetLastError());
  const EdgeGeom g = edge_geom(k, X, ldx, xdt, Y, ldy);
  SPED_TRY(stream_batches(m, src_h, dst_h, w_h, bsz, w.src, w.dst, w.w, s,
                          [&](int64_t, const int32_t *bs, const int32_t *bd, const float *bw, int64_t cnt) {
                            return launch_edge_apply(g, cnt, bs, bd, bw, scale, n, k, X, ldx, xdt, Y, ldy, alpha,
                                                     w.invalid, s);
                          }));
  return read_invalid(w.invalid, s);
}

extern "C" sped_status sped_minibatch_oja(int64_t n, int64_t m, const int32_t *src_h, const int32_t *dst_h,
                                          const float *w_h, const float *scale, int32_t degree, double lambda_bound,
                                          int64_t k, float *V, int64_t ldv, int64_t batch, double eta, int32_t iters,
                                          uint64_t seed, int64_t batch0, void *ws, size_t *ws_bytes,
                                          sped_stream_t stream) {
  clear_error();
  if (n < 1 || n >= (int64_t(1) << 31)) return fail(SPED_E_INVALID, "n out of range");
  if (k < 1 || k > 96) return fail(SPED_E_UNSUPPORTED, "k outside [1, 96]");
  if (ldv < k) return fail(SPED_E_INVALID, "ldv < k");
  if (!V) return fail(SPED_E_INVALID, "V NULL");
  if (m < 1 || !src_h || !dst_h) return fail(SPED_E_INVALID, "empty or NULL edge list");
  if (batch < 1 || batch > m) return fail(SPED_E_INVALID, "batch outside [1, m]");
  if (degree < 0 || degree > 1024) return fail(SPED_E_INVALID, "degree outside [0, 1024]");
  if (degree == 0 && !(std::isfinite(lambda_bound) && lambda_bound > 0.0)) return fail(SPED_E_INVALID, "lambda_bound");
  if (!(std::isfinite(eta) && eta > 0.0)) return fail(SPED_E_INVALID, "eta");
  if (iters < 0) return fail(SPED_E_INVALID, "iters < 0");
  if (m >= (int64_t(1) << 32)) return fail(SPED_E_UNSUPPORTED, "m >= 2^32 edges");
  if (batch0 < 0) return fail(SPED_E_INVALID, "batch0 < 0");
  StreamWs w;
  Carver c(ws);
  const size_t stage = carve_stream_ws(ws, batch, &w);
  c.off = stage;
  float *W0 = c.take<float>(size_t(n) * k);
  float *W1 = c.take<float>(size_t(n) * k);
  size_t orth_need = 0;
  SPED_TRY(sped_orthonormalize(n, k, V, ldv, SPED_F32, 2, nullptr, nullptr, &orth_need, stream));
  void *orth_ws = c.take<char>(orth_need);
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, c.bytes(), &query));
  if (query) return SPED_OK;
  clear_error();
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, w.invalid);
  SPED_CHECK_HIP(hipGetLastError());
  const int F = degree == 0 ? 1 : int(degree);
  const EdgeGeom g = edge_geom(k, V, ldv, SPED_F32, W0, k);
  const unsigned blocks = grid_blocks(n * k);
  const float a = degree == 0 ? float(-double(m) / double(batch)) : float(-double(m) / double(batch) / F);
  float *cur = W0, *nxt = W1;
  // Batch j of the call (global index J = batch0 + j) holds the edges
  // (o_J + r) mod m, r < batch, from a uniform offset o_J in [0, m) drawn by
  // Philox (key = seed, counter (J mod 2^32, J >> 32, 0, 0)) with Lemire's
  // bound: each edge is in a batch with probability batch / m, and the
  // batches of different factors are independent, so the product of the
  // factors' estimates has the product of their expectations as its mean.
  const uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32);
  const sped_status st = stream_segments(
      int64_t(iters) * F, src_h, dst_h, w_h, w.src, w.dst, w.w, s,
      [&](int64_t j) {
        const uint64_t J = uint64_t(batch0 + j);
        const int64_t o = int64_t(lemire_draw(k0, k1, uint32_t(J), uint32_t(J >> 32), 0u, 0u, uint32_t(m)));
        const int64_t first = std::min(batch, m - o);
        Segs sg{{o, 0}, {first, batch - first}};
        return sg;
      },
      [&](int64_t j, const int32_t *bs, const int32_t *bd, const float *bw, int64_t cnt) -> sped_status {
        const int f = int(j % F);
        if (degree == 0) {  // W = lambda V - (m / b) L_B V
          hipLaunchKernelGGL(scale_copy_kernel, dim3(blocks), dim3(kBlock), 0, s, n, int(k), V, ldv, cur, k,
                             float(lambda_bound));
          SPED_CHECK_HIP(hipGetLastError());
          SPED_TRY(launch_edge_apply(g, cnt, bs, bd, bw, scale, n, k, V, ldv, SPED_F32, cur, k, a, w.invalid, s));
        } else {  // W <- (I - (m / b) L_B / l) W, W = V before the first factor
          const float *in = f == 0 ? V : cur;
          const int64_t ldi = f == 0 ? ldv : k;
          hipLaunchKernelGGL(scale_copy_kernel, dim3(blocks), dim3(kBlock), 0, s, n, int(k), in, ldi, nxt, k, 1.f);
          SPED_CHECK_HIP(hipGetLastError());
          SPED_TRY(launch_edge_apply(g, cnt, bs, bd, bw, scale, n, k, in, ldi, SPED_F32, nxt, k, a, w.invalid, s));
          std::swap(cur, nxt);
        }
        if (f == F - 1) {  // V <- orth(V + eta W)
          hipLaunchKernelGGL(axpy_block_kernel, dim3(blocks), dim3(kBlock), 0, s, n, int(k), V, ldv, cur, k,
                             float(eta));
          SPED_CHECK_HIP(hipGetLastError());
          size_t need = orth_need;
          SPED_TRY(sped_orthonormalize(n, k, V, ldv, SPED_F32, 2, nullptr, orth_need ? orth_ws : nullptr,
                                       orth_need ? &need : nullptr, stream));
        }
        return SPED_OK;
      });
  if (st != SPED_OK) return st;
  return read_invalid(w.invalid, s);
}
