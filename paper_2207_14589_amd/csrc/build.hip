// Graph -> split CSR Laplacian on the device (Sec. 2: L = X^T W X with
// incidence rows +1 at min(i, j) and -1 at max(i, j); Sec. 4.1 normalised
// form).  Steps:
//   1. every input edge (i, j, w), i != j, becomes the two directed keys
//      (i << 32 | j) and (j << 32 | i); self-loops (zero incidence row) become
//      a sentinel key that sorts last;
//   2. stable radix sort of (key, w);
//   3. repeated keys are merged by summing their weights in sorted order
//      (each repeat is its own row of X, so the weights add);
//   4. optionally keep the largest connected component: min-label hooking
//      with pointer jumping, component sizes, relabelling by exclusive scan;
//   5. row pointers, weighted degrees d_i, s_i, diag, values S_ij, the
//      position of every transposed entry, and the medium/heavy row bins.
#include <hipcub/hipcub.hpp>

#include <cmath>

#include "common.h"

namespace sped {
namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > 65536) b = 65536;
  return unsigned(b > 0 ? b : 1);
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < (n); i += int64_t(gridDim.x) * kBlock)

__global__ void emit_directed(int64_t n, int64_t m, const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                              const float *__restrict__ w, uint64_t *__restrict__ keys, float *__restrict__ vals,
                              int *__restrict__ err) {
  const uint64_t sentinel = uint64_t(n) << 32;
  GRID_STRIDE(e, m) {
    int32_t u = src[e], v = dst[e];
    float wt = w ? w[e] : 1.0f;
    bool bad = u < 0 || v < 0 || int64_t(u) >= n || int64_t(v) >= n || !(wt > 0.0f) || !isfinite(wt);
    if (bad) atomicOr(err, 1);
    if (bad || u == v) {
      keys[2 * e] = keys[2 * e + 1] = sentinel;
      vals[2 * e] = vals[2 * e + 1] = 0.0f;
    } else {
      keys[2 * e] = (uint64_t(uint32_t(u)) << 32) | uint32_t(v);
      keys[2 * e + 1] = (uint64_t(uint32_t(v)) << 32) | uint32_t(u);
      vals[2 * e] = vals[2 * e + 1] = wt;
    }
  }
}

__global__ void head_flags(int64_t cnt, const uint64_t *__restrict__ keys, uint64_t sentinel,
                           int64_t *__restrict__ flags) {
  GRID_STRIDE(p, cnt) {
    uint64_t k = keys[p];
    flags[p] = (k != sentinel && (p == 0 || keys[p - 1] != k)) ? 1 : 0;
  }
}

// For each run head, sum the run's weights in order and write the merged entry.
__global__ void merge_runs(int64_t cnt, const uint64_t *__restrict__ keys, const float *__restrict__ vals,
                           const int64_t *__restrict__ flags, const int64_t *__restrict__ pos,
                           uint64_t *__restrict__ ukeys, double *__restrict__ uw) {
  GRID_STRIDE(p, cnt) {
    if (!flags[p]) continue;
    uint64_t k = keys[p];
    double s = 0.0;
    for (int64_t q = p; q < cnt && keys[q] == k; ++q) s += double(vals[q]);
    ukeys[pos[p]] = k;
    uw[pos[p]] = s;
  }
}

__global__ void init_labels(int64_t n, int32_t *__restrict__ label) {
  GRID_STRIDE(i, n) label[i] = int32_t(i);
}

// Labels are read with device-scope atomic loads: other workgroups lower them
// concurrently and a stale cached copy could otherwise be read forever.
__device__ inline int32_t find_root(int32_t *label, int32_t x) {
  while (true) {
    int32_t p = __hip_atomic_load(&label[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p == x) return x;
    x = p;
  }
}

// hook the larger root under the smaller one; labels only ever decrease
__global__ void hook_edges(int64_t nnz, const uint64_t *__restrict__ keys, int32_t *label, int *changed) {
  GRID_STRIDE(p, nnz) {
    int32_t u = int32_t(keys[p] >> 32), v = int32_t(keys[p] & 0xffffffffu);
    if (u > v) continue;  // each undirected edge once
    while (true) {
      int32_t ru = find_root(label, u), rv = find_root(label, v);
      if (ru == rv) break;
      int32_t hi = ru > rv ? ru : rv, lo = ru > rv ? rv : ru;
      int32_t old = atomicMin(&label[hi], lo);
      if (old == hi) {
        *changed = 1;
        break;
      }
    }
  }
}

__global__ void compress_labels(int64_t n, int32_t *label) {
  GRID_STRIDE(i, n) label[i] = find_root(label, int32_t(i));
}

// Component sizes.  Most nodes of a real graph share one label (the giant
// component), so one counter would take an atomic per node; lanes of a
// wavefront whose label equals the first active lane's add once, as a group.
__global__ void count_components(int64_t n, const int32_t *__restrict__ label, int32_t *__restrict__ size) {
  GRID_STRIDE(i, n) {
    const int32_t l = label[i];
    const int32_t lead = __builtin_amdgcn_readfirstlane(l);
    const unsigned long long same = __ballot(l == lead);
    if (l != lead) {
      atomicAdd(&size[l], 1);
    } else if (int(threadIdx.x & 63) == __ffsll(static_cast<long long>(same)) - 1) {
      atomicAdd(&size[lead], __popcll(same));
    }
  }
}

// pick (largest size, then smallest root): max of size << 32 | ~root
__global__ void best_component(int64_t n, const int32_t *__restrict__ label, const int32_t *__restrict__ size,
                               unsigned long long *__restrict__ best) {
  GRID_STRIDE(i, n) {
    if (label[i] == int32_t(i)) {
      unsigned long long key = (uint64_t(uint32_t(size[i])) << 32) | uint64_t(0xffffffffu - uint32_t(i));
      atomicMax(best, key);
    }
  }
}

__global__ void keep_flags(int64_t n, const int32_t *__restrict__ label, const unsigned long long *__restrict__ best,
                           int64_t *__restrict__ keep) {
  const int32_t root = int32_t(0xffffffffu - uint32_t(*best & 0xffffffffu));
  GRID_STRIDE(i, n) keep[i] = label[i] == root ? 1 : 0;
}

__global__ void relabel_map(int64_t n, const int64_t *__restrict__ keep, const int64_t *__restrict__ newid,
                            int32_t *__restrict__ old_of_new) {
  GRID_STRIDE(i, n) if (keep[i] && old_of_new) old_of_new[newid[i]] = int32_t(i);
}

__global__ void entry_keep(int64_t nnz, const uint64_t *__restrict__ keys, const int64_t *__restrict__ keep,
                           int64_t *__restrict__ flags) {
  GRID_STRIDE(p, nnz) flags[p] = keep[keys[p] >> 32];
}

__global__ void compact_entries(int64_t nnz, const uint64_t *__restrict__ keys, const double *__restrict__ w,
                                const int64_t *__restrict__ flags, const int64_t *__restrict__ pos,
                                const int64_t *__restrict__ newid, uint64_t *__restrict__ okeys,
                                double *__restrict__ ow) {
  GRID_STRIDE(p, nnz) {
    if (!flags[p]) continue;
    uint64_t k = keys[p];
    uint64_t r = uint64_t(newid[k >> 32]), c = uint64_t(newid[k & 0xffffffffu]);
    okeys[pos[p]] = (r << 32) | c;
    ow[pos[p]] = w[p];
  }
}

__global__ void identity_map(int64_t n, int32_t *__restrict__ old_of_new) {
  GRID_STRIDE(i, n) old_of_new[i] = int32_t(i);
}

__global__ void row_pointers(int64_t n, int64_t nnz, const uint64_t *__restrict__ keys, int64_t *__restrict__ rowptr) {
  GRID_STRIDE(r, n + 1) {
    uint64_t target = uint64_t(r) << 32;
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < target) lo = mid + 1;
      else hi = mid;
    }
    rowptr[r] = lo;
  }
}

__global__ void degrees(int64_t n, const int64_t *__restrict__ rowptr, const double *__restrict__ w,
                        double *__restrict__ deg, int *__restrict__ maxcount) {
  GRID_STRIDE(r, n) {
    double s = 0.0;
    for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) s += w[p];
    deg[r] = s;
    atomicMax(maxcount, int(rowptr[r + 1] - rowptr[r]));
  }
}

__global__ void node_scales(int64_t n, int kind, const double *__restrict__ deg, float *__restrict__ scale,
                            float *__restrict__ diag, double *__restrict__ sd) {
  GRID_STRIDE(r, n) {
    double d = deg[r];
    double s = 1.0;
    if (kind == SPED_LAP_SYM_NORMALIZED) s = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    sd[r] = s;
    scale[r] = float(s);
    diag[r] = float(kind == SPED_LAP_SYM_NORMALIZED ? (d > 0.0 ? 1.0 : 0.0) : d);
  }
}

__global__ void entry_values(int64_t nnz, int kind, const uint64_t *__restrict__ keys, const double *__restrict__ w,
                             const double *__restrict__ sd, int32_t *__restrict__ col, float *__restrict__ val) {
  GRID_STRIDE(p, nnz) {
    uint64_t k = keys[p];
    int64_t r = int64_t(k >> 32), c = int64_t(k & 0xffffffffu);
    col[p] = int32_t(c);
    val[p] = float(kind == SPED_LAP_SYM_NORMALIZED ? w[p] * sd[r] * sd[c] : w[p]);
  }
}

__global__ void reverse_positions(int64_t nnz, const uint64_t *__restrict__ keys, const int64_t *__restrict__ rowptr,
                                  int64_t *__restrict__ rev) {
  GRID_STRIDE(p, nnz) {
    uint64_t k = keys[p];
    uint64_t target = ((k & 0xffffffffu) << 32) | (k >> 32);
    int64_t c = int64_t(k & 0xffffffffu);
    int64_t lo = rowptr[c], hi = rowptr[c + 1];
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < target) lo = mid + 1;
      else hi = mid;
    }
    rev[p] = lo;
  }
}

__global__ void walk_entry_records(int64_t nnz, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                   const float *__restrict__ val, const int64_t *__restrict__ rev,
                                   const float *__restrict__ scale, sped_walk_entry *__restrict__ we) {
  GRID_STRIDE(p, nnz) {
    const int32_t c = col[p];
    const int64_t c0 = rowptr[c];
    sped_walk_entry e;
    e.col = c;
    e.val = val[p];
    e.rev_local = int32_t(rev[p] - c0);
    e.degree = int32_t(rowptr[c + 1] - c0);
    e.start = c0;
    e.root_scale = sqrtf(scale[c]);
    e.pad = 0;
    we[p] = e;
  }
}

__global__ void walk_node_records(int64_t n, const int64_t *__restrict__ rowptr, const float *__restrict__ scale,
                                  sped_walk_node *__restrict__ wn) {
  GRID_STRIDE(r, n) {
    sped_walk_node v;
    v.start = rowptr[r];
    v.degree = int32_t(rowptr[r + 1] - rowptr[r]);
    v.root_scale = sqrtf(scale[r]);
    wn[r] = v;
  }
}

__global__ void bin_flags(int64_t n, const int64_t *__restrict__ rowptr, char *__restrict__ fmed,
                          char *__restrict__ fheavy) {
  GRID_STRIDE(r, n) {
    int64_t d = rowptr[r + 1] - rowptr[r];
    fmed[r] = (d > SPED_LIGHT_MAX && d <= SPED_MEDIUM_MAX) ? 1 : 0;
    fheavy[r] = d > SPED_MEDIUM_MAX ? 1 : 0;
  }
}

// Cost of a row for the light-row SpMM, in entry units: a light row pays its
// entries (one neighbour-row gather each) plus the row pointers and its own
// row's read and write; a medium or heavy row only the light kernel's early
// exit.  Prefix sums of this give the XCD row split (sped_csr.xcd_rows).
constexpr int64_t kLightRowCost = 2;

__global__ void light_work(int64_t n, const int64_t *__restrict__ rowptr, int64_t *__restrict__ work) {
  GRID_STRIDE(r, n + 1) {
    int64_t w = 0;
    if (r < n) {
      const int64_t d = rowptr[r + 1] - rowptr[r];
      w = d <= SPED_LIGHT_MAX ? d + kLightRowCost : 1;
    }
    work[r] = w;
  }
}

// splits[x] = smallest r with prefix[r] >= x total / 8, prefix exclusive over
// n + 1 entries (prefix[n] = total).  Work is >= 1 per row, so prefix is
// strictly increasing, splits[0] = 0 and splits[8] = n.
__global__ void xcd_splits(int64_t n, const int64_t *__restrict__ prefix, int64_t *__restrict__ splits) {
  const int x = threadIdx.x;
  if (x > kXcds) return;
  const int64_t total = prefix[n];
  const int64_t target = total / kXcds * x + total % kXcds * x / kXcds;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (prefix[mid] >= target) hi = mid;
    else lo = mid + 1;
  }
  splits[x] = lo;
}

struct BuildWs {
  uint64_t *kA, *kB;
  float *vA, *vB;
  double *wA, *wB;
  int64_t *flags, *pos;
  int64_t *keep, *newid;
  int32_t *label, *csize;
  double *deg, *sd, *dmax;
  char *fmed, *fheavy;
  int32_t *counting;
  int64_t *nsel, *splits;
  unsigned long long *best;
  int *err, *changed, *maxcount;
  void *temp;
  size_t temp_bytes;
};

size_t cub_temp_bytes(int64_t n, int64_t cnt) {
  size_t a = 0, b = 0, c = 0, d = 0, e = 0;
  hipcub::DeviceRadixSort::SortPairs(nullptr, a, (uint64_t *)nullptr, (uint64_t *)nullptr, (float *)nullptr,
                                     (float *)nullptr, cnt, 0, 64);
  hipcub::DeviceScan::ExclusiveSum(nullptr, b, (int64_t *)nullptr, (int64_t *)nullptr, cnt > n + 1 ? cnt : n + 1);
  hipcub::DeviceReduce::Max(nullptr, c, (double *)nullptr, (double *)nullptr, n > 0 ? n : 1);
  hipcub::CountingInputIterator<int32_t> rows(0);
  hipcub::DeviceSelect::Flagged(nullptr, d, rows, (char *)nullptr, (int32_t *)nullptr, (int64_t *)nullptr,
                                n > 0 ? n : 1);
  e = a > b ? a : b;
  e = e > c ? e : c;
  e = e > d ? e : d;
  return e;
}

}  // namespace
}  // namespace sped

using namespace sped;

extern "C" sped_status sped_laplacian_csr(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const float *w,
                                          int32_t kind, int32_t lcc_only, sped_csr *out, int32_t *old_of_new,
                                          void *ws, size_t *ws_bytes, sped_stream_t stream) {
  clear_error();
  if (n < 0 || n >= (int64_t(1) << 31) - 1) return fail(SPED_E_INVALID, "n outside [0, 2^31 - 1)");
  if (m < 0 || m > (int64_t(1) << 40)) return fail(SPED_E_INVALID, "m out of range");
  if (m > 0 && (!src || !dst)) return fail(SPED_E_INVALID, "src/dst NULL");
  if (kind != SPED_LAP_COMBINATORIAL && kind != SPED_LAP_SYM_NORMALIZED) return fail(SPED_E_INVALID, "kind");
  if (!out) return fail(SPED_E_INVALID, "out NULL");
  const int64_t cnt = 2 * m;
  Carver c(ws);
  BuildWs b;
  b.kA = c.take<uint64_t>(cnt > 0 ? cnt : 1);
  b.kB = c.take<uint64_t>(cnt > 0 ? cnt : 1);
  b.vA = c.take<float>(cnt > 0 ? cnt : 1);
  b.vB = c.take<float>(cnt > 0 ? cnt : 1);
  b.wA = c.take<double>(cnt > 0 ? cnt : 1);
  b.wB = c.take<double>(cnt > 0 ? cnt : 1);
  b.flags = c.take<int64_t>((cnt > n + 1 ? cnt : n + 1));
  b.pos = c.take<int64_t>((cnt > n + 1 ? cnt : n + 1));
  b.keep = c.take<int64_t>(n + 1);
  b.newid = c.take<int64_t>(n + 1);
  b.label = c.take<int32_t>(n + 1);
  b.csize = c.take<int32_t>(n + 1);
  b.deg = c.take<double>(n + 1);
  b.sd = c.take<double>(n + 1);
  b.dmax = c.take<double>(1);
  b.fmed = c.take<char>(n + 1);
  b.fheavy = c.take<char>(n + 1);
  b.counting = c.take<int32_t>(n + 1);
  b.nsel = c.take<int64_t>(2);
  b.splits = c.take<int64_t>(kXcds + 1);
  b.best = c.take<unsigned long long>(1);
  b.err = c.take<int>(4);
  b.changed = b.err ? b.err + 1 : nullptr;  // NULL in the size query
  b.maxcount = b.err ? b.err + 2 : nullptr;
  b.temp_bytes = cub_temp_bytes(n, cnt > 0 ? cnt : 1);
  b.temp = c.take<char>(b.temp_bytes);
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, c.bytes(), &query));
  if (query) return SPED_OK;
  if (!out->rowptr || (n > 0 && (!out->diag || !out->scale || !out->bins)) ||
      (cnt > 0 && (!out->col || !out->val || !out->rev)))
    return fail(SPED_E_INVALID, "output arrays NULL");

  hipStream_t s = as_stream(stream);
  SPED_CHECK_HIP(hipMemsetAsync(b.err, 0, 4 * sizeof(int), s));
  const uint64_t sentinel = uint64_t(n) << 32;
  int end_bit = 33;
  while (end_bit < 64 && (uint64_t(1) << (end_bit - 32)) <= uint64_t(n)) ++end_bit;
  int64_t nnz = 0;
  if (cnt > 0) {
    hipLaunchKernelGGL(emit_directed, dim3(grid_for(m)), dim3(kBlock), 0, s, n, m, src, dst, w, b.kA, b.vA, b.err);
    SPED_CHECK_HIP(hipGetLastError());
    size_t tb = b.temp_bytes;
    SPED_CHECK_HIP(hipcub::DeviceRadixSort::SortPairs(b.temp, tb, b.kA, b.kB, b.vA, b.vB, cnt, 0, end_bit, s));
    hipLaunchKernelGGL(head_flags, dim3(grid_for(cnt)), dim3(kBlock), 0, s, cnt, b.kB, sentinel, b.flags);
    SPED_CHECK_HIP(hipGetLastError());
    tb = b.temp_bytes;
    SPED_CHECK_HIP(hipcub::DeviceScan::ExclusiveSum(b.temp, tb, b.flags, b.pos, cnt, s));
    hipLaunchKernelGGL(merge_runs, dim3(grid_for(cnt)), dim3(kBlock), 0, s, cnt, b.kB, b.vB, b.flags, b.pos, b.kA,
                       b.wA);
    SPED_CHECK_HIP(hipGetLastError());
    int64_t last_pos = 0, last_flag = 0;
    int herr = 0;
    SPED_CHECK_HIP(hipMemcpyAsync(&last_pos, b.pos + cnt - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPED_CHECK_HIP(hipMemcpyAsync(&last_flag, b.flags + cnt - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPED_CHECK_HIP(hipMemcpyAsync(&herr, b.err, sizeof(int), hipMemcpyDeviceToHost, s));
    SPED_CHECK_HIP(hipStreamSynchronize(s));
    if (herr) return fail(SPED_E_INVALID, "edge endpoint outside [0, n) or weight not finite and > 0");
    nnz = last_pos + last_flag;
  } else {
    int herr = 0;
    SPED_CHECK_HIP(hipMemcpyAsync(&herr, b.err, sizeof(int), hipMemcpyDeviceToHost, s));
    SPED_CHECK_HIP(hipStreamSynchronize(s));
  }
  // merged entries now in (kA, wA), nnz of them
  uint64_t *keys = b.kA;
  double *wts = b.wA;
  int64_t n_out = n;
  if (lcc_only && n > 0) {
    hipLaunchKernelGGL(init_labels, dim3(grid_for(n)), dim3(kBlock), 0, s, n, b.label);
    SPED_CHECK_HIP(hipGetLastError());
    for (int round = 0; round < 64; ++round) {
      int hchanged = 0;
      SPED_CHECK_HIP(hipMemsetAsync(b.changed, 0, sizeof(int), s));
      if (nnz > 0) {
        hipLaunchKernelGGL(hook_edges, dim3(grid_for(nnz)), dim3(kBlock), 0, s, nnz, keys, b.label, b.changed);
        SPED_CHECK_HIP(hipGetLastError());
      }
      hipLaunchKernelGGL(compress_labels, dim3(grid_for(n)), dim3(kBlock), 0, s, n, b.label);
      SPED_CHECK_HIP(hipGetLastError());
      SPED_CHECK_HIP(hipMemcpyAsync(&hchanged, b.changed, sizeof(int), hipMemcpyDeviceToHost, s));
      SPED_CHECK_HIP(hipStreamSynchronize(s));
      if (!hchanged) break;
    }
    SPED_CHECK_HIP(hipMemsetAsync(b.csize, 0, sizeof(int32_t) * n, s));
    SPED_CHECK_HIP(hipMemsetAsync(b.best, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(count_components, dim3(grid_for(n)), dim3(kBlock), 0, s, n, b.label, b.csize);
    hipLaunchKernelGGL(best_component, dim3(grid_for(n)), dim3(kBlock), 0, s, n, b.label, b.csize, b.best);
    hipLaunchKernelGGL(keep_flags, dim3(grid_for(n)), dim3(kBlock), 0, s, n, b.label, b.best, b.keep);
    SPED_CHECK_HIP(hipGetLastError());
    size_t tb = b.temp_bytes;
    SPED_CHECK_HIP(hipcub::DeviceScan::ExclusiveSum(b.temp, tb, b.keep, b.newid, n + 0, s));
    hipLaunchKernelGGL(relabel_map, dim3(grid_for(n)), dim3(kBlock), 0, s, n, b.keep, b.newid, old_of_new);
    SPED_CHECK_HIP(hipGetLastError());
    int64_t lastk = 0, lastid = 0;
    SPED_CHECK_HIP(hipMemcpyAsync(&lastk, b.keep + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPED_CHECK_HIP(hipMemcpyAsync(&lastid, b.newid + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    int64_t new_nnz = 0;
    if (nnz > 0) {
      hipLaunchKernelGGL(entry_keep, dim3(grid_for(nnz)), dim3(kBlock), 0, s, nnz, keys, b.keep, b.flags);
      SPED_CHECK_HIP(hipGetLastError());
      tb = b.temp_bytes;
      SPED_CHECK_HIP(hipcub::DeviceScan::ExclusiveSum(b.temp, tb, b.flags, b.pos, nnz, s));
      hipLaunchKernelGGL(compact_entries, dim3(grid_for(nnz)), dim3(kBlock), 0, s, nnz, keys, wts, b.flags, b.pos,
                         b.newid, b.kB, b.wB);
      SPED_CHECK_HIP(hipGetLastError());
      int64_t lp = 0, lf = 0;
      SPED_CHECK_HIP(hipMemcpyAsync(&lp, b.pos + nnz - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      SPED_CHECK_HIP(hipMemcpyAsync(&lf, b.flags + nnz - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      SPED_CHECK_HIP(hipStreamSynchronize(s));
      new_nnz = lp + lf;
    }
    SPED_CHECK_HIP(hipStreamSynchronize(s));
    n_out = lastid + lastk;
    nnz = new_nnz;
    keys = b.kB;
    wts = b.wB;
  } else if (old_of_new && n > 0) {
    hipLaunchKernelGGL(identity_map, dim3(grid_for(n)), dim3(kBlock), 0, s, n, old_of_new);
    SPED_CHECK_HIP(hipGetLastError());
  }

  // CSR arrays
  hipLaunchKernelGGL(row_pointers, dim3(grid_for(n_out + 1)), dim3(kBlock), 0, s, n_out, nnz, keys, out->rowptr);
  SPED_CHECK_HIP(hipGetLastError());
  double lam = 2.0;
  int hmax = 0;
  int64_t n_med = 0, n_heavy = 0;
  if (n_out > 0) {
    hipLaunchKernelGGL(degrees, dim3(grid_for(n_out)), dim3(kBlock), 0, s, n_out, out->rowptr, wts, b.deg,
                       b.maxcount);
    hipLaunchKernelGGL(node_scales, dim3(grid_for(n_out)), dim3(kBlock), 0, s, n_out, kind, b.deg, out->scale,
                       out->diag, b.sd);
    SPED_CHECK_HIP(hipGetLastError());
    if (nnz > 0) {
      hipLaunchKernelGGL(entry_values, dim3(grid_for(nnz)), dim3(kBlock), 0, s, nnz, kind, keys, wts, b.sd, out->col,
                         out->val);
      hipLaunchKernelGGL(reverse_positions, dim3(grid_for(nnz)), dim3(kBlock), 0, s, nnz, keys, out->rowptr,
                         out->rev);
      SPED_CHECK_HIP(hipGetLastError());
    }
    if (out->wentry && nnz > 0) {
      hipLaunchKernelGGL(walk_entry_records, dim3(grid_for(nnz)), dim3(kBlock), 0, s, nnz, out->rowptr, out->col,
                         out->val, out->rev, out->scale, out->wentry);
      SPED_CHECK_HIP(hipGetLastError());
    }
    if (out->wnode) {
      hipLaunchKernelGGL(walk_node_records, dim3(grid_for(n_out)), dim3(kBlock), 0, s, n_out, out->rowptr,
                         out->scale, out->wnode);
      SPED_CHECK_HIP(hipGetLastError());
    }
    size_t tb = b.temp_bytes;
    SPED_CHECK_HIP(hipcub::DeviceReduce::Max(b.temp, tb, b.deg, b.dmax, n_out, s));
    hipLaunchKernelGGL(bin_flags, dim3(grid_for(n_out)), dim3(kBlock), 0, s, n_out, out->rowptr, b.fmed, b.fheavy);
    SPED_CHECK_HIP(hipGetLastError());
    hipcub::CountingInputIterator<int32_t> rows(0);
    tb = b.temp_bytes;
    SPED_CHECK_HIP(hipcub::DeviceSelect::Flagged(b.temp, tb, rows, b.fmed, out->bins, b.nsel, n_out, s));
    SPED_CHECK_HIP(hipMemcpyAsync(&n_med, b.nsel, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPED_CHECK_HIP(hipStreamSynchronize(s));
    tb = b.temp_bytes;
    SPED_CHECK_HIP(hipcub::DeviceSelect::Flagged(b.temp, tb, rows, b.fheavy, out->bins + n_med, b.nsel + 1, n_out, s));
    double dmax = 0.0;
    SPED_CHECK_HIP(hipMemcpyAsync(&n_heavy, b.nsel + 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPED_CHECK_HIP(hipMemcpyAsync(&dmax, b.dmax, sizeof(double), hipMemcpyDeviceToHost, s));
    SPED_CHECK_HIP(hipMemcpyAsync(&hmax, b.maxcount, sizeof(int), hipMemcpyDeviceToHost, s));
    SPED_CHECK_HIP(hipStreamSynchronize(s));
    lam = kind == SPED_LAP_SYM_NORMALIZED ? 2.0 : 2.0 * dmax;
    hipLaunchKernelGGL(light_work, dim3(grid_for(n_out + 1)), dim3(kBlock), 0, s, n_out, out->rowptr, b.flags);
    SPED_CHECK_HIP(hipGetLastError());
    tb = b.temp_bytes;
    SPED_CHECK_HIP(hipcub::DeviceScan::ExclusiveSum(b.temp, tb, b.flags, b.pos, n_out + 1, s));
    hipLaunchKernelGGL(xcd_splits, dim3(1), dim3(64), 0, s, n_out, b.pos, b.splits);
    SPED_CHECK_HIP(hipGetLastError());
    SPED_CHECK_HIP(hipMemcpyAsync(out->xcd_rows, b.splits, (kXcds + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  } else {
    for (int x = 0; x <= kXcds; ++x) out->xcd_rows[x] = 0;
  }
  SPED_CHECK_HIP(hipStreamSynchronize(s));
  out->n = n_out;
  out->nnz = nnz;
  out->n_medium = n_med;
  out->n_heavy = n_heavy;
  out->max_degree = hmax;
  out->kind = kind;
  out->lambda_bound = lam;
  return SPED_OK;
}
