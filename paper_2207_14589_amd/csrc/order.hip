// Node orders for gather locality, and the Laplacian built in such an order.
//
// p(L)V (Sec. 4.2) is the same operator under any relabelling of the nodes,
// with the rows of V permuted alike; the paper fixes no order.  Placing the
// neighbours of a node at nearby ids makes the neighbour-row gathers of the
// sparse products land on fewer distinct cache lines.
//
// Cuthill-McKee on the device: a level-synchronous breadth-first search.  The
// queue form appends the unvisited neighbours of each dequeued node by
// increasing (degree, id); a node is appended by its earliest-placed
// neighbour, which lies in the previous level.  So each level is the set of
// nodes first reached from the previous one, sorted by (position of the
// earliest-placed neighbour, degree, id): one wavefront per frontier node
// takes atomicMin of its position over its unplaced neighbours (the first to
// lower a neighbour's key appends it to the level's list), then two stable
// radix sorts (by id, then by (key, degree)) fix the level's order.  The
// result does not depend on the order of the atomics.  Nodes outside the
// search's component follow in increasing id.
//
// Label propagation (Raghavan, Albert and Kumara 2007), synchronous: every
// node starts with its id as label; a round gives every node with neighbours
// the label most frequent among its stored neighbours' labels of the previous
// round, ties going to the smallest splitmix64 output of (label XOR (round +
// 1) << 32); at most kLpRounds rounds, stopping after a round that changes no
// label.  A round sorts the (row, neighbour label) keys of all stored entries
// (one radix sort; rows stay in their CSR ranges); an inclusive max-scan of
// the run-start positions gives every entry the start of its run, so the
// thread at each run's last entry knows the run's length without walking
// it; three passes over the runs then take, per row, the largest count
// (atomicMax), the smallest tie-break key among the runs of that count
// (atomicMin), and the label of the run that holds both: the atomics' order
// does not matter.  The order groups the nodes by
// final label (increasing), inside a group by decreasing degree, then
// increasing id: one stable radix sort of (label, ~degree) keys with the ids
// as values.

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>

#include "common.h"

namespace sped {
namespace {

constexpr int kOB = 256;
inline unsigned oblocks(int64_t n) { return unsigned(std::max<int64_t>(1, (n + kOB - 1) / kOB)); }

int bits_for(uint64_t v) {  // smallest b with v < 2^b
  int b = 0;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

__global__ void fill_i32(int64_t n, int32_t *__restrict__ a, int32_t v) {
  const int64_t i = int64_t(blockIdx.x) * kOB + threadIdx.x;
  if (i < n) a[i] = v;
}

// largest (degree, -id): key = degree << 32 | (2^32 - 1 - id)
__global__ void root_key(int64_t n, const int64_t *__restrict__ rowptr, unsigned long long *__restrict__ best) {
  __shared__ unsigned long long red[kOB];
  const int64_t i = int64_t(blockIdx.x) * kOB + threadIdx.x;
  unsigned long long key = 0;
  if (i < n)
    key = (static_cast<unsigned long long>(rowptr[i + 1] - rowptr[i]) << 32) | (0xFFFFFFFFull - uint64_t(i));
  red[threadIdx.x] = key;
  __syncthreads();
  for (int h = kOB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(best, red[0]);
}

__global__ void place_root(const unsigned long long *__restrict__ best, int32_t *__restrict__ pos,
                           int32_t *__restrict__ order) {
  const int32_t r = int32_t(0xFFFFFFFFull - (*best & 0xFFFFFFFFull));
  pos[r] = 0;
  order[0] = r;
}

// One wavefront per frontier node (positions lo .. lo + cnt - 1).
__global__ __launch_bounds__(kOB) void expand_level(int64_t lo, int64_t cnt, const int32_t *__restrict__ order,
                                                    const int64_t *__restrict__ rowptr,
                                                    const int32_t *__restrict__ col, const int32_t *__restrict__ pos,
                                                    int32_t *__restrict__ pkey, int32_t *__restrict__ cand,
                                                    int32_t *__restrict__ ncand) {
  const int64_t f = int64_t(blockIdx.x) * (kOB / 64) + threadIdx.x / 64;
  if (f >= cnt) return;
  const int lane = threadIdx.x & 63;
  const int32_t q = int32_t(lo + f);
  const int32_t v = order[q];
  const int64_t end = rowptr[v + 1];
  for (int64_t e = rowptr[v] + lane; e < end; e += 64) {
    const int32_t u = col[e];
    // a key already at or below q needs no atomic (the node is claimed; a
    // stale read only costs an atomic that changes nothing)
    if (pos[u] < 0 && __hip_atomic_load(&pkey[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > q) {
      const int32_t old = atomicMin(&pkey[u], q);
      if (old == INT_MAX) cand[atomicAdd(ncand, 1)] = u;
    }
  }
}

// (earliest-placed neighbour's position - lo) << dbits | degree
__global__ void level_keys(int64_t cnt, int64_t lo, int dbits, const int32_t *__restrict__ ids,
                           const int32_t *__restrict__ pkey, const int64_t *__restrict__ rowptr,
                           uint64_t *__restrict__ keys) {
  const int64_t i = int64_t(blockIdx.x) * kOB + threadIdx.x;
  if (i >= cnt) return;
  const int32_t u = ids[i];
  keys[i] = (uint64_t(int64_t(pkey[u]) - lo) << dbits) | uint64_t(rowptr[u + 1] - rowptr[u]);
}

__global__ void place_run(int64_t cnt, int64_t base, const int32_t *__restrict__ ids, int32_t *__restrict__ pos,
                          int32_t *__restrict__ order) {
  const int64_t i = int64_t(blockIdx.x) * kOB + threadIdx.x;
  if (i >= cnt) return;
  const int32_t u = ids[i];
  pos[u] = int32_t(base + i);
  order[base + i] = u;
}

__global__ void unplaced_flags(int64_t n, const int32_t *__restrict__ pos, char *__restrict__ flags) {
  const int64_t i = int64_t(blockIdx.x) * kOB + threadIdx.x;
  if (i < n) flags[i] = pos[i] < 0;
}

// descending degree as an ascending key; ids 0..n-1 as values
__global__ void degree_keys(int64_t n, const int64_t *__restrict__ rowptr, uint32_t *__restrict__ keys,
                            int32_t *__restrict__ ids) {
  const int64_t i = int64_t(blockIdx.x) * kOB + threadIdx.x;
  if (i >= n) return;
  keys[i] = ~uint32_t(rowptr[i + 1] - rowptr[i]);
  ids[i] = int32_t(i);
}

constexpr int kLpRounds = 16;

// The output function of splitmix64 (Steele, Lea and Flood, OOPSLA 2014).
__device__ inline uint64_t mix64(uint64_t x) {
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void iota_i32(int64_t n, int32_t *__restrict__ a) {
  const int64_t i = int64_t(blockIdx.x) * kOB + threadIdx.x;
  if (i < n) a[i] = int32_t(i);
}

// (row << lbits) | label of the entry's neighbour, for every stored entry;
// groups of 16 lanes per row, grid-stride over the rows
constexpr int kLpGroup = 16;
__global__ __launch_bounds__(kOB) void lp_keys(int64_t n, int lbits, const int64_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col, const int32_t *__restrict__ lab,
                                               uint64_t *__restrict__ keys) {
  const int lig = threadIdx.x & (kLpGroup - 1);
  const int64_t groups = int64_t(gridDim.x) * (kOB / kLpGroup);
  for (int64_t r = int64_t(blockIdx.x) * (kOB / kLpGroup) + threadIdx.x / kLpGroup; r < n; r += groups) {
    const int64_t end = rowptr[r + 1];
    for (int64_t e = rowptr[r] + lig; e < end; e += kLpGroup)
      keys[e] = (uint64_t(r) << lbits) | uint64_t(uint32_t(lab[col[e]]));
  }
}

// Per node: no count yet, the largest tie-break key, the label kept.
__global__ void lp_reset(int64_t n, const int32_t *__restrict__ lab, int32_t *__restrict__ nlab,
                         int32_t *__restrict__ bestcnt, uint64_t *__restrict__ besth) {
  const int64_t u = int64_t(blockIdx.x) * kOB + threadIdx.x;
  if (u >= n) return;
  nlab[u] = lab[u];
  bestcnt[u] = 0;
  besth[u] = ~uint64_t(0);
}

__device__ inline bool run_start(const uint64_t *__restrict__ keys, int64_t p) {
  return p == 0 || keys[p - 1] != keys[p];
}

// info[p] = p at the first entry of each run of equal sorted keys, 0
// elsewhere; an inclusive max-scan then leaves each entry its run's start.
__global__ void lp_mark(int64_t nnz, const uint64_t *__restrict__ keys, uint64_t *__restrict__ info) {
  const int64_t p = int64_t(blockIdx.x) * kOB + threadIdx.x;
  if (p < nnz) info[p] = run_start(keys, p) ? uint64_t(p) : 0;
}

// Lanes of a wavefront cover consecutive sorted entries, so the lanes of one
// row are contiguous: an inclusive segmented scan over lanes of equal row
// leaves the row's maximum (minimum) in its last lane, which alone touches
// the row's slot.  Every lane takes part (inactive ones with the neutral
// value and a row id of their own).
__device__ inline int32_t seg_max_i32(int32_t v, int64_t row, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t vo = __shfl_up(v, off, 64);
    const int64_t ro = __shfl_up(row, off, 64);
    if (lane >= off && ro == row) v = max(v, vo);
  }
  return v;
}
__device__ inline unsigned long long seg_min_u64(unsigned long long v, int64_t row, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long vo = __shfl_up(v, off, 64);
    const int64_t ro = __shfl_up(row, off, 64);
    if (lane >= off && ro == row && vo < v) v = vo;
  }
  return v;
}
__device__ inline bool seg_last(int64_t row, int lane) {
  const int64_t rn = __shfl_down(row, 1, 64);
  return lane == 63 || rn != row;
}

// The thread at the last entry of each run reads the run's start from the
// scanned info, stores (count << 32 | label) at info[start] (the only slot
// of the run read later: the passes below read run starts only); the row's
// largest count goes to bestcnt through one atomicMax per row and wavefront,
// skipped when a read shows it would change nothing (a hub's row has
// thousands of runs, all of count 1 in the first round).
__global__ __launch_bounds__(kOB) void lp_count(int64_t nnz, int lbits, const uint64_t *__restrict__ keys,
                                                uint64_t *__restrict__ info, int32_t *__restrict__ bestcnt) {
  const int64_t p = int64_t(blockIdx.x) * kOB + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int32_t cnt = 0;
  int64_t row = -1 - int64_t(lane);  // distinct for lanes past the end
  if (p < nnz) {
    const uint64_t k = keys[p];
    row = int64_t(k >> lbits);
    if (p + 1 >= nnz || keys[p + 1] != k) {  // the run's last entry
      const int64_t start = int64_t(info[p]);
      cnt = int32_t(p - start + 1);
      const uint64_t mask = (uint64_t(1) << lbits) - 1;
      info[start] = (uint64_t(cnt) << 32) | (k & mask);
    }
  }
  const int32_t m = seg_max_i32(cnt, row, lane);
  if (p < nnz && seg_last(row, lane) && m > 0) {
    int32_t *slot = &bestcnt[row];
    if (m > __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(slot, m);
  }
}

// Runs of the row's largest count: the smallest tie-break key, one guarded
// atomicMin per row and wavefront as in lp_count.
__global__ __launch_bounds__(kOB) void lp_ties(int64_t nnz, int lbits, const uint64_t *__restrict__ keys,
                                               const uint64_t *__restrict__ info,
                                               const int32_t *__restrict__ bestcnt,
                                               unsigned long long *__restrict__ besth, uint64_t salt) {
  const int64_t p = int64_t(blockIdx.x) * kOB + threadIdx.x;
  const int lane = threadIdx.x & 63;
  unsigned long long h = ~0ull;
  int64_t row = -1 - int64_t(lane);
  if (p < nnz) {
    row = int64_t(keys[p] >> lbits);
    if (run_start(keys, p)) {
      const uint64_t v = info[p];
      if (int32_t(v >> 32) == bestcnt[row]) h = static_cast<unsigned long long>(mix64((v & 0xFFFFFFFFull) ^ salt));
    }
  }
  const unsigned long long m = seg_min_u64(h, row, lane);
  if (p < nnz && seg_last(row, lane) && m != ~0ull &&
      m < __hip_atomic_load(&besth[row], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMin(&besth[row], m);
}

// The run holding both the largest count and the smallest key (one per row:
// labels differ inside a row and mix64 is a bijection) sets the new label.
__global__ void lp_pick(int64_t nnz, int lbits, const uint64_t *__restrict__ keys, const uint64_t *__restrict__ info,
                        const int32_t *__restrict__ bestcnt, const uint64_t *__restrict__ besth,
                        const int32_t *__restrict__ lab, int32_t *__restrict__ nlab, uint64_t salt,
                        int32_t *__restrict__ changed) {
  const int64_t p = int64_t(blockIdx.x) * kOB + threadIdx.x;
  if (p >= nnz || !run_start(keys, p)) return;
  const uint64_t v = info[p];
  const int32_t cnt = int32_t(v >> 32);
  const int64_t row = int64_t(keys[p] >> lbits);
  const uint64_t l = v & 0xFFFFFFFFull;
  if (cnt == bestcnt[row] && mix64(l ^ salt) == besth[row]) {
    nlab[row] = int32_t(l);
    if (int32_t(l) != lab[row]) *changed = 1;
  }
}

// (label << 32) | ~degree, and the ids 0 .. n-1 as values
__global__ void lp_order_keys(int64_t n, const int64_t *__restrict__ rowptr, const int32_t *__restrict__ lab,
                              uint64_t *__restrict__ keys, int32_t *__restrict__ ids) {
  const int64_t i = int64_t(blockIdx.x) * kOB + threadIdx.x;
  if (i >= n) return;
  keys[i] = (uint64_t(uint32_t(lab[i])) << 32) | uint64_t(~uint32_t(rowptr[i + 1] - rowptr[i]));
  ids[i] = int32_t(i);
}

struct OrderWs {
  int32_t *pkey, *order, *cand, *candS, *ids2;
  uint64_t *k2, *k2s;
  uint32_t *k32, *k32s;
  char *flags;
  int32_t *ncand;
  int64_t *nsel;
  unsigned long long *best;
  // label propagation only (NULL otherwise): entry keys and their sorted
  // copy, the labels of two rounds
  uint64_t *ek, *eks;
  int32_t *lab, *nlab;
  void *temp;
  size_t temp_bytes;
};

size_t order_temp_bytes(int64_t n) {
  const int64_t c = n > 0 ? n : 1;
  size_t a = 0, b = 0, d = 0, e = 0;
  (void)hipcub::DeviceRadixSort::SortKeys(nullptr, a, (uint32_t *)nullptr, (uint32_t *)nullptr, c);
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b, (uint64_t *)nullptr, (uint64_t *)nullptr, (int32_t *)nullptr,
                                     (int32_t *)nullptr, c);
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, d, (uint32_t *)nullptr, (uint32_t *)nullptr, (int32_t *)nullptr,
                                     (int32_t *)nullptr, c);
  hipcub::CountingInputIterator<int32_t> ids(0);
  (void)hipcub::DeviceSelect::Flagged(nullptr, e, ids, (char *)nullptr, (int32_t *)nullptr, (int64_t *)nullptr, c);
  return std::max(std::max(a, b), std::max(d, e));
}

// keys of label propagation's entry sort: (row << lbits) | label
inline int lp_label_bits(int64_t n) { return std::max(bits_for(uint64_t(n)), 1); }

size_t lp_temp_bytes(int64_t n, int64_t nnz) {
  size_t a = 0, b = 0;
  const int bits = 2 * lp_label_bits(n);
  const int64_t items = nnz > 0 ? nnz : int64_t(1);
  (void)hipcub::DeviceRadixSort::SortKeys(nullptr, a, (uint64_t *)nullptr, (uint64_t *)nullptr, items, 0, bits);
  (void)hipcub::DeviceScan::InclusiveScan(nullptr, b, (uint64_t *)nullptr, hipcub::Max(), items);
  return std::max(a, b);
}

// With lp, the arrays of label propagation: the labels of two rounds (n
// each, also when L has no entries) and two keys per stored entry (nnz_lp,
// at least 1); the other methods need none of them.
OrderWs carve_order(Carver &c, int64_t n, bool lp = false, int64_t nnz_lp = 0) {
  const int64_t m = n > 0 ? n : 1;
  OrderWs o;
  o.pkey = c.take<int32_t>(m);
  o.order = c.take<int32_t>(m);
  o.cand = c.take<int32_t>(m);
  o.candS = c.take<int32_t>(m);
  o.ids2 = c.take<int32_t>(m);
  o.k2 = c.take<uint64_t>(m);
  o.k2s = c.take<uint64_t>(m);
  o.k32 = reinterpret_cast<uint32_t *>(o.k2);  // the degree order reuses the 64-bit key arrays
  o.k32s = reinterpret_cast<uint32_t *>(o.k2s);
  o.flags = c.take<char>(m);
  o.ncand = c.take<int32_t>(1);
  o.nsel = c.take<int64_t>(1);
  o.best = c.take<unsigned long long>(1);
  o.ek = o.eks = nullptr;
  o.lab = o.nlab = nullptr;
  o.temp_bytes = order_temp_bytes(n);
  if (lp) {
    const int64_t e = nnz_lp > 0 ? nnz_lp : 1;
    o.ek = c.take<uint64_t>(e);
    o.eks = c.take<uint64_t>(e);
    o.lab = c.take<int32_t>(m);
    o.nlab = c.take<int32_t>(m);
    o.temp_bytes = std::max(o.temp_bytes, lp_temp_bytes(n, e));
  }
  o.temp = c.take<char>(o.temp_bytes);
  return o;
}

sped_status cuthill_mckee(const sped_csr *L, int32_t *pos, const OrderWs &o, hipStream_t s) {
  const int64_t n = L->n;
  hipLaunchKernelGGL(fill_i32, dim3(oblocks(n)), dim3(kOB), 0, s, n, pos, int32_t(-1));
  hipLaunchKernelGGL(fill_i32, dim3(oblocks(n)), dim3(kOB), 0, s, n, o.pkey, int32_t(INT_MAX));
  SPED_CHECK_HIP(hipMemsetAsync(o.best, 0, sizeof(unsigned long long), s));
  hipLaunchKernelGGL(root_key, dim3(oblocks(n)), dim3(kOB), 0, s, n, L->rowptr, o.best);
  hipLaunchKernelGGL(place_root, dim3(1), dim3(1), 0, s, o.best, pos, o.order);
  SPED_CHECK_HIP(hipGetLastError());
  unsigned long long best = 0;  // its high half is the largest degree
  SPED_CHECK_HIP(hipMemcpyAsync(&best, o.best, sizeof(best), hipMemcpyDeviceToHost, s));
  SPED_CHECK_HIP(hipStreamSynchronize(s));
  const int dbits = bits_for(best >> 32);
  const int idbits = bits_for(uint64_t(n));
  int64_t lo = 0, hi = 1;
  while (lo < hi) {
    const int64_t cnt = hi - lo;
    SPED_CHECK_HIP(hipMemsetAsync(o.ncand, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(expand_level, dim3(unsigned((cnt + kOB / 64 - 1) / (kOB / 64))), dim3(kOB), 0, s, lo, cnt,
                       o.order, L->rowptr, L->col, pos, o.pkey, o.cand, o.ncand);
    SPED_CHECK_HIP(hipGetLastError());
    int32_t found = 0;
    SPED_CHECK_HIP(hipMemcpyAsync(&found, o.ncand, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SPED_CHECK_HIP(hipStreamSynchronize(s));
    if (found <= 0) break;
    if (hi + found > n) return fail(SPED_E_INVALID, "adjacency is not symmetric or has repeated entries");
    size_t tb = o.temp_bytes;
    SPED_CHECK_HIP(hipcub::DeviceRadixSort::SortKeys(o.temp, tb, reinterpret_cast<uint32_t *>(o.cand),
                                                     reinterpret_cast<uint32_t *>(o.candS), found, 0,
                                                     std::max(idbits, 1), s));
    const int kbits = bits_for(uint64_t(cnt - 1)) + dbits;
    hipLaunchKernelGGL(level_keys, dim3(oblocks(found)), dim3(kOB), 0, s, int64_t(found), lo, dbits, o.candS, o.pkey,
                       L->rowptr, o.k2);
    SPED_CHECK_HIP(hipGetLastError());
    tb = o.temp_bytes;
    SPED_CHECK_HIP(hipcub::DeviceRadixSort::SortPairs(o.temp, tb, o.k2, o.k2s, o.candS, o.ids2, found, 0,
                                                      std::max(kbits, 1), s));
    hipLaunchKernelGGL(place_run, dim3(oblocks(found)), dim3(kOB), 0, s, int64_t(found), hi, o.ids2, pos, o.order);
    SPED_CHECK_HIP(hipGetLastError());
    lo = hi;
    hi += found;
  }
  if (hi < n) {  // nodes outside the searched component, in increasing id
    hipLaunchKernelGGL(unplaced_flags, dim3(oblocks(n)), dim3(kOB), 0, s, n, pos, o.flags);
    SPED_CHECK_HIP(hipGetLastError());
    hipcub::CountingInputIterator<int32_t> ids(0);
    size_t tb = o.temp_bytes;
    SPED_CHECK_HIP(hipcub::DeviceSelect::Flagged(o.temp, tb, ids, o.flags, o.cand, o.nsel, n, s));
    hipLaunchKernelGGL(place_run, dim3(oblocks(n - hi)), dim3(kOB), 0, s, n - hi, hi, o.cand, pos, o.order);
    SPED_CHECK_HIP(hipGetLastError());
  }
  SPED_CHECK_HIP(hipStreamSynchronize(s));
  return SPED_OK;
}

sped_status degree_order(const sped_csr *L, int32_t *pos, const OrderWs &o, hipStream_t s) {
  const int64_t n = L->n;
  hipLaunchKernelGGL(degree_keys, dim3(oblocks(n)), dim3(kOB), 0, s, n, L->rowptr, o.k32, o.cand);
  SPED_CHECK_HIP(hipGetLastError());
  size_t tb = o.temp_bytes;
  SPED_CHECK_HIP(hipcub::DeviceRadixSort::SortPairs(o.temp, tb, o.k32, o.k32s, o.cand, o.candS, n, 0, 32, s));
  hipLaunchKernelGGL(place_run, dim3(oblocks(n)), dim3(kOB), 0, s, n, int64_t(0), o.candS, pos, o.order);
  SPED_CHECK_HIP(hipGetLastError());
  SPED_CHECK_HIP(hipStreamSynchronize(s));
  return SPED_OK;
}

sped_status label_order(const sped_csr *L, int32_t *pos, const OrderWs &o, hipStream_t s) {
  const int64_t n = L->n, nnz = L->nnz;
  if (!o.lab || !o.nlab || !o.ek || !o.eks) return fail(SPED_E_INVALID, "label propagation workspace not carved");
  const int lbits = lp_label_bits(n);
  int32_t *lab = o.lab, *nlab = o.nlab;
  hipLaunchKernelGGL(iota_i32, dim3(oblocks(n)), dim3(kOB), 0, s, n, lab);
  SPED_CHECK_HIP(hipGetLastError());
  const unsigned kblocks = unsigned(std::min<int64_t>(8192, std::max<int64_t>(1, (n + kOB / kLpGroup - 1) /
                                                                                   (kOB / kLpGroup))));
  for (int r = 0; r < kLpRounds && nnz > 0; ++r) {
    hipLaunchKernelGGL(lp_keys, dim3(kblocks), dim3(kOB), 0, s, n, lbits, L->rowptr, L->col, lab, o.ek);
    SPED_CHECK_HIP(hipGetLastError());
    size_t tb = o.temp_bytes;
    SPED_CHECK_HIP(hipcub::DeviceRadixSort::SortKeys(o.temp, tb, o.ek, o.eks, nnz, 0, 2 * lbits, s));
    const uint64_t salt = uint64_t(r + 1) << 32;
    // per-row maxima in arrays this method leaves free: the search keys
    // (int32 [n]) and the 64-bit level keys (uint64 [n])
    int32_t *bestcnt = o.pkey;
    uint64_t *besth = o.k2;
    SPED_CHECK_HIP(hipMemsetAsync(o.ncand, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(lp_reset, dim3(oblocks(n)), dim3(kOB), 0, s, n, lab, nlab, bestcnt, besth);
    hipLaunchKernelGGL(lp_mark, dim3(oblocks(nnz)), dim3(kOB), 0, s, nnz, o.eks, o.ek);
    SPED_CHECK_HIP(hipGetLastError());
    tb = o.temp_bytes;
    SPED_CHECK_HIP(hipcub::DeviceScan::InclusiveScan(o.temp, tb, o.ek, hipcub::Max(), nnz, s));
    hipLaunchKernelGGL(lp_count, dim3(oblocks(nnz)), dim3(kOB), 0, s, nnz, lbits, o.eks, o.ek, bestcnt);
    hipLaunchKernelGGL(lp_ties, dim3(oblocks(nnz)), dim3(kOB), 0, s, nnz, lbits, o.eks, o.ek, bestcnt,
                       reinterpret_cast<unsigned long long *>(besth), salt);
    hipLaunchKernelGGL(lp_pick, dim3(oblocks(nnz)), dim3(kOB), 0, s, nnz, lbits, o.eks, o.ek, bestcnt, besth, lab,
                       nlab, salt, o.ncand);
    SPED_CHECK_HIP(hipGetLastError());
    int32_t changed = 0;
    SPED_CHECK_HIP(hipMemcpyAsync(&changed, o.ncand, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SPED_CHECK_HIP(hipStreamSynchronize(s));
    if (!changed) break;  // nlab equals lab
    std::swap(lab, nlab);
  }
  // stable sort of (label, ~degree) with the ids (increasing) as values;
  // the 64-bit key arrays are free again after the rounds
  hipLaunchKernelGGL(lp_order_keys, dim3(oblocks(n)), dim3(kOB), 0, s, n, L->rowptr, lab, o.k2, o.cand);
  SPED_CHECK_HIP(hipGetLastError());
  size_t tb = o.temp_bytes;
  SPED_CHECK_HIP(hipcub::DeviceRadixSort::SortPairs(o.temp, tb, o.k2, o.k2s, o.cand, o.candS, n, 0, 32 + lbits, s));
  hipLaunchKernelGGL(place_run, dim3(oblocks(n)), dim3(kOB), 0, s, n, int64_t(0), o.candS, pos, o.order);
  SPED_CHECK_HIP(hipGetLastError());
  SPED_CHECK_HIP(hipStreamSynchronize(s));
  return SPED_OK;
}

sped_status run_order(const sped_csr *L, int32_t method, int32_t *pos, const OrderWs &o, hipStream_t s) {
  if (L->n == 0) return SPED_OK;
  if (method == SPED_ORDER_LABEL_PROPAGATION) return label_order(L, pos, o, s);
  return method == SPED_ORDER_CUTHILL_MCKEE ? cuthill_mckee(L, pos, o, s) : degree_order(L, pos, o, s);
}

bool known_method(int32_t method) {
  return method == SPED_ORDER_CUTHILL_MCKEE || method == SPED_ORDER_DEGREE || method == SPED_ORDER_LABEL_PROPAGATION;
}

// map[old_of_new1[i]] = pos[i] for the kept nodes; -1 elsewhere
__global__ void scatter_kept(int64_t n1, const int32_t *__restrict__ old_of_new1, const int32_t *__restrict__ pos,
                             int32_t *__restrict__ map) {
  const int64_t i = int64_t(blockIdx.x) * kOB + threadIdx.x;
  if (i < n1) map[old_of_new1[i]] = pos[i];
}

// Kept edges take their endpoints' positions; an edge of a dropped component
// becomes the self-loop (0, 0), which the build ignores; endpoints outside
// [0, n) are left as they are, for the build to reject.
__global__ void relabel(int64_t m, int64_t n, const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                        const int32_t *__restrict__ map, int32_t *__restrict__ src2, int32_t *__restrict__ dst2) {
  const int64_t e = int64_t(blockIdx.x) * kOB + threadIdx.x;
  if (e >= m) return;
  const int32_t a = src[e], b = dst[e];
  int32_t a2 = (a >= 0 && a < n) ? map[a] : a;
  int32_t b2 = (b >= 0 && b < n) ? map[b] : b;
  if ((a >= 0 && a < n && a2 < 0) || (b >= 0 && b < n && b2 < 0)) a2 = b2 = 0;
  src2[e] = a2;
  dst2[e] = b2;
}

__global__ void compose_old(int64_t n1, const int32_t *__restrict__ old_of_new1, const int32_t *__restrict__ pos,
                            int32_t *__restrict__ old_of_new) {
  const int64_t i = int64_t(blockIdx.x) * kOB + threadIdx.x;
  if (i < n1) old_of_new[pos[i]] = old_of_new1[i];
}

// the build's workspace size (a size query: nothing runs)
size_t build_ws_bytes(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t kind) {
  size_t b = 0;
  sped_csr probe{};
  sped_laplacian_csr(n, m, src, dst, nullptr, kind, 0, &probe, nullptr, nullptr, &b, nullptr);
  return b;
}

}  // namespace
}  // namespace sped

using namespace sped;

extern "C" sped_status sped_locality_order(const sped_csr *L, int32_t method, int32_t *new_of_old, void *ws,
                                           size_t *ws_bytes, sped_stream_t stream) {
  clear_error();
  if (!known_method(method)) return fail(SPED_E_INVALID, "method");
  if (!L) return fail(SPED_E_INVALID, "L NULL");
  if (L->n < 0 || L->n >= (int64_t(1) << 31) - 1) return fail(SPED_E_INVALID, "n outside [0, 2^31 - 1)");
  if (L->nnz < 0) return fail(SPED_E_INVALID, "nnz < 0");
  Carver c(ws);
  const bool lp = method == SPED_ORDER_LABEL_PROPAGATION;
  const OrderWs o = carve_order(c, L->n, lp, lp ? L->nnz : 0);
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, c.bytes(), &query));
  if (query) return SPED_OK;
  if (L->n > 0 && (!L->rowptr || !new_of_old || (L->nnz > 0 && !L->col))) return fail(SPED_E_INVALID, "NULL array");
  return run_order(L, method, new_of_old, o, as_stream(stream));
}

extern "C" sped_status sped_laplacian_csr_ordered(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                                                  const float *w, int32_t kind, int32_t lcc_only, int32_t method,
                                                  sped_csr *out, int32_t *old_of_new, void *ws, size_t *ws_bytes,
                                                  sped_stream_t stream) {
  clear_error();
  if (!known_method(method)) return fail(SPED_E_INVALID, "method");
  if (n < 0 || n >= (int64_t(1) << 31) - 1) return fail(SPED_E_INVALID, "n outside [0, 2^31 - 1)");
  if (m < 0 || m > (int64_t(1) << 40)) return fail(SPED_E_INVALID, "m out of range");
  if (m > 0 && (!src || !dst)) return fail(SPED_E_INVALID, "src/dst NULL");
  if (kind != SPED_LAP_COMBINATORIAL && kind != SPED_LAP_SYM_NORMALIZED) return fail(SPED_E_INVALID, "kind");
  if (!out) return fail(SPED_E_INVALID, "out NULL");
  // region A serves the two builds and the order in turn; region B holds the
  // relabelled edges and the maps between the three labellings.  The built
  // Laplacian stores at most 2m entries, which bounds label propagation's
  // entry arrays.
  const size_t a_bytes = std::max(build_ws_bytes(n, m, src, dst, kind), [&] {
    Carver t(nullptr);
    const bool lp = method == SPED_ORDER_LABEL_PROPAGATION;
    carve_order(t, n, lp, lp ? 2 * m : 0);
    return t.bytes();
  }());
  Carver c(ws);
  char *regionA = c.take<char>(a_bytes);
  int32_t *src2 = c.take<int32_t>(m > 0 ? m : 1);
  int32_t *dst2 = c.take<int32_t>(m > 0 ? m : 1);
  int32_t *oon1 = c.take<int32_t>(n > 0 ? n : 1);
  int32_t *pos = c.take<int32_t>(n > 0 ? n : 1);
  int32_t *map = c.take<int32_t>(n > 0 ? n : 1);
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, c.bytes(), &query));
  if (query) return SPED_OK;
  hipStream_t s = as_stream(stream);
  size_t ab = a_bytes;
  SPED_TRY(sped_laplacian_csr(n, m, src, dst, w, kind, lcc_only, out, oon1, regionA, &ab, stream));
  const int64_t n1 = out->n;
  if (n1 == 0) return SPED_OK;
  ab = a_bytes;
  SPED_TRY(sped_locality_order(out, method, pos, regionA, &ab, stream));
  SPED_CHECK_HIP(hipMemsetAsync(map, 0xFF, sizeof(int32_t) * n, s));  // -1: not kept
  hipLaunchKernelGGL(scatter_kept, dim3(oblocks(n1)), dim3(kOB), 0, s, n1, oon1, pos, map);
  SPED_CHECK_HIP(hipGetLastError());
  if (m > 0) {
    hipLaunchKernelGGL(relabel, dim3(oblocks(m)), dim3(kOB), 0, s, m, n, src, dst, map, src2, dst2);
    SPED_CHECK_HIP(hipGetLastError());
  }
  // The kept nodes now carry ids 0 .. n1-1 in the computed order and every
  // other edge is a self-loop: the second build takes all n1 nodes as they are.
  ab = a_bytes;
  SPED_TRY(sped_laplacian_csr(n1, m, src2, dst2, w, kind, 0, out, nullptr, regionA, &ab, stream));
  if (out->n != n1) return fail(SPED_E_INVALID, "reordered build kept a different node count");
  if (old_of_new) {
    hipLaunchKernelGGL(compose_old, dim3(oblocks(n1)), dim3(kOB), 0, s, n1, oon1, pos, old_of_new);
    SPED_CHECK_HIP(hipGetLastError());
  }
  SPED_CHECK_HIP(hipStreamSynchronize(s));
  return SPED_OK;
}
