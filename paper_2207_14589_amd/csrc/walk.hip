// Random-walk estimate of sum_i c_i L^i X (Sec. 4.3): the chains of
// eq. walk_summand are walks on the edge-incidence graph H (self-loops
// included); a walker's state is an edge of G, stored as its CSR position p in
// row a (the endpoint the walk last stood on) with other endpoint b = col[p].
//
// Incidence entries: for edge e = (a, b), h(e, a) = sign sqrt(w_e) s_a with
// sign +1 when a < b (Sec. 2 convention), and sqrt(w_e) s_a = sqrt(val s_a/s_b)
// because val = w_e s_a s_b.  Entries and inner products are float32; the
// walk weights (products of up to 16 factors) are float64.  Table 1 generalises to x_e^T x_f = h(e,u) h(f,u)
// for distinct edges meeting at u, and h(e,a)^2 + h(e,b)^2 for e = f.
//
// Moving from e = (a, b): draw t uniform in [0, d_a + d_b - 1); t < d_a picks
// entry t of row a (this includes e itself, the self-loop of H), otherwise
// entry t - d_a of row b with b's copy of e (position rev[p]) skipped.
//
// importance sampler: one lane group per output row; each lane of the group
// drives its own walk of that row and the group gathers X rows together; the
// walk weight
//   omega_1 = d_r h(e_1, r),   omega_{i+1} = omega_i (x_{e_i}^T x_{e_{i+1}}) deg_H(e_i)
// is alpha_c (x_{e_1})_r / q(c) for the proposal q, so each prefix adds
// c_i omega_i (x_{e_i}^T X) to row r; one store writes the row.  No atomics:
// the result is deterministic.
//
// rejection sampler: lane groups run trials; e_1 is uniform over the stored
// entries (each edge twice), prefix i is kept with probability
// prod_{t<i} deg_H(e_t) / (2 deg* - 1) (decided in float64 with the oracle's
// operation order) and contributes (|E|/N) prod_t (2deg*-1) x_et^T x_et+1 c_i
// x_{e_1} (x_{e_i}^T X), added to both endpoints of e_1 with float atomics.
#include <cmath>

#include "common.h"

namespace sped {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxDeg = 255;

// Polynomial coefficients travel by value in the kernel arguments (2 KiB), so
// concurrent calls with different polynomials never share state.
struct Coefs {
  double c[kMaxDeg + 1];
};

// A walker's current edge e = (a, b): CSR position p in row a, the row
// ranges of both endpoints, the square roots of their scales (r_u = sqrt(s_u))
// and the incidence entries h(e, a), h(e, b).  Kept in registers.
struct Edge {
  int64_t p;
  int64_t a0, a1, b0, b1;
  int32_t a, b;
  float ra, rb;
  float ha, hb;
};

struct Graph {
  const int64_t *rowptr;
  const sped_walk_entry *we;
  const sped_walk_node *wn;
};

// h(e, a) = sign sqrt(w_e) s_a with sqrt(w_e) s_a = sqrt(val) r_a / r_b
// (val = w_e s_a s_b), sign + when a < b.
__device__ inline void edge_entries(Edge &e, float val) {
  const float sv = sqrtf(val);
  const float ga = sv * (e.ra / e.rb);
  const float gb = sv * (e.rb / e.ra);
  const float sg = e.a < e.b ? 1.f : -1.f;
  e.ha = sg * ga;
  e.hb = -sg * gb;
}

// The walk state after picking entry p of row r (node record nr).  *rev_p
// receives the position of the edge's copy in the other endpoint's row.
__device__ inline Edge first_edge(const Graph &g, int32_t r, const sped_walk_node &nr, int64_t p, int64_t *rev_p) {
  const sped_walk_entry en = g.we[p];
  Edge e;
  e.p = p;
  e.a = r; e.a0 = nr.start; e.a1 = nr.start + nr.degree; e.ra = nr.root_scale;
  e.b = en.col; e.b0 = en.start; e.b1 = en.start + en.degree; e.rb = en.root_scale;
  edge_entries(e, en.val);
  *rev_p = en.start + en.rev_local;
  return e;
}

// Neighbour number t of e on H (t < deg_H(e) = d_a + d_b - 1): t < d_a picks
// entry t of row a (t = p - a0 is e itself, H's self-loop), otherwise entry
// t - d_a of row b, skipping b's copy of e at rev_p.  Returns the entry's CSR
// position; *fa tells whether it lies in row a.
__device__ inline int64_t pick(const Edge &e, uint32_t t, int64_t rev_p, bool *fa) {
  const int64_t da = e.a1 - e.a0;
  *fa = int64_t(t) < da;
  int64_t qb = e.b0 + (int64_t(t) - da);
  qb += qb >= rev_p ? 1 : 0;
  return *fa ? e.a0 + int64_t(t) : qb;
}

// Step from e to the edge f at position q (picked by `pick`, record en: one
// 32-byte load that carries the far endpoint's row range and scale); *rev_p
// is updated for f.  Returns x_e^T x_f.
__device__ inline float advance(Edge &e, int64_t q, bool fa, const sped_walk_entry &en, int64_t *rev_p) {
  const float dot_same = e.ha * e.ha + e.hb * e.hb;
  const float h_eu = fa ? e.ha : e.hb;
  Edge f;
  f.p = q;
  f.a = fa ? e.a : e.b;
  f.a0 = fa ? e.a0 : e.b0;
  f.a1 = fa ? e.a1 : e.b1;
  f.ra = fa ? e.ra : e.rb;
  f.b = en.col; f.b0 = en.start; f.b1 = en.start + en.degree; f.rb = en.root_scale;
  edge_entries(f, en.val);
  *rev_p = en.start + en.rev_local;
  const float dot = (q == e.p) ? dot_same : h_eu * f.ha;  // f.ha: entry of f at the shared node
  e = f;
  return dot;
}

__device__ inline float move(const Graph &g, Edge &e, uint32_t t, int64_t *rev_p) {
  bool fa;
  const int64_t q = pick(e, t, *rev_p, &fa);
  const sped_walk_entry en = g.we[q];
  return advance(e, q, fa, en, rev_p);
}

// Row gathers of up to 8 walks of a group: lane j of the group holds the
// weight w_j and node_j of walk j0 + j.  issue() starts the loads of
// X[node_j, c0 .. c0+VEC) for all 8 slots; consume() adds w_j times them to acc
// for the slots below nlive with nonzero weight.  Slots past nlive re-read a
// valid row of the group and are discarded.
template <typename TX, int VEC>
struct RowBatch {
  float w[8];
  float x[8][VEC];
  __device__ void issue(const TX *__restrict__ X, int64_t ldx, int cc, int G, int j0, float wl, int32_t node) {
    int32_t nj[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      w[u] = __shfl(wl, (j0 + u) & (G - 1), G);
      nj[u] = __shfl(node, (j0 + u) & (G - 1), G);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) VecIO<TX, VEC>::load(X + int64_t(nj[u]) * ldx + cc, x[u]);
  }
  __device__ void consume(bool col_ok, int j0, int nlive, float (&acc)[VEC]) const {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool use = col_ok && (j0 + u < nlive) && w[u] != 0.f;
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[v] = use ? fmaf(w[u], x[u][v], acc[v]) : acc[v];
    }
  }
};

template <typename TX, int VEC>
__device__ inline void gather_weighted_rows(const TX *__restrict__ X, int64_t ldx, int c0, bool col_ok, int G,
                                            int nlive, float w, int32_t node, float (&acc)[VEC]) {
  const int cc = col_ok ? c0 : 0;
  RowBatch<TX, VEC> rb;
  for (int j0 = 0; j0 < nlive; j0 += 8) {
    rb.issue(X, ldx, cc, G, j0, w, node);
    rb.consume(col_ok, j0, nlive, acc);
  }
}

// One group of G lanes owns output row r.  Lane j of the group drives the
// control path (random draws, index loads, weights) of walks j, j + G, ...
// so G walks advance in parallel; after each step the group gathers, for all
// of those walks at once, the X row of the node each walk just left (every
// lane its VEC columns) and adds them into the row's sum in walk order.  All
// walks of a row meet in the same registers: one store per row, no atomics.
// LDS the importance-walk launch reserves (and leaves unused) so that at most
// 3 of its 256-thread blocks share a CU (160 KB of LDS each): fewer walks in
// flight keep more of the active neighbourhoods' entry records and rows in
// cache.  On a clustered 1e6-node SBM this is 4% faster than the 4 blocks the
// registers allow; on a power-law graph with scattered communities it makes
// no difference.
constexpr int kWalkLdsReserve = 48 * 1024;

template <typename TX, typename TY, int VEC>
__global__ __launch_bounds__(kBlock) void walk_importance_kernel(
    int64_t n, int64_t nb, int k, int G, int lgG, Graph g, int ell, const TX *__restrict__ X, int64_t ldx,
    TY *__restrict__ Y, int64_t ldy, int64_t walks, uint32_t k0, uint32_t k1, uint32_t ctr, Coefs cf) {
  // each XCD takes a contiguous range of rows, so walks that stay near their
  // start (clustered graphs) reuse that XCD's L2
  const int64_t lb = xcd_logical_block(nb);
  if (lb >= nb) return;  // padding block (no barriers below)
  const int lig = threadIdx.x & (G - 1);
  const int64_t r = lb * (kBlock >> lgG) + (threadIdx.x >> lgG);
  const int c0 = blockIdx.y * 64 * VEC + lig * VEC;
  const bool col_ok = c0 < k;
  const bool row_ok = r < n;
  float acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = 0.f;
  sped_walk_node nr{0, 0, 0.f};
  if (row_ok) nr = g.wn[r];
  const int64_t r0 = nr.start;
  const int64_t dr = nr.degree;
  // every lane of a group sees the same dr, so the loops below are uniform per group
  if (dr > 0) {
    for (int64_t wbase = 0; wbase < walks; wbase += G) {
      const int64_t w = wbase + lig;
      const bool live = w < walks;
      const int nlive = int(min<int64_t>(G, walks - wbase));
      Edge e;
      double omega = 0.0;
      int64_t rev_p = 0;
      if (live) {
        uint32_t t0 = lemire_draw(k0, k1, uint32_t(r), uint32_t(w), ctr, 0u, uint32_t(dr));
        e = first_edge(g, int32_t(r), nr, r0 + t0, &rev_p);
        omega = double(dr) * double(e.ha);
      } else {
        e.a = e.b = int32_t(r);
        e.ha = e.hb = 0.f;
      }
      // Coefficients of X[e.a] and X[e.b] not yet gathered.  Consecutive edges
      // of a walk share a node, so a node's row is gathered once, when the
      // walk leaves it (and both at the end): one row gather per step.
      double pa = live ? cf.c[1] * omega * double(e.ha) : 0.0;
      double pb = live ? cf.c[1] * omega * double(e.hb) : 0.0;
      for (int i = 2; i <= ell + 1; ++i) {
        int32_t leave = e.a;
        double wleave = 0.0;
        if (i <= ell) {
          if (live) {
            uint32_t bound = uint32_t((e.a1 - e.a0) + (e.b1 - e.b0) - 1);
            uint32_t t = lemire_draw(k0, k1, uint32_t(r), uint32_t(w), ctr, uint32_t(i - 1), bound);
            const int32_t oa = e.a, ob = e.b;
            float dot = move(g, e, t, &rev_p);
            omega = omega * double(dot) * double(bound);
            const double ci = cf.c[i] * omega;
            if (e.a == oa && e.b == ob) {  // stayed on the same edge
              pa += ci * double(e.ha);
              pb += ci * double(e.hb);
            } else {                        // kept node e.a, left the other one
              const bool kept_a = e.a == oa;
              leave = kept_a ? ob : oa;
              wleave = kept_a ? pb : pa;
              pa = (kept_a ? pa : pb) + ci * double(e.ha);
              pb = ci * double(e.hb);
            }
          }
        } else {  // after the last prefix: flush both endpoints (second one below)
          leave = e.a;
          wleave = pa;
        }
        gather_weighted_rows<TX, VEC>(X, ldx, c0, col_ok, G, nlive, float(wleave), leave, acc);
      }
      gather_weighted_rows<TX, VEC>(X, ldx, c0, col_ok, G, nlive, float(pb), e.b, acc);
    }
  }
  if (row_ok && col_ok) {
    float x[VEC], o[VEC];
    VecIO<TX, VEC>::load(X + r * ldx + c0, x);
    const float inv = float(1.0 / double(walks));
    const float c0f = float(cf.c[0]);
#pragma unroll
    for (int v = 0; v < VEC; ++v) o[v] = fmaf(c0f, x[v], acc[v] * inv);
    VecIO<TY, VEC>::store(Y + r * ldy + c0, o);
  }
}

// ---------------------------------------------------------------- lazy node walks
// (I - L/l)^l X for the limit polynomial of Table 2 by lazy random walks on the
// nodes.  Normalised L: I - L/l = D^{1/2} P D^{-1/2}, P = (1 - 1/l) I +
// (1/l) D^{-1} A, so row r is E[s_Z X_Z] / s_r over the position Z after l
// lazy steps from r.  Combinatorial L with l >= max d: I - L/l is itself
// stochastic (move with probability d_z / l), row r is E[X_Z].  The stays
// between moves are drawn as geometric gaps (one draw per move).  A move picks a
// neighbour with probability proportional to w: up to 16 uniform proposals
// accepted with probability x_j / max x (x = S_ij / s_j or w_ij, float64 from
// the stored float32 values; ratios within 2^-20 of 1 count as 1), then an
// exact inverse-CDF draw over the row.  Weights are bounded by max s / min s,
// and each walk gathers one X row.
constexpr int kLazyAttempts = 16;
constexpr double kLazyEqual = 1.0 - 0x1.0p-20;

__device__ inline double lazy_x(int kind, const int32_t *__restrict__ col, const float *__restrict__ val,
                                const float *__restrict__ scale, int64_t p) {
  return kind == SPED_LAP_SYM_NORMALIZED ? double(val[p]) / double(scale[col[p]]) : double(val[p]);
}

// Per row: the largest move weight (one wavefront per row, lanes striding
// over the entries; the maximum does not depend on the order).
__global__ __launch_bounds__(kBlock) void lazy_row_max_kernel(int64_t n, int kind,
                                                              const int64_t *__restrict__ rowptr,
                                                              const int32_t *__restrict__ col,
                                                              const float *__restrict__ val,
                                                              const float *__restrict__ scale,
                                                              double *__restrict__ xmax) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = int64_t(gridDim.x) * (kBlock / 64);
  for (int64_t r = int64_t(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6); r < n; r += waves) {
    double m = 0.0;
    const int64_t e = rowptr[r + 1];
    for (int64_t p = rowptr[r] + lane; p < e; p += 64) m = fmax(m, lazy_x(kind, col, val, scale, p));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if (lane == 0) xmax[r] = m;
  }
}

template <typename TX, typename TY, int VEC>
__global__ __launch_bounds__(kBlock) void walk_lazy_kernel(
    int64_t n, int64_t nb, int k, int G, int lgG, int kind, const int64_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const float *__restrict__ val, const float *__restrict__ scale,
    const float *__restrict__ diag, const double *__restrict__ xmax, int ell,
    const TX *__restrict__ X, int64_t ldx, TY *__restrict__ Y, int64_t ldy, int64_t walks, uint32_t k0,
    uint32_t k1, uint32_t ctr) {
  const int64_t lb = xcd_logical_block(nb);
  if (lb >= nb) return;  // padding block (no barriers below)
  const int lig = threadIdx.x & (G - 1);
  const int64_t r = lb * (kBlock >> lgG) + (threadIdx.x >> lgG);
  const int c0 = blockIdx.y * 64 * VEC + lig * VEC;
  const bool col_ok = c0 < k;
  const bool row_ok = r < n;
  const int cc = col_ok ? c0 : 0;
  const bool norm = kind == SPED_LAP_SYM_NORMALIZED;
  const double inv_ell = 1.0 / double(ell);
  const double rs = row_ok ? double(scale[r]) : 1.0;
  float acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = 0.f;
  if (row_ok) {
    RowBatch<TX, VEC> rb;
    for (int64_t wbase = 0; wbase < walks; wbase += G) {
      const int64_t w = wbase + lig;
      const bool live = w < walks;
      const int nlive = int(min<int64_t>(G, walks - wbase));
      int32_t z = int32_t(r);
      if (live) {
        int64_t z0 = rowptr[z];
        int64_t dz = rowptr[z + 1] - z0;
        // The stays between moves are geometric: from node z the next move
        // comes after G = floor(log(1 - u) / log1p(-p_move(z))) more stays
        // (u the m-th gap draw), the same law as one Bernoulli draw per step,
        // at one draw per move.
        int t = 0;
        for (int m = 0; dz > 0; ++m) {  // an isolated node never moves
          const double pm = norm ? inv_ell : double(diag[z]) * inv_ell;
          const double u = uniform53(k0, k1, uint32_t(r), uint32_t(w), ctr, uint32_t(m));
          const double gap = floor(log(1.0 - u) / log1p(-pm));
          if (!(gap < double(ell - t))) break;  // no move within the remaining steps
          t += int(gap) + 1;                     // the move happens at step t
          int64_t chosen = -1;
          for (int a = 0; a < kLazyAttempts && chosen < 0; ++a) {
            const uint32_t j = lemire_draw(k0, k1, uint32_t(r), uint32_t(w), ctr, 256u + 1024u * uint32_t(t) + a,
                                           uint32_t(dz));
            const int64_t p = z0 + j;
            const double ratio = lazy_x(kind, col, val, scale, p) / xmax[z];
            if (ratio >= kLazyEqual ||
                uniform53(k0, k1, uint32_t(r), uint32_t(w), ctr, (1u << 20) + 1024u * uint32_t(t) + a) < ratio)
              chosen = p;
          }
          if (chosen < 0) {  // exact inverse-CDF draw over the row (total summed in row order first)
            double total = 0.0;
            for (int64_t p = z0; p < z0 + dz; ++p) total += lazy_x(kind, col, val, scale, p);
            const double target = uniform53(k0, k1, uint32_t(r), uint32_t(w), ctr, (1u << 21) + uint32_t(t)) * total;
            double run = 0.0;
            chosen = z0 + dz - 1;
            for (int64_t p = z0; p < z0 + dz; ++p) {
              run += lazy_x(kind, col, val, scale, p);
              if (run > target) {
                chosen = p;
                break;
              }
            }
          }
          z = col[chosen];
          z0 = rowptr[z];
          dz = rowptr[z + 1] - z0;
        }
      }
      double wt = 0.0;
      if (live) wt = (norm && rs > 0.0) ? double(scale[z]) / rs : 1.0;
      for (int j0 = 0; j0 < nlive; j0 += 8) {
        rb.issue(X, ldx, cc, G, j0, float(wt), z);
        rb.consume(col_ok, j0, nlive, acc);
      }
    }
  }
  if (row_ok && col_ok) {
    float o[VEC];
    const float inv = float(1.0 / double(walks));
#pragma unroll
    for (int v = 0; v < VEC; ++v) o[v] = acc[v] * inv;
    VecIO<TY, VEC>::store(Y + r * ldy + c0, o);
  }
}

template <typename TX>
__global__ __launch_bounds__(kBlock) void scale_init_kernel(int64_t n, int k, const TX *__restrict__ X,
                                                             int64_t ldx, float *__restrict__ Y, int64_t ldy,
                                                             double c0d) {
  const float c0 = float(c0d);
  const int64_t total = n * k;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < total; i += int64_t(gridDim.x) * kBlock) {
    int64_t r = i / k, c = i - r * k;
    Y[r * ldy + c] = c0 * to_f32<TX>(X[r * ldx + c]);
  }
}

__device__ inline int32_t row_of(const int64_t *rowptr, int64_t n, int64_t p) {
  // largest r with rowptr[r] <= p
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (rowptr[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  return int32_t(lo);
}

template <typename TX, int VEC>
__global__ __launch_bounds__(kBlock) void walk_reject_kernel(
    int64_t n, int64_t nnz, int k, int G, int lgG, Graph g, int ell, const TX *__restrict__ X, int64_t ldx,
    float *__restrict__ Y, int64_t ldy, int64_t trials, uint32_t k0, uint32_t k1, uint32_t ctr,
    double scale, double d_inc, unsigned long long *__restrict__ counts, Coefs cf) {
  __shared__ unsigned int bcount[kMaxDeg];
  for (int i = threadIdx.x; i < ell; i += kBlock) bcount[i] = 0;
  __syncthreads();
  const int lig = threadIdx.x & (G - 1);
  const int grp = threadIdx.x >> lgG;
  const int gpb = kBlock >> lgG;
  const int c0 = blockIdx.y * 64 * VEC + lig * VEC;
  const bool col_ok = c0 < k;
  for (int64_t T = int64_t(blockIdx.x) * gpb + grp; T < trials; T += int64_t(gridDim.x) * gpb) {
    const uint32_t tc0 = uint32_t(uint64_t(T) & 0xffffffffu);
    const uint32_t tc1 = uint32_t(uint64_t(T) >> 32) | 0x80000000u;
    uint32_t p0 = lemire_draw(k0, k1, tc0, tc1, ctr, 0u, uint32_t(nnz));
    const int32_t ra_ = row_of(g.rowptr, n, int64_t(p0));
    int64_t rev_p = 0;
    Edge e = first_edge(g, ra_, g.wn[ra_], int64_t(p0), &rev_p);
    const int32_t a1 = e.a, b1 = e.b;
    const float h1a = e.ha, h1b = e.hb;
    double rho = 1.0, accept_p = 1.0;
    float acc_a[VEC], acc_b[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc_a[v] = acc_b[v] = 0.f;
    bool any = false;
    for (int i = 1; i <= ell; ++i) {
      bool ok = true;
      if (i > 1) {
        uint32_t bound = uint32_t((e.a1 - e.a0) + (e.b1 - e.b0) - 1);
        uint32_t t = lemire_draw(k0, k1, tc0, tc1, ctr, uint32_t(i - 1), bound);
        float dot = move(g, e, t, &rev_p);
        rho = rho * (double(dot) * d_inc);
        accept_p = (accept_p * double(bound)) / d_inc;
        double u = uniform53(k0, k1, tc0, tc1, ctr, uint32_t(ell + i));
        ok = u < accept_p;
      }
      if (ok) {
        if (lig == 0) atomicAdd(&bcount[i - 1], 1u);
        any = true;
        if (col_ok) {
          float xa[VEC], xb[VEC];
          VecIO<TX, VEC>::load(X + int64_t(e.a) * ldx + c0, xa);
          VecIO<TX, VEC>::load(X + int64_t(e.b) * ldx + c0, xb);
          const double base = cf.c[i] * scale * rho;
          const float wa = float(base * double(e.ha)), wb = float(base * double(e.hb));
          const float fa = h1a, fb = h1b;
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            float val = fmaf(wa, xa[v], wb * xb[v]);
            acc_a[v] = fmaf(fa, val, acc_a[v]);
            acc_b[v] = fmaf(fb, val, acc_b[v]);
          }
        }
      }
    }
    if (any && col_ok) {
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        atomicAdd(Y + int64_t(a1) * ldy + c0 + v, acc_a[v]);
        atomicAdd(Y + int64_t(b1) * ldy + c0 + v, acc_b[v]);
      }
    }
  }
  __syncthreads();
  if (counts && blockIdx.y == 0)
    for (int i = threadIdx.x; i < ell; i += kBlock)
      if (bcount[i]) atomicAdd(counts + i, (unsigned long long)bcount[i]);
}

__global__ void zero_u64_kernel(unsigned long long *p, int count) {
  int i = threadIdx.x;
  if (i < count) p[i] = 0ull;
}

template <typename TX, typename TY>
sped_status launch_is(const sped_csr *L, int64_t k, const void *X, int64_t ldx, void *Y, int64_t ldy,
                      int ell, int64_t walks, uint32_t k0, uint32_t k1, uint32_t ctr, const Coefs &cf,
                      hipStream_t s) {
  int vec = pick_vec(k, {ldx, ldy}, {X, Y}, {int(sizeof(TX)), int(sizeof(TY))});
  int lanes = int((k + vec - 1) / vec);
  int ytiles = (lanes + 63) / 64;
  int G = lanes >= 64 ? 64 : next_pow2(lanes);
  int lgG = ilog2(G);
  Graph g{L->rowptr, L->wentry, L->wnode};
  const int64_t rows_per_block = kBlock >> lgG;
  const int64_t nb = (L->n + rows_per_block - 1) / rows_per_block;
  const dim3 grid = dim3(unsigned(xcd_padded_grid(nb)), unsigned(ytiles));
#define SPED_IS(V)                                                                                     \
  hipLaunchKernelGGL((walk_importance_kernel<TX, TY, V>), grid, dim3(kBlock), kWalkLdsReserve, s, L->n, nb, \
                     int(k), G, lgG, g, ell, static_cast<const TX *>(X), ldx, static_cast<TY *>(Y), ldy, walks, \
                     k0, k1, ctr, cf)
  if (vec == 4) SPED_IS(4);
  else if (vec == 2) SPED_IS(2);
  else SPED_IS(1);
#undef SPED_IS
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

template <typename TX>
sped_status launch_rej(const sped_csr *L, int64_t k, const void *X, int64_t ldx, float *Y, int64_t ldy, int ell,
                       int64_t trials, uint32_t k0, uint32_t k1, uint32_t ctr, int64_t *counts, const Coefs &cf,
                       hipStream_t s) {
  int vec = pick_vec(k, {ldx, ldy}, {X, Y}, {int(sizeof(TX)), 4});
  int lanes = int((k + vec - 1) / vec);
  int ytiles = (lanes + 63) / 64;
  int G = lanes >= 64 ? 64 : next_pow2(lanes);
  int lgG = ilog2(G);
  Graph g{L->rowptr, L->wentry, L->wnode};
  const int64_t total = L->n * k;
  int64_t iblocks = (total + kBlock - 1) / kBlock;
  if (iblocks > 4096) iblocks = 4096;
  hipLaunchKernelGGL((scale_init_kernel<TX>), dim3(unsigned(iblocks > 0 ? iblocks : 1)), dim3(kBlock), 0, s,
                     L->n, int(k), static_cast<const TX *>(X), ldx, Y, ldy, cf.c[0]);
  SPED_CHECK_HIP(hipGetLastError());
  unsigned long long *cnt = reinterpret_cast<unsigned long long *>(counts);
  if (cnt) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(kBlock), 0, s, cnt, ell);
    SPED_CHECK_HIP(hipGetLastError());
  }
  if (L->nnz == 0) return SPED_OK;  // no edges: the estimate is c_0 X exactly
  const double n_edges = double(L->nnz / 2);
  const double scale = n_edges / double(trials);
  const double d_inc = double(2 * int64_t(L->max_degree) - 1);
  int64_t gpb = kBlock >> lgG;
  int64_t blocks = (trials + gpb - 1) / gpb;
  if (blocks > 65536) blocks = 65536;
  const dim3 grid = dim3(unsigned(blocks), unsigned(ytiles));
#define SPED_REJ(V)                                                                                  \
  hipLaunchKernelGGL((walk_reject_kernel<TX, V>), grid, dim3(kBlock), 0, s, L->n, L->nnz, int(k), G, lgG, g, \
                     ell, static_cast<const TX *>(X), ldx, Y, ldy, trials, k0, k1, ctr, scale, d_inc, cnt, cf)
  if (vec == 4) SPED_REJ(4);
  else if (vec == 2) SPED_REJ(2);
  else SPED_REJ(1);
#undef SPED_REJ
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

}  // namespace

sped_status walk_estimate_impl(const sped_csr *L, const double *coeffs, int degree, int64_t k, const void *X,
                               int64_t ldx, int xdt, void *Y, int64_t ldy, int ydt, int sampler, int64_t walks,
                               uint64_t seed, uint64_t counter, int64_t *accept_counts, hipStream_t s) {
  Coefs cf{};
  for (int i = 0; i <= degree; ++i) cf.c[i] = coeffs[i];
  const uint32_t k0 = uint32_t(seed & 0xffffffffu), k1 = uint32_t(seed >> 32);
  const uint32_t ctr = uint32_t(counter);
  if (sampler == 0) {
    if (xdt == SPED_F32 && ydt == SPED_F32) return launch_is<float, float>(L, k, X, ldx, Y, ldy, degree, walks, k0, k1, ctr, cf, s);
    if (xdt == SPED_F32 && ydt == SPED_BF16) return launch_is<float, bf16_t>(L, k, X, ldx, Y, ldy, degree, walks, k0, k1, ctr, cf, s);
    if (xdt == SPED_BF16 && ydt == SPED_F32) return launch_is<bf16_t, float>(L, k, X, ldx, Y, ldy, degree, walks, k0, k1, ctr, cf, s);
    return launch_is<bf16_t, bf16_t>(L, k, X, ldx, Y, ldy, degree, walks, k0, k1, ctr, cf, s);
  }
  if (xdt == SPED_F32)
    return launch_rej<float>(L, k, X, ldx, static_cast<float *>(Y), ldy, degree, walks, k0, k1, ctr, accept_counts, cf, s);
  return launch_rej<bf16_t>(L, k, X, ldx, static_cast<float *>(Y), ldy, degree, walks, k0, k1, ctr, accept_counts, cf, s);
}

template <typename TX, typename TY>
sped_status launch_lazy(const sped_csr *L, int64_t k, const void *X, int64_t ldx, void *Y, int64_t ldy, int ell,
                        int64_t walks, uint32_t k0, uint32_t k1, uint32_t ctr, const double *xmax,
                        hipStream_t s) {
  int vec = pick_vec(k, {ldx, ldy}, {X, Y}, {int(sizeof(TX)), int(sizeof(TY))});
  int lanes = int((k + vec - 1) / vec);
  int ytiles = (lanes + 63) / 64;
  int G = lanes >= 64 ? 64 : next_pow2(lanes);
  int lgG = ilog2(G);
  const int64_t rows_per_block = kBlock >> lgG;
  const int64_t nb = (L->n + rows_per_block - 1) / rows_per_block;
  const dim3 grid = dim3(unsigned(xcd_padded_grid(nb)), unsigned(ytiles));
#define SPED_LZ(V)                                                                                          \
  hipLaunchKernelGGL((walk_lazy_kernel<TX, TY, V>), grid, dim3(kBlock), 0, s, L->n, nb, int(k), G, lgG,     \
                     int(L->kind), L->rowptr, L->col, L->val, L->scale, L->diag, xmax, ell,                 \
                     static_cast<const TX *>(X), ldx, static_cast<TY *>(Y), ldy, walks, k0, k1, ctr)
  if (vec == 4) SPED_LZ(4);
  else if (vec == 2) SPED_LZ(2);
  else SPED_LZ(1);
#undef SPED_LZ
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

}  // namespace sped

using namespace sped;

namespace sped {
namespace {

// Argument checks shared by the walk estimators (degree checked by the caller);
// `walking` false checks only what an exact evaluation needs.
sped_status validate_walk_args(const sped_csr *L, const double *coeffs, int degree, int64_t k, const void *X,
                               int64_t ldx, int xdt, const void *Y, int64_t ldy, int ydt, int sampler,
                               int64_t walks, uint64_t counter, bool walking = true) {
  if (!coeffs) return fail(SPED_E_INVALID, "coeffs NULL");
  for (int i = 0; i <= degree; ++i)
    if (!std::isfinite(coeffs[i])) return fail(SPED_E_INVALID, "coefficient not finite");
  if (k < 1) return fail(SPED_E_INVALID, "k < 1");
  if (ldx < k || ldy < k) return fail(SPED_E_INVALID, "leading dimension < k");
  if ((xdt != SPED_F32 && xdt != SPED_BF16) || (ydt != SPED_F32 && ydt != SPED_BF16))
    return fail(SPED_E_UNSUPPORTED, "dtype");
  if (L->n > 0 && (!X || !Y)) return fail(SPED_E_INVALID, "X or Y NULL");
  if (!walking) return SPED_OK;
  if (L->nnz > 0 && (!L->wentry || !L->wnode)) return fail(SPED_E_INVALID, "csr walk records NULL");
  if (sampler != 0 && sampler != 1) return fail(SPED_E_INVALID, "sampler must be 0 or 1");
  if (walks < 1) return fail(SPED_E_INVALID, "walks < 1");
  if (counter >= (uint64_t(1) << 32)) return fail(SPED_E_INVALID, "counter >= 2^32");
  if (sampler == 0 && walks >= (int64_t(1) << 32)) return fail(SPED_E_INVALID, "walks per row >= 2^32");
  if (sampler == 1 && L->nnz >= (int64_t(1) << 32))
    return fail(SPED_E_UNSUPPORTED, "rejection sampler needs nnz < 2^32");
  return SPED_OK;
}

}  // namespace
}  // namespace sped

extern "C" sped_status sped_apply_poly_stochastic(const sped_csr *L, const double *coeffs, int32_t degree,
                                                  int64_t k, const void *X, int64_t ldx, int32_t xdt, void *Y,
                                                  int64_t ldy, int32_t ydt, int32_t sampler, int64_t walks,
                                                  uint64_t seed, uint64_t counter, int64_t *accept_counts,
                                                  void *ws, size_t *ws_bytes, sped_stream_t stream) {
  clear_error();
  SPED_TRY(validate_csr(L));
  if (degree < 1 || degree > kMaxDeg) return fail(SPED_E_INVALID, "degree outside [1, 255]");
  SPED_TRY(validate_walk_args(L, coeffs, degree, k, X, ldx, xdt, Y, ldy, ydt, sampler, walks, counter));
  if (sampler == 1 && ydt != SPED_F32) return fail(SPED_E_UNSUPPORTED, "rejection sampler needs a float32 Y");
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, 0, &query));
  if (query || L->n == 0) return SPED_OK;
  return walk_estimate_impl(L, coeffs, degree, k, X, ldx, xdt, Y, ldy, ydt, sampler, walks, seed, counter,
                            accept_counts, as_stream(stream));
}

namespace sped {

sped_status hybrid_estimate_impl(const sped_csr *L, const double *coeffs, int degree, int m, int64_t k,
                                 const void *X, int64_t ldx, int xdt, void *Y, int64_t ldy, int ydt, int sampler,
                                 int64_t walks, uint64_t seed, uint64_t counter, float *T0, float *T1,
                                 void *step_ws, hipStream_t s, int64_t *spmm_count) {
  if (L->n == 0) return SPED_OK;
  if (m == 0)
    return walk_estimate_impl(L, coeffs, degree, k, X, ldx, xdt, Y, ldy, ydt, sampler, walks, seed, counter,
                              nullptr, s);
  float *T[2] = {T0, T1};
  const bool sampled = m < degree;
  // U starts as the sampled tail T (or, with no tail, as X scaled by c_degree in the first step)
  const void *U = X;
  int64_t ldu = ldx;
  int tu = xdt;
  float first_a = float(coeffs[degree]);
  if (sampled) {
    SPED_TRY(walk_estimate_impl(L, coeffs + m, degree - m, k, X, ldx, xdt, T[0], k, SPED_F32, sampler, walks, seed,
                                counter, nullptr, s));
    U = T[0];
    ldu = k;
    tu = SPED_F32;
    first_a = 1.f;
  }
  int next = sampled ? 1 : 0;
  for (int i = m - 1; i >= 0; --i) {
    StepArgs a{};
    a.heavy_ws = step_ws;
    a.U = U; a.ldu = ldu; a.tu = tu;
    a.V = X; a.ldv = ldx; a.tv = xdt;
    if (i == 0) {
      a.O = Y; a.ldo = ldy; a.to = ydt;
    } else {
      a.O = T[next]; a.ldo = k; a.to = SPED_F32;
    }
    a.a = i == m - 1 ? first_a : 1.f;
    a.b = 0.f;
    a.g = float(coeffs[i]);
    SPED_TRY(launch_spmm_step(L, k, a, s));
    if (spmm_count) ++*spmm_count;
    U = a.O;
    ldu = a.ldo;
    tu = a.to;
    next ^= 1;
  }
  return SPED_OK;
}

}  // namespace sped

// Exact low-order terms, sampled tail:
//   Y = sum_{i<m} c_i L^i X + L^m T,   T = walk estimate of sum_{j>=0} c_{m+j} L^j X,
// evaluated as m Horner steps U <- L U + c_i X (i = m-1 .. 0) starting from T.
extern "C" sped_status sped_apply_poly_hybrid(const sped_csr *L, const double *coeffs, int32_t degree,
                                              int32_t exact_terms, int64_t k, const void *X, int64_t ldx,
                                              int32_t xdt, void *Y, int64_t ldy, int32_t ydt, int32_t sampler,
                                              int64_t walks, uint64_t seed, uint64_t counter, void *ws,
                                              size_t *ws_bytes, sped_stream_t stream) {
  clear_error();
  SPED_TRY(validate_csr(L));
  if (degree < 1 || degree > kMaxDeg) return fail(SPED_E_INVALID, "degree outside [1, 255]");
  if (exact_terms < 0 || exact_terms > degree) return fail(SPED_E_INVALID, "exact_terms outside [0, degree]");
  const int m = exact_terms;
  const bool sampled = m < degree;
  if (sampled) {
    SPED_TRY(validate_walk_args(L, coeffs, degree, k, X, ldx, xdt, Y, ldy, ydt, sampler, walks, counter));
    if (sampler == 1 && m == 0 && ydt != SPED_F32)
      return fail(SPED_E_UNSUPPORTED, "rejection sampler needs a float32 Y");
  } else {
    SPED_TRY(validate_walk_args(L, coeffs, degree, k, X, ldx, xdt, Y, ldy, ydt, sampler, walks, counter, false));
  }
  const int64_t n = L->n;
  Carver c(ws);
  float *T[2] = {nullptr, nullptr};
  if (m >= 1) T[0] = c.take<float>(size_t(n > 0 ? n : 1) * size_t(k));
  if (m >= 2) T[1] = c.take<float>(size_t(n > 0 ? n : 1) * size_t(k));
  const size_t sw = m >= 1 ? spmm_step_ws_bytes(L, k) : 0;
  void *step_ws = sw ? c.take<char>(sw) : nullptr;
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, c.bytes(), &query));
  if (query || n == 0) return SPED_OK;
  const char *xb = static_cast<const char *>(X), *yb = static_cast<const char *>(Y);
  size_t xs = size_t((n - 1) * ldx + k) * dtype_size(xdt), ys = size_t((n - 1) * ldy + k) * dtype_size(ydt);
  if (xb < yb + ys && yb < xb + xs) return fail(SPED_E_INVALID, "X and Y overlap");
  return hybrid_estimate_impl(L, coeffs, degree, m, k, X, ldx, xdt, Y, ldy, ydt, sampler, walks, seed, counter,
                              T[0], T[1], step_ws, as_stream(stream));
}

namespace sped {

sped_status lazy_row_max(const sped_csr *L, double *xmax, hipStream_t s) {
  if (L->n == 0) return SPED_OK;
  int64_t blocks = (L->n + kBlock / 64 - 1) / (kBlock / 64);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(lazy_row_max_kernel, dim3(unsigned(blocks)), dim3(kBlock), 0, s, L->n, int(L->kind),
                     L->rowptr, L->col, L->val, L->scale, xmax);
  SPED_CHECK_HIP(hipGetLastError());
  return SPED_OK;
}

sped_status lazy_walk_impl(const sped_csr *L, int ell, int64_t k, const void *X, int64_t ldx, int xdt, void *Y,
                           int64_t ldy, int ydt, int64_t walks, uint64_t seed, uint64_t counter, const double *xmax,
                           hipStream_t s) {
  if (L->n == 0) return SPED_OK;
  const uint32_t k0 = uint32_t(seed & 0xffffffffu), k1 = uint32_t(seed >> 32), ctr = uint32_t(counter);
  if (xdt == SPED_F32 && ydt == SPED_F32)
    return launch_lazy<float, float>(L, k, X, ldx, Y, ldy, ell, walks, k0, k1, ctr, xmax, s);
  if (xdt == SPED_F32 && ydt == SPED_BF16)
    return launch_lazy<float, bf16_t>(L, k, X, ldx, Y, ldy, ell, walks, k0, k1, ctr, xmax, s);
  if (xdt == SPED_BF16 && ydt == SPED_F32)
    return launch_lazy<bf16_t, float>(L, k, X, ldx, Y, ldy, ell, walks, k0, k1, ctr, xmax, s);
  return launch_lazy<bf16_t, bf16_t>(L, k, X, ldx, Y, ldy, ell, walks, k0, k1, ctr, xmax, s);
}

sped_status validate_lazy(const sped_csr *L, int ell, int64_t walks, uint64_t counter) {
  if (ell < 1 || ell > kMaxDeg) return fail(SPED_E_INVALID, "ell outside [1, 255]");
  if (walks < 1 || walks >= (int64_t(1) << 32)) return fail(SPED_E_INVALID, "walks per row outside [1, 2^32)");
  if (counter >= (uint64_t(1) << 32)) return fail(SPED_E_INVALID, "counter >= 2^32");
  if (L->n >= (int64_t(1) << 31)) return fail(SPED_E_UNSUPPORTED, "n >= 2^31");
  // combinatorial: the stay probability 1 - d/l must be non-negative
  if (L->kind == SPED_LAP_COMBINATORIAL && 0.5 * L->lambda_bound > double(ell))
    return fail(SPED_E_INVALID, "combinatorial lazy walk needs ell >= the largest weighted degree");
  return SPED_OK;
}

}  // namespace sped

extern "C" sped_status sped_apply_limit_lazy(const sped_csr *L, int32_t ell, int64_t k, const void *X, int64_t ldx,
                                             int32_t xdt, void *Y, int64_t ldy, int32_t ydt, int64_t walks,
                                             uint64_t seed, uint64_t counter, void *ws, size_t *ws_bytes,
                                             sped_stream_t stream) {
  clear_error();
  SPED_TRY(validate_csr(L));
  if (k < 1) return fail(SPED_E_INVALID, "k < 1");
  if (ldx < k || ldy < k) return fail(SPED_E_INVALID, "leading dimension < k");
  if ((xdt != SPED_F32 && xdt != SPED_BF16) || (ydt != SPED_F32 && ydt != SPED_BF16))
    return fail(SPED_E_UNSUPPORTED, "dtype");
  if (L->n > 0 && (!X || !Y)) return fail(SPED_E_INVALID, "X or Y NULL");
  SPED_TRY(validate_lazy(L, ell, walks, counter));
  Carver c(ws);
  double *xmax = c.take<double>(size_t(L->n > 0 ? L->n : 1));
  bool query;
  SPED_TRY(check_ws(ws, ws_bytes, c.bytes(), &query));
  if (query || L->n == 0) return SPED_OK;
  const char *xb = static_cast<const char *>(X), *yb = static_cast<const char *>(Y);
  size_t xs = size_t((L->n - 1) * ldx + k) * dtype_size(xdt), ys = size_t((L->n - 1) * ldy + k) * dtype_size(ydt);
  if (xb < yb + ys && yb < xb + xs) return fail(SPED_E_INVALID, "X and Y overlap");
  hipStream_t s = as_stream(stream);
  SPED_TRY(lazy_row_max(L, xmax, s));
  return lazy_walk_impl(L, ell, k, X, ldx, xdt, Y, ldy, ydt, walks, seed, counter, xmax, s);
}
