/*
 * sped.h -- C ABI of libsped: eigengap dilation (SPED) of graph Laplacians on
 * one AMD Instinct MI355X (gfx950).
 *
 * The paper is van der Pol, Gemp, Bachrach, Everett, "Stochastic Parallelizable
 * Eigengap Dilation for Large Graph Clustering" (arXiv 2207.14589).  Every entry
 * point below names the passage that defines the operation it computes.
 *
 * Conventions for every call
 *  - Pointers documented as DEVICE point to memory on the current HIP device,
 *    allocated and owned by the caller; HOST pointers point to host memory.
 *    The library never allocates device memory: calls that need scratch take a
 *    caller workspace (ws, ws_bytes).  Calling with ws == NULL and ws_bytes
 *    != NULL stores the required size in *ws_bytes and returns SPED_OK
 *    without launching work; calling with ws != NULL and *ws_bytes below that
 *    size returns SPED_E_WORKSPACE.  A call whose required size is 0 runs
 *    with ws == NULL and ws_bytes == NULL.  Workspace must be 256-byte aligned.
 *  - Dense blocks are row-major: element (r, c) of an n x k block with leading
 *    dimension ld sits at base[r * ld + c]; ld >= k.  A node's k values are
 *    contiguous.  Element types are given by sped_dtype.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *    Calls return without synchronising unless documented otherwise.
 *  - Arguments are validated on the host before any launch.  On a non-OK
 *    status nothing has been launched unless documented otherwise, outputs are
 *    unspecified, and sped_last_error() returns a message for this thread.
 *  - No C++ exception crosses this interface.
 */
#ifndef SPED_H
#define SPED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *sped_stream_t; /* hipStream_t */

typedef enum {
  SPED_OK = 0,
  SPED_E_INVALID = 1,       /* bad argument, shape, pointer or value */
  SPED_E_WORKSPACE = 2,     /* workspace smaller than required */
  SPED_E_DEVICE = 3,        /* a HIP runtime call failed */
  SPED_E_NUMERIC = 4,       /* NaN/Inf, or Cholesky breakdown after the shift fallback */
  SPED_E_NOT_CONVERGED = 5, /* iteration cap reached before the tolerance */
  SPED_E_UNSUPPORTED = 6    /* valid but not implemented combination */
} sped_status;

typedef enum { SPED_F32 = 0, SPED_BF16 = 1, SPED_F64 = 2 } sped_dtype;

typedef enum {
  SPED_LAP_COMBINATORIAL = 0,  /* L = D - A = X^T W X (Sec. 2) */
  SPED_LAP_SYM_NORMALIZED = 1  /* D^{-1/2} L D^{-1/2} (normalised Laplacian, Sec. 4.1) */
} sped_lap_kind;

/*
 * The Laplacian in split CSR form: L = diag(diag) - S, S the off-diagonal
 * part with S_ij >= 0.  Built by sped_laplacian_csr; all arrays DEVICE.
 *  rowptr [n+1] int64   row r's entries are [rowptr[r], rowptr[r+1])
 *  col    [nnz] int32   neighbour ids, strictly ascending within a row
 *  val    [nnz] float   S_ij = w_ij (combinatorial) or w_ij s_i s_j (normalised)
 *  rev    [nnz] int64   position of the transposed entry (j, i) of entry (i, j)
 *  diag   [n]   float   L_ii = d_i (combinatorial) or 1 (normalised; 0 if d_i = 0)
 *  scale  [n]   float   s_i = 1 (combinatorial) or d_i^{-1/2} (normalised; 0 if d_i = 0)
 *  bins   [n]   int32   rows with more than SPED_LIGHT_MAX entries, medium rows
 *                       (<= SPED_MEDIUM_MAX entries) first, then heavy rows
 *  wentry [nnz], wnode [n]  packed walk records (see above), optional
 * d_i is the weighted degree; nnz = 2 x the number of distinct undirected edges.
 */
#define SPED_LIGHT_MAX 128
#define SPED_MEDIUM_MAX 8192
/* Packed records read by the walk estimators.  An entry record carries what a
 * walk needs about the entry's far endpoint v = col[p], so a move is one
 * 32-byte load (one cache line):
 *  sped_walk_entry[p] = (v, val[p], rev[p] - rowptr[v], rowptr[v+1] - rowptr[v],
 *                        rowptr[v], sqrt(scale[v]), 0)
 *  sped_walk_node[u]  = (rowptr[u], rowptr[u+1] - rowptr[u], sqrt(scale[u])) */
typedef struct {
  int32_t col;
  float val;
  int32_t rev_local;
  int32_t degree;     /* of col */
  int64_t start;      /* rowptr[col] */
  float root_scale;   /* sqrt(scale[col]) */
  int32_t pad;
} sped_walk_entry;
typedef struct {
  int64_t start;
  int32_t degree;
  float root_scale;
} sped_walk_node;
typedef struct {
  int64_t n;
  int64_t nnz;
  int64_t *rowptr;
  int32_t *col;
  float *val;
  int64_t *rev;
  float *diag;
  float *scale;
  int32_t *bins;
  sped_walk_entry *wentry; /* [nnz], or NULL (then the walk estimators are unavailable) */
  sped_walk_node *wnode;   /* [n], or NULL */
  int64_t n_medium;
  int64_t n_heavy;
  int32_t max_degree;   /* largest number of neighbours of any node (deg* of Sec. 4.3) */
  int32_t kind;         /* sped_lap_kind */
  double lambda_bound;  /* 2 (normalised) or 2 max_i d_i (combinatorial): >= lambda_max */
  /* Row split of the light-row SpMM over the 8 XCDs (accelerator complex
   * dies, each with its own L2): XCD x handles rows [xcd_rows[x],
   * xcd_rows[x+1]), ranges of equal light-row work (entries plus a per-row
   * cost), so a degree-sorted graph does not load one die with most of the
   * entries.  Filled by sped_laplacian_csr; a caller-built struct sets all nine
   * to zero (any array that is not 0 = x_0 <= ... <= x_8 = n is ignored and
   * the rows are split evenly). */
  int64_t xcd_rows[9];
} sped_csr;

/*
 * sped_laplacian_csr -- build the Laplacian of an undirected, optionally
 * weighted graph (Sec. 2: L = X^T X with incidence rows +1 at min(i,j), -1 at
 * max(i,j); weighted form X^T W X; Sec. 4.1 normalised form).
 *  n, m        node count (< 2^31) and input edge count
 *  src, dst    DEVICE int32 [m] endpoints in [0, n); self-loops are ignored
 *              (their incidence row is zero); repeated pairs add their weights
 *  w           DEVICE float [m] weights, finite and > 0, or NULL for all ones
 *  kind        sped_lap_kind
 *  lcc_only    nonzero: keep only the largest connected component (ties: the
 *              one holding the smallest node id), relabelled in increasing id
 *  out         HOST struct; on entry its array pointers must point to DEVICE
 *              buffers of at least rowptr n+1, col/val/rev/wentry 2m,
 *              diag/scale/bins/wnode n elements (wentry, wnode may be NULL).  On return n, nnz, n_medium, n_heavy, max_degree,
 *              kind, lambda_bound and xcd_rows are filled in.
 *  old_of_new  DEVICE int32 [n] or NULL: original id of each kept node
 * Synchronises `stream` before returning (sizes are read back).  Invalid
 * endpoints or weights found on the device return SPED_E_INVALID.
 */
sped_status sped_laplacian_csr(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                               const float *w, int32_t kind, int32_t lcc_only, sped_csr *out,
                               int32_t *old_of_new, void *ws, size_t *ws_bytes,
                               sped_stream_t stream);

/*
 * Node orders for gather locality.  p(L)V (Sec. 4.2) is the same operator
 * under any relabelling of the nodes, with the rows of V permuted alike; the
 * paper fixes no order.  An order that places neighbours at nearby ids lets
 * the sparse products' neighbour-row gathers share cache lines.
 *  SPED_ORDER_CUTHILL_MCKEE  breadth-first search from the node of largest
 *      degree (ties: smallest id), appending the unvisited neighbours of
 *      each dequeued node by increasing (degree, id) (Cuthill and McKee,
 *      1969); nodes outside that node's component follow in increasing id.
 *  SPED_ORDER_DEGREE  decreasing degree, ties in increasing id.
 *  SPED_ORDER_LABEL_PROPAGATION  nodes grouped by the communities found by
 *      synchronous label propagation (Raghavan, Albert and Kumara, 2007):
 *      labels start as the ids; each round, every node with neighbours takes
 *      the label most frequent among its neighbours' labels of the previous
 *      round (unweighted counts), ties going to the label with the smallest
 *      splitmix64 output of (label XOR (round + 1) << 32), rounds from 0; at
 *      most 16 rounds, stopping after one that changes no label.  Groups in
 *      increasing label; inside a group decreasing degree, then increasing
 *      id.
 * Degree = number of distinct neighbours (row length of L's off-diagonal part).
 */
typedef enum {
  SPED_ORDER_CUTHILL_MCKEE = 0,
  SPED_ORDER_DEGREE = 1,
  SPED_ORDER_LABEL_PROPAGATION = 2
} sped_order;

/*
 * sped_locality_order -- the position of each node of L in the order `method`.
 *  L           built by sped_laplacian_csr (its rowptr and col are read; the
 *              off-diagonal pattern must be symmetric, with columns in [0, n))
 *  new_of_old  DEVICE int32 [L->n], written: a permutation of 0 .. n-1
 * Synchronises `stream` (once per search level or propagation round, and
 * before returning).  The result is deterministic (independent of the order
 * in which the device's atomics land).  Label propagation's workspace holds
 * two 8-byte keys per stored entry.  An unknown method or a NULL array
 * returns SPED_E_INVALID before any launch; a search that reaches more nodes
 * than L has (an adjacency that is not a valid CSR) returns SPED_E_INVALID.
 */
sped_status sped_locality_order(const sped_csr *L, int32_t method, int32_t *new_of_old, void *ws,
                                size_t *ws_bytes, sped_stream_t stream);

/*
 * sped_laplacian_csr_ordered -- sped_laplacian_csr, with the kept nodes
 * numbered in the order `method` computed on the built Laplacian: the graph
 * is built, ordered, relabelled and built again (the second build takes the
 * kept nodes only; edges of dropped components become ignored self-loops).
 * Arguments, output buffers and errors as for sped_laplacian_csr, plus
 * SPED_E_INVALID for an unknown method; old_of_new (DEVICE int32 [n] or
 * NULL) receives the original id of each row of the result, so a block V
 * given in original ids enters as V[old_of_new] and results return by the
 * inverse scatter.  The workspace holds the larger of the build's and the
 * order's needs plus 2m + 3n int32.  Synchronises `stream` before returning.
 */
sped_status sped_laplacian_csr_ordered(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                                       const float *w, int32_t kind, int32_t lcc_only, int32_t method,
                                       sped_csr *out, int32_t *old_of_new, void *ws, size_t *ws_bytes,
                                       sped_stream_t stream);

/*
 * A polynomial of the Laplacian (Sec. 4.1-4.2, Table 2, reversed by eq. reveig).
 *  SPED_POLY_MONOMIAL: M = sum_{i=0..degree} coeffs[i] Lt^i,
 *                      Lt = (L - shift I) / scale, evaluated by Horner's rule.
 *  SPED_POLY_LIMIT:    M = (I - L/degree)^degree, the limit approximation of
 *                      -exp(-L) reversed with lambda* = 0, evaluated as degree
 *                      factor applications; coeffs/shift/scale are ignored.
 * coeffs is HOST [degree+1].  1 <= degree <= 1024.
 */
typedef enum { SPED_POLY_MONOMIAL = 0, SPED_POLY_LIMIT = 1 } sped_poly_kind;
typedef struct {
  int32_t kind;
  int32_t degree;
  const double *coeffs;
  double shift;
  double scale;
} sped_poly;

/*
 * Table 2 transforms reversed by eq. reveig, as monomial coefficients of M.
 *  SPED_T_PLAIN       identity transform: M = lambda_bound I - L (degree 1)
 *  SPED_T_LIMIT       limit approximation of -exp(-L), lambda* = 0:
 *                     M = (I - L/l)^l, c_i = C(l, i) (-1/l)^i
 *  SPED_T_TAYLOR_EXP  Taylor series of -exp(-L), lambda* = 0: c_i = (-1)^i / i!
 *  SPED_T_TAYLOR_LOG  Taylor series of log(L + eps I) in y = L - (1 - eps) I,
 *                     lambda* = f(lambda_bound): c_0 = f(lambda_bound),
 *                     c_i = (-1)^i / i; shift = 1 - eps, scale = 1
 * (Sec. 4.1 requires f increasing where the wanted eigenvalues lie; Table 2
 * takes l odd.  The Taylor log with an even degree is not increasing on
 * [0, 2] and returns SPED_E_UNSUPPORTED.)  coeffs HOST [degree+1]; shift,
 * scale HOST.
 */
typedef enum { SPED_T_PLAIN = 0, SPED_T_LIMIT = 1, SPED_T_TAYLOR_EXP = 2, SPED_T_TAYLOR_LOG = 3 } sped_transform;
sped_status sped_transform_coeffs(int32_t transform, int32_t degree, double lambda_bound, double eps,
                                  double *coeffs, double *shift, double *scale);

/* sped_poly_monomial -- the coefficients of p in powers of L itself
 * (binomial expansion of the shift and scale, or of the limit product);
 * out HOST [degree+1]. */
sped_status sped_poly_monomial(const sped_poly *p, double *out);

/* sped_poly_rebase -- the coefficients of p in the variable
 * Lt = (L - shift I) / scale (scale != 0), so that p = sum_i out[i] Lt^i:
 * the learnable coefficients of Sec. 6 start from a Table 2 row written in
 * the variable where the tuning runs.  The limit polynomial is expanded
 * directly, (a + b Lt)^l with a = 1 - shift/l, b = -scale/l; a monomial
 * polynomial through its coefficients in L.  out HOST [degree+1]. */
sped_status sped_poly_rebase(const sped_poly *p, double shift, double scale, double *out);

/*
 * sped_apply_poly -- Y = M X for the polynomial p (Sec. 4.2): `degree` fused
 * sparse-times-block steps, each U' = a (L U) + b U + g X.
 *  X  DEVICE n x k (ldx), dtype xdt in {F32, BF16}
 *  Y  DEVICE n x k (ldy), dtype ydt in {F32, BF16}; must not overlap X
 *  intermediate blocks are F32 and live in the workspace.
 */
sped_status sped_apply_poly(const sped_csr *L, const sped_poly *p, int64_t k, const void *X,
                            int64_t ldx, int32_t xdt, void *Y, int64_t ldy, int32_t ydt,
                            void *ws, size_t *ws_bytes, sped_stream_t stream);

/*
 * sped_apply_poly_noalloc -- sped_apply_poly for callers that cannot allocate
 * device memory or pass a workspace: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, kernels
 * and results (bit for bit) as sped_apply_poly, without (ws, ws_bytes).
 * The chain's intermediate F32 blocks live in a library-owned static device
 * array of SPED_NOALLOC_SCRATCH_BYTES (64 MiB), one per GPU, held from the
 * library's load on that GPU until the process ends; this call allocates nothing.
 * Limit: degree >= 3 needs two blocks of n x k floats (each rounded up to
 * 256 bytes), degree 2 one, degree 1 none; larger n x k returns
 * SPED_E_WORKSPACE before any launch (n k <= 8,388,608 at degree >= 3, e.g.
 * 262,144 x 32).  Every call on a GPU shares that GPU's array: calls that
 * overlap in time on one GPU (different streams or threads) race and give
 * wrong results; serialise them.  Uses the current device's array; `stream`
 * must belong to the current device.  Asynchronous on `stream`.
 */
#define SPED_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sped_status sped_apply_poly_noalloc(const sped_csr *L, const sped_poly *p, int64_t k, const void *X,
                                    int64_t ldx, int32_t xdt, void *Y, int64_t ldy, int32_t ydt,
                                    sped_stream_t stream);

/*
 * sped_apply_poly_blocked -- Y = M X as sped_apply_poly, with the chain's
 * steps fused two at a time (a matrix-powers form for graphs whose rows are
 * ordered by community).  Sec. 4.3 weighs ways of forming a product of l
 * factors (a binary tree in log l time, or walks that use L's incidence
 * structure); this fuses consecutive factors per block of rows instead.  Each launch gives one workgroup the `block_rows` consecutive
 * rows [b B, (b+1) B): it loads their rows of the current block into LDS,
 * forms the first step's rows there (neighbours outside the block read from
 * global memory), overwrites the LDS copy with them, and forms the second
 * step (neighbours outside the block are recomputed from the first step's
 * input).  The intermediate block never reaches global memory.  An odd
 * degree ends with one single fused step.  Equal to sped_apply_poly up to the
 * order of the float32 sums; fast only when most neighbours of a row lie in
 * its block.
 *  X, Y        DEVICE F32 n x k, 16-byte aligned, ldx and ldy multiples of 4
 *  k           4, 8, 16, 32 or 64
 *  block_rows  1 .. min(8 x 4096 / k, 160 KiB / (4 k)) (1000 for k = 32)
 *  ws          two n x k F32 blocks plus the heavy rows' step scratch, or the
 *              size-query form
 * Asynchronous on `stream`.
 */
sped_status sped_apply_poly_blocked(const sped_csr *L, const sped_poly *p, int64_t block_rows, int64_t k,
                                    const void *X, int64_t ldx, int32_t xdt, void *Y, int64_t ldy, int32_t ydt,
                                    void *ws, size_t *ws_bytes, sped_stream_t stream);

/*
 * sped_apply_poly_stochastic -- unbiased random-walk estimate of
 * Y = sum_{i=0..degree} coeffs[i] L^i X (Sec. 4.3: eq. walk_summand, Table 1,
 * the edge-incidence graph with self-loops, rejection sampling, prefix reuse).
 * coeffs HOST [degree+1] are monomial coefficients in L itself.
 *  sampler 0 (importance, row-owned): `walks` walks start at every row; the
 *    first edge is uniform over the row's edges, each next edge uniform over
 *    the deg_H = d_a + d_b - 1 edges incident to the current edge (d_a of them
 *    at its first endpoint, including itself, then the others at the second);
 *    prefix i adds coeffs[i] * omega_i * (x_{e_i}^T X) with
 *    omega_i = alpha_c (x_{e_1})_r / q(c); the row's sum is divided by `walks`
 *    and coeffs[0] X added.  Deterministic (no atomics).
 *  sampler 1 (rejection, the paper's literal sampler): `walks` trials, first
 *    edge uniform over all edges, prefix i accepted with probability
 *    prod_{t<i} deg_H(e_t) / (2 deg* - 1); accepted prefixes add
 *    |E| (2 deg* - 1)^{i-1} / walks * coeffs[i] alpha_c x_{e_1} (x_{e_i}^T X)
 *    to both endpoints of e_1 (float atomics: summation order varies).
 *    Requires ydt = F32.  accept_counts (DEVICE int64 [degree], or NULL) gets
 *    the number of accepted trials per prefix length (overwritten).
 * Random numbers: Philox4x32-10 with key (seed mod 2^32, seed >> 32) and
 * counter (c0, c1, counter, (step << 8) | j); importance: c0 = row,
 * c1 = walk; rejection: c0 = trial mod 2^32, c1 = (trial >> 32) | 2^31.  Step 0
 * draws e_1, step t draws e_{t+1}; the rejection sampler's accept uniform for
 * prefix i uses step degree + i, words 0 and 1: (w0 2^21 + (w1 >> 11)) 2^-53.
 * Bounded draws use Lemire's multiply-shift with rejection, consuming the 4
 * words of j = 0, 1, ... in order.  counter < 2^32, degree <= 255,
 * walks >= 1 (sampler 1: walks < 2^63).
 */
sped_status sped_apply_poly_stochastic(const sped_csr *L, const double *coeffs, int32_t degree,
                                       int64_t k, const void *X, int64_t ldx, int32_t xdt,
                                       void *Y, int64_t ldy, int32_t ydt, int32_t sampler,
                                       int64_t walks, uint64_t seed, uint64_t counter,
                                       int64_t *accept_counts, void *ws, size_t *ws_bytes,
                                       sped_stream_t stream);

/*
 * sped_apply_poly_hybrid -- unbiased estimate of Y = sum_{i=0..degree} c_i L^i X
 * with the low-order terms exact and only the tail sampled (a variance
 * reduction of the Sec. 4.3 estimator; Sec. 6 leaves variance open):
 *   Y = sum_{i<m} c_i L^i X + L^m T,  T = walk estimate of sum_{j>=0} c_{m+j} L^j X
 * with m = exact_terms.  Since L^m commutes with the tail polynomial,
 * E[L^m T] is the tail sum_{i>=m} c_i L^i X.  T is one
 * sped_apply_poly_stochastic call with the shifted coefficients (c_m, ...,
 * c_degree) and the same sampler, walks, seed and counter, so its walks are
 * those of that call; then m fused sparse steps U <- L U + c_i X
 * (i = m-1 .. 0, float32 intermediates) give Y.  m = 0 is the plain
 * estimate; m = degree uses no walks (exact Horner evaluation, X scaled by
 * c_degree in the first step).  Cost: m sparse steps plus walks of length
 * degree - m.
 *  coeffs     HOST [degree+1] monomial coefficients in L; degree 1..255
 *  exact_terms 0..degree
 *  X, Y       DEVICE n x k (ldx, ldy), F32 or BF16 each; must not overlap
 *  sampler    0 importance, 1 rejection (with m = 0 the rejection sampler
 *             needs a float32 Y; with m >= 1 its tail goes to float32 scratch)
 *  ws         DEVICE scratch: n k floats for m = 1, 2 n k for m >= 2; or the
 *             size query
 * Asynchronous on `stream`.  Errors as sped_apply_poly_stochastic.
 */
sped_status sped_apply_poly_hybrid(const sped_csr *L, const double *coeffs, int32_t degree,
                                   int32_t exact_terms, int64_t k, const void *X, int64_t ldx,
                                   int32_t xdt, void *Y, int64_t ldy, int32_t ydt, int32_t sampler,
                                   int64_t walks, uint64_t seed, uint64_t counter, void *ws,
                                   size_t *ws_bytes, sped_stream_t stream);

/*
 * sped_apply_limit_lazy -- unbiased random estimate of Y = (I - L/ell)^ell X,
 * the limit approximation of Table 2 (the default dilation), by lazy random
 * walks on the nodes: a lower-variance estimator than the edge chains of
 * Sec. 4.3 for this polynomial (the variance question Sec. 6 leaves open).
 * For the normalised L, I - L/ell = D^{1/2} P D^{-1/2} with P the lazy walk
 * that stays with probability 1 - 1/ell and otherwise moves to neighbour j with
 * probability w_ij / d_i, so Y_r = E[s_Z X_Z] / s_r over the walk's position Z
 * after ell steps from r.  For the combinatorial L, I - L/ell is itself the
 * lazy walk (move with probability d_z / ell; requires ell >= max_i d_i), and
 * Y_r = E[X_Z].  Each output row averages `walks` walks; each walk gathers one
 * row of X.  Draws: Philox4x32-10 keyed by seed, counter (r, walk, counter,
 * step << 8 | j); the stays before each move are drawn at once as a geometric
 * variable (one draw per move, not per step); moves propose uniform
 * neighbours accepted with probability w_j / max w (ratios within 2^-20 of 1
 * accept), falling back after 16 rejections to an exact inverse-CDF draw.
 *  ell     1..255
 *  X       DEVICE n x k (ldx), F32 or BF16; Y DEVICE n x k (ldy), F32 or BF16;
 *          X and Y must not overlap
 *  ws      DEVICE scratch (n doubles: each row's largest move weight) or the
 *          size-query form
 * Asynchronous on `stream`.
 */
sped_status sped_apply_limit_lazy(const sped_csr *L, int32_t ell, int64_t k, const void *X,
                                  int64_t ldx, int32_t xdt, void *Y, int64_t ldy, int32_t ydt,
                                  int64_t walks, uint64_t seed, uint64_t counter, void *ws,
                                  size_t *ws_bytes, sped_stream_t stream);

/*
 * sped_poly_backward -- coefficient gradient of Y = sum_j theta_j Lt^j X
 * (learnable dilation coefficients, the meta-learning direction of Sec. 6):
 * dtheta[j] = <dY, Lt^j X>_F for j = 0..degree, with Lt = (L - shift I)/scale.
 * The powers Lt^j X are recomputed step by step and never stored; each step
 * fuses the inner product into the sparse product.  The X gradient
 * p(L) dY is sped_apply_poly on dY (L is symmetric).
 *  X, dY   DEVICE F32 n x k (ldx, lddy)
 *  dtheta  DEVICE double [degree+1] (overwritten)
 */
sped_status sped_poly_backward(const sped_csr *L, int32_t degree, double shift, double scale,
                               int64_t k, const float *X, int64_t ldx, const float *dY,
                               int64_t lddy, double *dtheta, void *ws, size_t *ws_bytes,
                               sped_stream_t stream);

/*
 * sped_gram -- G = A^T B in float64 (the inner products behind the projector
 * V V^dagger of the subspace-error metric, Sec. 5.2, and the orthonormalisation
 * of a block solver).  A DEVICE n x ka (lda), B DEVICE n x kb (ldb), both of
 * dtype dt in {F32, BF16}; G DEVICE double ka x kb row-major (overwritten).
 * Products are upconverted to float64 and accumulated with float64 matrix-core
 * instructions in a fixed order (bitwise reproducible).  ka, kb <= 128.
 */
sped_status sped_gram(int64_t n, int64_t ka, int64_t kb, const void *A, int64_t lda,
                      const void *B, int64_t ldb, int32_t dt, double *G, void *ws,
                      size_t *ws_bytes, sped_stream_t stream);

/*
 * sped_orthonormalize -- in place V <- V R^{-1} with R the Cholesky factor of
 * V^T V (Cholesky QR), repeated `passes` times (2 = CholQR2).  If a pivot
 * breaks down, the Gram matrix is shifted by a multiple of its trace and the
 * factorisation retried.  V DEVICE n x k (ldv), dtype F32 or BF16 (the Gram
 * is float64 either way; products are rounded to V's dtype); k <= 96.
 * R_out DEVICE double k x k or NULL: R of the last pass (upper triangular).
 */
sped_status sped_orthonormalize(int64_t n, int64_t k, void *V, int64_t ldv, int32_t dt,
                                int32_t passes, double *R_out, void *ws, size_t *ws_bytes,
                                sped_stream_t stream);

/*
 * sped_rayleigh_ritz -- Ritz pairs of L on span(Q) for orthonormal Q
 * (the eigenvector estimate of an iterative solver, Sec. 3 and Sec. 5):
 * Z = L Q, H = Q^T Z (float64), H = S Theta S^T with Theta ascending,
 * Q <- Q S, and residuals resid[i] = ||L q_i - theta_i q_i||_2.
 *  Q DEVICE F32 n x k (ldq), updated in place; k <= 96
 *  theta, resid DEVICE double [k]
 */
sped_status sped_rayleigh_ritz(const sped_csr *L, int64_t k, void *Q, int64_t ldq, int32_t dt,
                               double *theta, double *resid, void *ws, size_t *ws_bytes,
                               sped_stream_t stream);

/*
 * sped_bottomk_solve -- bottom-k eigenvectors of L (Sec. 1 and 3): block
 * subspace iteration (or block Oja with step eta) on the reversed operator
 * M = p(L) (eq. reveig; p = NULL means the identity transform reversed,
 * M = lambda_bound I - L), Cholesky-QR2 after every application, and a
 * Rayleigh-Ritz step on L every check_every iterations.  mu-EigenGame (the
 * other solver Sec. 5 names) instead moves each unit vector v_i along its
 * projected gradient M v_i - sum_{j<i} <v_i, M v_j> v_j (minus its v_i part)
 * with step eta and renormalises; its checks run Rayleigh-Ritz on an
 * orthonormalised copy.  The block carries
 * k + guard columns; the stopping test is
 *     rho / (theta_k - ||r_k|| - theta_{k-1}) <= tol,   R = [L q_i - theta_i q_i]_{i<k}
 * with rho = sqrt(min(||R^T R||_inf, ||R||_F^2)) >= ||R||_2 (R^T R in float64)
 * (a Davis-Kahan bound on the sine of the largest angle to the true bottom-k
 * subspace; the gap is estimated from the first guard Ritz value theta_k
 * lowered by its residual r_k; guard >= 1).
 *  V0      DEVICE F32 n x (k+guard) (ldv0): start block
 *  V_out   DEVICE F32 n x k (ldvo): Ritz vectors, ascending (mu-EigenGame: the
 *          game's own unit vectors, players in order)
 *  vdt     storage of the iterate: F32, or BF16 (float32 sums, float64 Gram,
 *          Cholesky and Rayleigh-Ritz) until the bound reaches coarse_tol or
 *          the largest residual stops improving (8 checks without a 2% drop:
 *          bf16's rounding floor),
 *          followed by a float32 refinement sweep down to tol
 *  evals   HOST double [k]: Ritz values of L, ascending (for mu-EigenGame those
 *          of L on the span of its vectors)
 *  resid   HOST double [k] or NULL: final residual norms
 *  o, st   HOST options / statistics
 * Synchronous: each check copies 2(k + guard) + 3 doubles (Ritz values,
 * residual norms, norm bound, flags) into a small pinned host buffer that
 * the call allocates and frees itself.  Returns SPED_E_NOT_CONVERGED (with
 * outputs and stats filled) when max_iters is reached first.  A start block that is rank deficient (a
 * repeated or zero column) has those columns replaced by uniform random ones
 * (Philox keyed by seed) before the first iteration, counted in
 * st->reseeded; a start block that is not finite returns SPED_E_NUMERIC.
 */
typedef struct {
  int32_t solver;          /* 0 = subspace iteration (eta = inf), 1 = block Oja,
                              2 = mu-EigenGame (F32 storage only) */
  double eta;              /* Oja step (iterate on M + I/eta), or the mu-EigenGame step */
  double tol;              /* stopping bound */
  int32_t max_iters;
  int32_t check_every;     /* Rayleigh-Ritz cadence, >= 1 */
  int32_t guard;           /* extra columns, >= 1 */
  int32_t orth_passes;     /* Cholesky-QR passes per iteration (1 or 2) */
  int32_t stochastic_iters;/* first iterations use the random estimate (stochastic_sampler) */
  int64_t walks_per_row;   /* walks per row for those iterations */
  uint64_t seed;           /* Philox key; iteration t (1, 2, ...) uses counter counter_base + t */
  double coarse_tol;       /* BF16 phase stops at this bound (<= 0: 1e-2) */
  int32_t stochastic_sampler; /* 0 = importance edge walks (Sec. 4.3), 1 = lazy node walks
                                 (sped_apply_limit_lazy; needs the limit polynomial, solver 0 or 2) */
  int32_t stochastic_exact_terms; /* sampler 0: the first m terms of the polynomial exact, the
                                     tail sampled (sped_apply_poly_hybrid); 0..degree */
  int32_t use_graphs;      /* nonzero: each exact iteration's launches are captured once into a
                              HIP graph (per buffer pair, storage and check) and replayed
                              (bit-identical results; fewer launch overheads on small graphs) */
  int32_t polish_checks;   /* > 0 with p != NULL (solver 0): the float32 iterations on p(L) end
                              once the largest residual has not dropped by 2% for this many
                              consecutive checks with the bound at or below 1e3 tol (the rounding
                              floor of the degree-l chain), and
                              iterations on the plain operator lambda_bound I - L continue from
                              its Ritz vectors down to tol (one product per iteration: a lower
                              floor).  0: off */
  double *trace;           /* HOST [4 trace_cap] or NULL: each check appends (iteration, seconds
                              since the call began, stopping bound, largest residual) */
  int32_t trace_cap;       /* checks the trace holds; later checks are not recorded */
  uint64_t counter_base;   /* added to the walk counters: a stochastic solve resumed from the
                              block an earlier call returned after T iterations continues that
                              call's random stream with counter_base = T */
} sped_solve_opts;

typedef struct {
  int32_t iters;
  int64_t spmm_count;      /* sparse products applied (chain steps + Rayleigh-Ritz) */
  double seconds;          /* wall time inside the call */
  double max_residual;
  double gap_estimate;
  double bound;            /* the stopping quantity at exit (rho / gap) */
  int32_t converged;
  int32_t cholqr_shifts;   /* breakdowns repaired by the shift */
  int32_t coarse_iters;    /* iterations done with BF16 storage */
  int32_t polish_iters;    /* iterations done on the plain operator after p(L) stalled */
  int32_t trace_len;       /* checks recorded in o->trace */
  int32_t reseeded;        /* start-block columns replaced by random ones (rank deficient V0) */
} sped_solve_stats;

sped_status sped_bottomk_solve(const sped_csr *L, const sped_poly *p, int64_t k, const void *V0,
                               int64_t ldv0, void *V_out, int64_t ldvo, int32_t vdt,
                               double *evals, double *resid, const sped_solve_opts *o,
                               sped_solve_stats *st, void *ws, size_t *ws_bytes,
                               sped_stream_t stream);

/*
 * sped_cluster_embed -- hard clustering of the spectral embedding with k-means
 * (Sec. 1: the bottom-k eigenvectors embed each node; k-means on them gives
 * the clusters; Sec. 2.1 uses k = 2 on the Fiedler vector).
 *  V              DEVICE n x k (ldv), dtype vdt in {F32, BF16}
 *  row_normalize  nonzero: rows scaled to unit length first
 *  init           DEVICE double n_clusters x k or NULL.  NULL: k-means++
 *                 seeding with Philox draws keyed by `seed` (pick c uses
 *                 counter (c, 0, 0, 0) words 0 and 1 as a 53-bit uniform).
 *  labels         DEVICE int32 [n]: nearest centre (ties: lowest index)
 *  centroids      DEVICE double n_clusters x k
 *  inertia, iters HOST or NULL: final sum of squared distances, Lloyd rounds
 * Lloyd rounds run until no label changes or max_iters.  Distances and
 * centroid sums are float64.  Synchronous.  n_clusters <= 256, k <= 128.
 */
sped_status sped_cluster_embed(const void *V, int64_t n, int64_t k, int64_t ldv, int32_t vdt,
                               int32_t n_clusters, int32_t row_normalize, uint64_t seed,
                               int32_t max_iters, const double *init, int32_t *labels,
                               double *centroids, double *inertia, int32_t *iters, void *ws,
                               size_t *ws_bytes, sped_stream_t stream);

/*
 * Edge-batch products, for graphs whose edge list is not resident on the
 * device (Sec. 3: when the data cannot be held in memory, a solver sees
 * batches of edge vectors x_e; the conclusion's stochastic model).  L is the
 * sum of x_e x_e^T over the edges (Sec. 2, weighted X^T W X), x_e =
 * sqrt(w) (s_i e_i - s_j e_j) with s the node scales (Sec. 4.1; all ones for
 * the combinatorial Laplacian), so a batch B adds, per edge e = (i, j, w),
 *   w s_i (s_i X_i - s_j X_j) to row i and -w s_j (s_i X_i - s_j X_j) to row j.
 * Self-loops add nothing; repeated edges add their weights.  A uniformly drawn
 * batch of b of the m edges, scaled by alpha = m / b, estimates L X without
 * bias; all m edges with alpha = 1 give L X.  Rows are summed with float32
 * atomics, so the order of the additions (and the last bits) varies from run
 * to run.  Y is float32; X is F32 or BF16, n x k with leading dimension ldx;
 * Y must not be X.
 */

/* sped_edge_apply -- Y += alpha sum_{e in batch} x_e x_e^T X for a batch of m
 * DEVICE edges (src, dst int32 [m]; w float [m] or NULL for ones; scale
 * DEVICE float [n] or NULL for ones).  An edge with an endpoint outside
 * [0, n) or a weight that is not finite and > 0 is skipped and counted in
 * *invalid (DEVICE uint64, added to; may be NULL).  Asynchronous. */
sped_status sped_edge_apply(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const float *w,
                            const float *scale, int64_t k, const void *X, int64_t ldx, int32_t xdt, float *Y,
                            int64_t ldy, float alpha, unsigned long long *invalid, sped_stream_t stream);

/* sped_stream_node_scales -- the weighted degrees d (DEVICE double [n]) and
 * node scales s (DEVICE float [n]: d^{-1/2}, 0 for d = 0, under
 * SPED_LAP_SYM_NORMALIZED; 1 under SPED_LAP_COMBINATORIAL) of the graph whose
 * m edges are HOST arrays src_h, dst_h (int32) and w_h (float, or NULL for
 * ones), read in batches of `batch` edges (pinned host memory lets the copies
 * overlap the kernels).  Workspace: two staging batches.  Synchronises
 * `stream`; the host arrays may be released on return.  Invalid edges (as
 * above) are skipped and make the call return SPED_E_INVALID. */
sped_status sped_stream_node_scales(int64_t n, int64_t m, const int32_t *src_h, const int32_t *dst_h,
                                    const float *w_h, int32_t kind, int64_t batch, double *degree, float *scale,
                                    void *ws, size_t *ws_bytes, sped_stream_t stream);

/* sped_stream_laplacian_apply -- Y = alpha sum_e x_e x_e^T X (accumulate = 0)
 * or Y += that (accumulate != 0) over the m HOST edges src_h, dst_h, w_h,
 * streamed in batches of `batch` edges: the copy of each batch overlaps the
 * previous batch's kernel.  scale: DEVICE float [n] (from
 * sped_stream_node_scales) or NULL for the combinatorial Laplacian.
 * Workspace: two staging batches.  Synchronises `stream`.  Invalid edges are
 * skipped and make the call return SPED_E_INVALID. */
sped_status sped_stream_laplacian_apply(int64_t n, int64_t m, const int32_t *src_h, const int32_t *dst_h,
                                        const float *w_h, const float *scale, int64_t k, const void *X, int64_t ldx,
                                        int32_t xdt, float *Y, int64_t ldy, float alpha, int32_t accumulate,
                                        int64_t batch, void *ws, size_t *ws_bytes, sped_stream_t stream);

/* sped_minibatch_oja -- `iters` Oja steps V <- orth(V + eta M_hat V) on a
 * host-resident edge list (Sec. 3: edge vectors fed to the solver in
 * minibatches; Sec. 5: Oja's update; orth = Cholesky QR, two passes).  Batch
 * j of the call is the run of `batch` edges of the host arrays that starts at
 * a uniform random offset o_J and wraps past the end: edges (o_J + r) mod m,
 * r < batch, with J = batch0 + j and o_J = Lemire's bounded draw in [0, m)
 * from Philox4x32-10 keyed by seed, counter (J mod 2^32, J >> 32, 0, 0), the
 * words of j' = 0, 1, ... in order (as sped_apply_poly_stochastic's draws).
 * Every edge is in a batch with probability b / m, and different batches are
 * independent; each batch is scaled by m / b.  (Shuffle the list once if its
 * order is not random: the edges of one batch are then a uniform sample.)
 *  degree 0:   M_hat V = lambda_bound V - (m / b) L_B V (the plain reversed
 *              operator, one batch per step);
 *  degree l:   M_hat V = (I - (m / b) L_{B_l} / l) ... (I - (m / b) L_{B_1} / l) V,
 *              the limit polynomial (I - L/l)^l with its own batch per factor;
 *              independent factors make E[M_hat] = (I - L/l)^l (l batches per
 *              step).
 * A solve split over several calls continues the same batch stream when each
 * call passes batch0 = the number of batches drawn before it (iters x max(1,
 * degree) per call).
 * scale as in sped_stream_laplacian_apply; V DEVICE float n x k (ldv), k <= 96,
 * updated in place.  1 <= batch <= m < 2^32.  Workspace: two staging
 * batches, two n x k float blocks and the orthonormalisation's.  Synchronises
 * `stream`; invalid edges are skipped and make the call return
 * SPED_E_INVALID. */
sped_status sped_minibatch_oja(int64_t n, int64_t m, const int32_t *src_h, const int32_t *dst_h, const float *w_h,
                               const float *scale, int32_t degree, double lambda_bound, int64_t k, float *V,
                               int64_t ldv, int64_t batch, double eta, int32_t iters, uint64_t seed,
                               int64_t batch0, void *ws, size_t *ws_bytes, sped_stream_t stream);

/*
 * sped_stream_copy -- dst <- src, `bytes` bytes (multiple of 16, 16-byte
 * aligned DEVICE pointers): a plain streaming copy used to calibrate the
 * chip's achievable HBM bandwidth and its memory counters.
 */
sped_status sped_stream_copy(const void *src, void *dst, size_t bytes, sped_stream_t stream);

/*
 * sped_gather_probe -- the chip's rate for the sparse step's load pattern:
 * `blocks` x 256 threads, each 8-lane group loading `iters` 128-byte rows of
 * `table` (16 bytes per lane, 8 rows per wavefront instruction, 8 loads in
 * flight), rows pseudo-random per group (scattered != 0) or 8 consecutive rows
 * per wavefront.  A measurement aid like sped_stream_copy.
 *  table  DEVICE, 16-byte aligned, rows x 128 bytes; rows a power of two >= 8
 *  iters  positive multiple of 8
 *  out    DEVICE uint32 [blocks x 256] (overwritten; keeps the loads alive)
 */
sped_status sped_gather_probe(const void *table, int64_t rows, int32_t iters, int32_t scattered,
                              int32_t blocks, uint32_t *out, sped_stream_t stream);

/* Message for the last non-OK status on this thread ("" if none). */
const char *sped_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int32_t sped_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPED_H */
