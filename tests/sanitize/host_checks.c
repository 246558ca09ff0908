/* Host-only exercise of libsped's argument validation and workspace size
 * queries, for a build whose host code carries AddressSanitizer and
 * UndefinedBehaviorSanitizer.  No call here reaches the GPU: every case is
 * refused on the host or answers a size query.  Exit status 0 when every
 * call returned the expected status. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "sped.h"

static int failures = 0;

static void expect(const char *what, sped_status got, sped_status want) {
  if (got != want) {
    fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, sped_last_error());
    ++failures;
  }
}

int main(void) {
  size_t need = 0;
  double coeffs[17], shift = 0.0, scale = 1.0;
  /* Table 2 coefficients for every transform and a range of degrees */
  for (int t = 0; t <= 3; ++t)
    for (int deg = 1; deg <= 16; ++deg) {
      sped_status st = sped_transform_coeffs(t, t == SPED_T_PLAIN ? 1 : deg, 2.0, 1e-3, coeffs, &shift, &scale);
      int even_log = t == SPED_T_TAYLOR_LOG && deg % 2 == 0;
      expect("transform_coeffs", st, even_log ? SPED_E_UNSUPPORTED : SPED_OK);
    }
  expect("transform_coeffs bad kind", sped_transform_coeffs(9, 4, 2.0, 1e-3, coeffs, &shift, &scale), SPED_E_INVALID);

  sped_csr c;
  memset(&c, 0, sizeof c);
  c.n = 1000;
  c.nnz = 8000;
  c.kind = SPED_LAP_SYM_NORMALIZED;
  /* fake, 256-byte aligned device addresses: never dereferenced on these paths */
  c.rowptr = (int64_t *)(uintptr_t)0x10000;
  c.col = (int32_t *)(uintptr_t)0x20000;
  c.val = (float *)(uintptr_t)0x30000;
  c.diag = (float *)(uintptr_t)0x40000;
  c.scale = (float *)(uintptr_t)0x50000;
  void *X = (void *)(uintptr_t)0x100000, *Y = (void *)(uintptr_t)0x800000;
  sped_poly p = {SPED_POLY_LIMIT, 16, NULL, 0.0, 1.0};
  double mono[17], rebased[17];
  expect("poly_monomial", sped_poly_monomial(&p, mono), SPED_OK);
  expect("poly_rebase", sped_poly_rebase(&p, 1.0, 1.0, rebased), SPED_OK);
  expect("apply_poly query", sped_apply_poly(&c, &p, 32, X, 32, SPED_F32, Y, 32, SPED_F32, NULL, &need, NULL),
         SPED_OK);
  expect("apply_poly NULL csr", sped_apply_poly(NULL, &p, 32, X, 32, SPED_F32, Y, 32, SPED_F32, NULL, &need, NULL),
         SPED_E_INVALID);
  expect("apply_poly ld < k", sped_apply_poly(&c, &p, 32, X, 16, SPED_F32, Y, 32, SPED_F32, NULL, &need, NULL),
         SPED_E_INVALID);
  expect("apply_poly f64", sped_apply_poly(&c, &p, 32, X, 32, SPED_F64, Y, 32, SPED_F32, NULL, &need, NULL),
         SPED_E_UNSUPPORTED);
  sped_poly bad = {SPED_POLY_MONOMIAL, 0, coeffs, 0.0, 1.0};
  expect("apply_poly degree 0", sped_apply_poly(&c, &bad, 32, X, 32, SPED_F32, Y, 32, SPED_F32, NULL, &need, NULL),
         SPED_E_INVALID);
  expect("noalloc too large", sped_apply_poly_noalloc(&c, &p, 1 << 20, X, 1 << 20, SPED_F32, Y, 1 << 20, SPED_F32,
                                                      NULL), SPED_E_WORKSPACE);
  expect("blocked k", sped_apply_poly_blocked(&c, &p, 125, 12, X, 12, SPED_F32, Y, 12, SPED_F32, NULL, &need, NULL),
         SPED_E_UNSUPPORTED);
  expect("blocked query", sped_apply_poly_blocked(&c, &p, 1000, 32, X, 32, SPED_F32, Y, 32, SPED_F32, NULL, &need,
                                                  NULL), SPED_OK);
  expect("stochastic counter", sped_apply_poly_stochastic(&c, coeffs, 4, 8, X, 8, SPED_F32, Y, 8, SPED_F32, 0, 8, 1,
                                                          (uint64_t)1 << 33, NULL, NULL, &need, NULL),
         SPED_E_INVALID);
  expect("lazy ell", sped_apply_limit_lazy(&c, 0, 8, X, 8, SPED_F32, Y, 8, SPED_F32, 8, 1, 0, NULL, &need, NULL),
         SPED_E_INVALID);
  expect("backward degree", sped_poly_backward(&c, -1, 0.0, 1.0, 8, (const float *)X, 8, (const float *)Y, 8, NULL,
                                               NULL, &need, NULL), SPED_E_INVALID);
  expect("gram query", sped_gram(1000, 32, 32, X, 32, Y, 32, SPED_F32, (double *)(uintptr_t)0x900000, NULL, &need,
                                 NULL), SPED_OK);
  expect("orthonormalize k > n", sped_orthonormalize(3, 5, X, 5, SPED_F32, 2, NULL, NULL, &need, NULL),
         SPED_E_INVALID);
  expect("rayleigh_ritz k", sped_rayleigh_ritz(&c, 200, X, 200, SPED_F32, NULL, NULL, NULL, &need, NULL),
         SPED_E_INVALID);
  sped_solve_opts o;
  memset(&o, 0, sizeof o);
  o.tol = 1e-6;
  o.max_iters = 10;
  o.check_every = 1;
  o.guard = 4;
  o.orth_passes = 2;
  double evals[10];
  sped_solve_stats stt;
  expect("solve query", sped_bottomk_solve(&c, &p, 10, X, 14, Y, 10, SPED_F32, evals, NULL, &o, &stt, NULL, &need,
                                           NULL), SPED_OK);
  o.guard = 0;
  expect("solve guard 0", sped_bottomk_solve(&c, &p, 10, X, 14, Y, 10, SPED_F32, evals, NULL, &o, &stt, NULL, &need,
                                             NULL), SPED_E_INVALID);
  o.guard = 4;
  o.polish_checks = 2;
  o.solver = 1;
  o.eta = 1.0;
  expect("solve polish with Oja", sped_bottomk_solve(&c, &p, 10, X, 14, Y, 10, SPED_F32, evals, NULL, &o, &stt, NULL,
                                                     &need, NULL), SPED_E_UNSUPPORTED);
  o.polish_checks = 0;
  o.solver = 0;
  o.trace_cap = 5;
  expect("solve trace NULL", sped_bottomk_solve(&c, &p, 10, X, 14, Y, 10, SPED_F32, evals, NULL, &o, &stt, NULL,
                                                &need, NULL), SPED_E_INVALID);
  expect("cluster too many", sped_cluster_embed(X, 10, 2, 2, SPED_F32, 11, 1, 0, 10, NULL, NULL, NULL, NULL, NULL,
                                                NULL, &need, NULL), SPED_E_INVALID);
  int32_t src[4] = {0, 1, 2, 3}, dst[4] = {1, 2, 3, 0};
  sped_csr out;
  memset(&out, 0, sizeof out);
  expect("laplacian query", sped_laplacian_csr(4, 4, src, dst, NULL, SPED_LAP_SYM_NORMALIZED, 0, &out, NULL, NULL,
                                               &need, NULL), SPED_OK);
  expect("laplacian kind", sped_laplacian_csr(4, 4, src, dst, NULL, 7, 0, &out, NULL, NULL, &need, NULL),
         SPED_E_INVALID);
  expect("edge_apply k", sped_edge_apply(10, 4, src, dst, NULL, NULL, 0, X, 4, SPED_F32, Y, 4, 1.0f, NULL, NULL),
         SPED_E_INVALID);
  printf("%s: %d failure(s); version %d\n", failures ? "FAIL" : "ok", failures, (int)sped_version());
  return failures ? 1 : 0;
}
