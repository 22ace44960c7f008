/*
 * Host-side driver for the sanitizer build (tests/test_sanitize.py): the CPU
 * oracle (built with AddressSanitizer and UndefinedBehaviorSanitizer) on
 * small, ragged and degenerate inputs, and the C ABI's host-side paths
 * (argument checks, workspace queries, status strings) that return before
 * any device work. Exit status = number of failed checks; the sanitizers
 * abort on the first report.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "trinv.h"

int64_t oracle_tril_inverse(int64_t n, const double *L, int64_t ldl, int32_t unit, double *X, int64_t ldx);
int64_t oracle_tril_inverse_columns(int64_t n, const double *L, int64_t ldl, int32_t unit, const int64_t *cols,
                                    int64_t ncols, double *out);
int64_t oracle_chain_sum_inverse(int64_t n, const double *L, int64_t ldl, int32_t unit, double *X, int64_t ldx);
int64_t oracle_chain_count(int64_t a, int64_t b);
int64_t oracle_crout_lu(int64_t n, const double *A, int64_t lda, double *L, double *U);
int64_t oracle_factored_inverse(int64_t n, const double *L, int64_t ldl, int32_t l_unit, const double *U,
                                int64_t ldu, int32_t u_unit, double *Linv, double *Uinv, double *Ainv);
int64_t oracle_tril_inverse_backward(int64_t n, const double *L, int64_t ldl, const double *G, int64_t ldg,
                                     double *grad);
int64_t oracle_tril_inverse_backward_rows(int64_t n, const double *L, int64_t ldl, const double *G, int64_t ldg,
                                          const int64_t *rows, int64_t nrows, double *out);
void oracle_residuals(int64_t n, const double *L, int64_t ldl, const double *X, int64_t ldx, double *out);
void oracle_residual_matrix(int64_t n, const double *L, int64_t ldl, const double *X, int64_t ldx, double *out);
void oracle_residual_columns(int64_t n, const double *L, int64_t ldl, const double *X, int64_t ldx,
                             const int64_t *cols, int64_t ncols, double *out);
int64_t oracle_sqr(int64_t n, const double *A, int64_t lda, double *Q, double *R, double *S);
int64_t oracle_inverse(int64_t n, const double *A, int64_t lda, double *X);

static int failures = 0;

#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "check failed (line %d): %s\n", __LINE__, #cond); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

/* xorshift64*: deterministic inputs without the C library's rand() */
static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand(void) {
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (double)((rng_state * 0x2545f4914f6cdd1dull) >> 11) * (1.0 / 9007199254740992.0);
}

/* exactly-sized allocations, so that any overrun is a sanitizer report */
static double *alloc(int64_t count) { return (double *)calloc((size_t)(count > 0 ? count : 1), sizeof(double)); }

static void lower(int64_t n, int64_t ld, double *L, int unit_like) {
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < ld; ++j)
      L[i * ld + j] = j < i ? (urand() - 0.5) / (double)(n > 1 ? n : 1) : (j == i ? (unit_like ? 1.0 : 1.0 + urand()) : 0.0);
}

static double max_abs_lx_minus_i(int64_t n, const double *L, int64_t ldl, const double *X, int64_t ldx) {
  double m = 0.0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (int64_t k = 0; k < n; ++k) s += L[i * ldl + k] * X[k * ldx + j];
      s -= (i == j) ? 1.0 : 0.0;
      if (fabs(s) > m) m = fabs(s);
    }
  return m;
}

static void oracle_cases(void) {
  const int64_t sizes[] = {0, 1, 2, 3, 7, 17, 33};
  for (size_t t = 0; t < sizeof(sizes) / sizeof(sizes[0]); ++t) {
    const int64_t n = sizes[t], ld = n + 3;
    double *L = alloc(n * ld), *X = alloc(n * ld), *G = alloc(n * n), *grad = alloc(n * n);
    lower(n, ld, L, 0);
    CHECK(oracle_tril_inverse(n, L, ld, 0, X, ld) == 0);
    CHECK(max_abs_lx_minus_i(n, L, ld, X, ld) < 1e-12);
    /* unit diagonal: the stored diagonal is not read */
    for (int64_t i = 0; i < n; ++i) L[i * ld + i] = 7.0;
    CHECK(oracle_tril_inverse(n, L, ld, 1, X, ld) == 0);
    for (int64_t i = 0; i < n; ++i) CHECK(X[i * ld + i] == 1.0);
    lower(n, ld, L, 0);
    if (n > 0) {
      int64_t cols[2] = {0, n - 1};
      double *out = alloc(2 * n);
      CHECK(oracle_tril_inverse_columns(n, L, ld, 0, cols, 2, out) == 0);
      free(out);
      double res[4];
      CHECK(oracle_tril_inverse(n, L, ld, 0, X, ld) == 0);
      oracle_residuals(n, L, ld, X, ld, res);
      CHECK(res[0] < 1e-12 * (1.0 + res[2] * res[3]));
      double *R = alloc(n * n), *rc = alloc(2);
      oracle_residual_matrix(n, L, ld, X, ld, R);
      oracle_residual_columns(n, L, ld, X, ld, cols, 2, rc);
      free(R);
      free(rc);
      for (int64_t i = 0; i < n * n; ++i) G[i] = urand() - 0.5;
      CHECK(oracle_tril_inverse_backward(n, L, ld, G, n, grad) == 0);
      int64_t rows[1] = {n / 2};
      double *gr = alloc(n);
      CHECK(oracle_tril_inverse_backward_rows(n, L, ld, G, n, rows, 1, gr) == 0);
      free(gr);
      /* singular: zero diagonal at position n/2 reported 1-based */
      L[(n / 2) * ld + n / 2] = 0.0;
      CHECK(oracle_tril_inverse(n, L, ld, 0, X, ld) == n / 2 + 1);
    }
    if (n <= 17) {
      lower(n, ld, L, 1);
      CHECK(oracle_chain_sum_inverse(n, L, ld, 1, X, ld) == 0);
      CHECK(max_abs_lx_minus_i(n, L, ld, X, ld) < 1e-12);
    }
    free(L);
    free(X);
    free(G);
    free(grad);
  }
  CHECK(oracle_chain_count(0, 1) == 1);
  CHECK(oracle_chain_count(1, 5) == 8);
  CHECK(oracle_chain_count(3, 3) == 0);

  const int64_t dn[] = {1, 5, 12};
  for (size_t t = 0; t < sizeof(dn) / sizeof(dn[0]); ++t) {
    const int64_t n = dn[t];
    double *A = alloc(n * n), *L = alloc(n * n), *U = alloc(n * n), *Q = alloc(n * n), *R = alloc(n * n),
           *S = alloc(n * n), *Ai = alloc(n * n), *Li = alloc(n * n), *Ui = alloc(n * n), *Af = alloc(n * n);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) A[i * n + j] = (i == j ? (double)n + 1.0 : 0.0) + urand() - 0.5;
    CHECK(oracle_crout_lu(n, A, n, L, U) == 0);
    CHECK(oracle_factored_inverse(n, L, n, 0, U, n, 1, Li, Ui, Af) == 0);
    CHECK(oracle_sqr(n, A, n, Q, R, S) == 0);
    CHECK(oracle_inverse(n, A, n, Ai) == 0);
    double m = 0.0;
    for (int64_t i = 0; i < n * n; ++i) m = fmax(m, fabs(Ai[i] - Af[i]));
    CHECK(m < 1e-10);
    free(A); free(L); free(U); free(Q); free(R); free(S); free(Ai); free(Li); free(Ui); free(Af);
  }
}

/* fake device addresses: every call below must return before using them */
#define P(x) ((void *)(uintptr_t)(x))

static void abi_cases(void) {
  trinv_opts o;
  trinv_default_opts(&o);
  CHECK(o.leaf == 0 && o.upper == 0 && o.max_iter > 0 && o.tol > 0.0);
  for (int s = -3; s < 12; ++s) CHECK(trinv_status_string(s) != NULL && strlen(trinv_status_string(s)) > 0);

  CHECK(trinv_workspace_bytes(TRINV_F64, 0, NULL) == 0);
  CHECK(trinv_workspace_bytes(TRINV_F64, 1024, NULL) > 0);
  CHECK(trinv_workspace_bytes(TRINV_BF16_REFINE, (int64_t)1 << 40, NULL) == 0);
  CHECK(trinv_backward_workspace_bytes(TRINV_F32, 4, 100) >= 4 * 100 * 100 * 4);
  CHECK(trinv_residual_workspace_bytes(TRINV_F64, 300) > 0);
  CHECK(trinv_refine_residual_workspace_bytes(TRINV_BF16_REFINE, (int64_t)1 << 40) == 0);

  trinv_info info;
  CHECK(trinv_tril_inverse(TRINV_F64, -1, NULL, 0, NULL, 0, NULL, NULL, 0, NULL, &info) == TRINV_ERR_ARG);
  CHECK(trinv_tril_inverse(TRINV_F64, 10, P(8), 5, P(16), 10, NULL, NULL, 0, NULL, NULL) == TRINV_ERR_ARG);
  CHECK(trinv_tril_inverse(TRINV_F64, 10, NULL, 10, NULL, 10, NULL, NULL, 0, NULL, NULL) == TRINV_ERR_ARG);
  CHECK(trinv_tril_inverse(9, 10, P(8), 10, P(4096), 10, NULL, NULL, 0, NULL, NULL) == TRINV_ERR_UNSUPPORTED);
  CHECK(trinv_tril_inverse(TRINV_F64, 10, P(4096), 10, P(4096 + 8), 10, NULL, NULL, 0, NULL, NULL) == TRINV_ERR_ARG);
  CHECK(trinv_tril_inverse(TRINV_F64, 0, NULL, 0, NULL, 0, NULL, NULL, 0, NULL, &info) == TRINV_OK);

  trinv_opts r;
  trinv_default_opts(&r);
  r.resid = 7;
  CHECK(trinv_tril_inverse(TRINV_BF16_REFINE, 64, P(1ull << 30), 64, P(1ull << 34), 64, &r, NULL, 0, NULL, NULL) ==
        TRINV_ERR_ARG);
  trinv_default_opts(&r);
  r.beta = 1;
  CHECK(trinv_tril_inverse(TRINV_F64, 1000, P(1ull << 30), 1000, P(1ull << 34), 1000, &r, NULL, 0, NULL, NULL) ==
        TRINV_ERR_ARG);

  CHECK(trinv_tril_inverse_backward(TRINV_F64, 1, 4, NULL, NULL, NULL, 16, NULL, 0, NULL) == TRINV_ERR_ARG);
  CHECK(trinv_factored_inverse(TRINV_F64, 4, NULL, 4, 0, NULL, 4, 1, NULL, 4, NULL, 4, NULL, 4, NULL, NULL, 0, NULL,
                               NULL) == TRINV_ERR_ARG);
  CHECK(trinv_factored_inverse(TRINV_F64, 4, P(1 << 20), 3, 0, P(2 << 20), 4, 1, P(3 << 20), 4, P(4 << 20), 4, NULL,
                               0, NULL, NULL, 0, NULL, NULL) == TRINV_ERR_ARG);
  CHECK(trinv_residual(TRINV_F64, -2, NULL, 0, NULL, 0, NULL, 0, NULL, NULL) == TRINV_ERR_ARG);
  double out5[5];
  CHECK(trinv_refine_residual(TRINV_BF16_REFINE, -1, P(1ull << 30), 64, P(1ull << 34), 64, 3, P(1ull << 36), 64, NULL,
                              0, NULL, out5) == TRINV_ERR_ARG);
  CHECK(trinv_refine_residual(TRINV_F64, 64, P(1ull << 30), 64, P(1ull << 34), 64, 3, P(1ull << 36), 64, NULL, 0,
                              NULL, out5) == TRINV_ERR_UNSUPPORTED);

  int32_t n3[3] = {5, 64, 100};
  int64_t off3[3] = {0, 25, 25 + 64 * 64};
  int32_t st3[3];
  CHECK(trinv_tril_inverse_batched(TRINV_F32, -1, n3, P(1 << 20), off3, P(2 << 20), P(1ull << 30), P(1ull << 31),
                                   P(1ull << 32), &o, NULL, 0, NULL) == TRINV_ERR_ARG);
  int32_t bad3[3] = {5, -64, 100};
  CHECK(trinv_tril_inverse_batched(TRINV_F32, 3, bad3, P(1 << 20), off3, P(2 << 20), P(1ull << 30), P(1ull << 31),
                                   P(1ull << 32), &o, NULL, 0, NULL) == TRINV_ERR_ARG);
  CHECK(trinv_batched_workspace_bytes(TRINV_F32, 3, n3, &o) >= 3 * 4 + 4);
  trinv_batched_config cfg = {16, 1, -1.0f, 0};
  CHECK(trinv_batched_set_config(TRINV_F32, 3, n3, &cfg) == TRINV_ERR_ARG);
  (void)st3;

  trinv_profile_entry pe[4];
  CHECK(trinv_profile_read(pe, 4) >= 0);
}

int main(void) {
  oracle_cases();
  abi_cases();
  if (failures) fprintf(stderr, "%d check(s) failed\n", failures);
  else printf("sanitize driver: all checks passed\n");
  return failures;
}
