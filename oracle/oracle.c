/*
 * CPU FP64 oracle for the triangular-inverse engine.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * Everything here is plain FP64 C with the loops in the order the definitions
 * state them; there is no blocking, fusion or reordering. OpenMP only runs
 * independent columns (or rows) on different threads; it does not change the
 * arithmetic of any single entry.
 *
 * Conventions (the paper states its results for unit upper-triangular T,
 * eq. defT, and says the lower case follows by transposition and the
 * non-unit case through a diagonal factor R = D T, Section 4):
 *   - matrices are row-major with a leading dimension; element (i, j) of a
 *     matrix A with leading dimension lda is A[i * lda + j];
 *   - "lower" inputs: only the lower triangle (j <= i) is read, the strict
 *     upper part is ignored whatever it holds;
 *   - unit != 0 means the diagonal is taken as 1 and never read.
 *
 * Functions whose parity is pinned, and by what, are listed in the Python
 * wrapper (oracle/__init__.py) and in the test file of the oracle pins.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_API __attribute__((visibility("default")))

/* Element (i, j) of a matrix seen through strides; lets the upper factor of
 * the factored inverse be read as the lower matrix U^T without a copy. */
static inline double at(const double *A, int64_t rs, int64_t cs, int64_t i, int64_t j) {
  return A[i * rs + j * cs];
}

/* First zero diagonal entry, 1-based (LAPACK convention), 0 if none. */
static int64_t first_zero_diag(int64_t n, const double *A, int64_t rs, int64_t cs, int unit) {
  if (unit) return 0;
  for (int64_t i = 0; i < n; ++i)
    if (at(A, rs, cs, i, i) == 0.0) return i + 1;
  return 0;
}

/*
 * Column j of X = L^{-1} by the column recurrence CRIT (Section 4.2, algorithm
 * CRIT), transposed to the lower case: the paper grows row i of S = R^{-1} for
 * upper R with
 *     S(i,i) = 1 / R(i,i),   S(i,j) = -S(i, i:j-1) . R(i:j-1, j) / R(j,j);
 * for lower L this reads, for column j of X,
 *     X(j,j) = 1 / L(j,j),   X(i,j) = -(sum_{k=j}^{i-1} L(i,k) X(k,j)) / L(i,i)
 * for i = j+1 .. n-1, summed in ascending k. Entries above the diagonal are 0.
 * The loop starts at i = j+1 (the paper's unit variant CRIT* starts one later
 * because X(j+1,j) = -L(j+1,j) there is a plain sign flip).
 */
static void crit_column(int64_t n, const double *L, int64_t rs, int64_t cs, int unit, int64_t j,
                        double *x) {
  for (int64_t i = 0; i < j; ++i) x[i] = 0.0;
  x[j] = unit ? 1.0 : 1.0 / at(L, rs, cs, j, j);
  for (int64_t i = j + 1; i < n; ++i) {
    double s = 0.0;
    for (int64_t k = j; k < i; ++k) s += at(L, rs, cs, i, k) * x[k];
    x[i] = unit ? -s : -s / at(L, rs, cs, i, i);
  }
}

/* X = L^{-1} for lower L viewed through strides (rs, cs); X row-major, ldx.
 * Returns 0, or the 1-based index of the first zero diagonal (X untouched). */
static int64_t tril_inverse_strided(int64_t n, const double *L, int64_t rs, int64_t cs, int unit,
                                    double *X, int64_t ldx) {
  int64_t bad = first_zero_diag(n, L, rs, cs, unit);
  if (bad) return bad;
#pragma omp parallel
  {
    double *x = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; ++j) {
      crit_column(n, L, rs, cs, unit, j, x);
      for (int64_t i = 0; i < n; ++i) X[i * ldx + j] = x[i];
    }
    free(x);
  }
  return 0;
}

ORACLE_API int64_t oracle_tril_inverse(int64_t n, const double *L, int64_t ldl, int32_t unit,
                                       double *X, int64_t ldx) {
  return tril_inverse_strided(n, L, ldl, 1, unit, X, ldx);
}

/* Selected columns of X = L^{-1}: out is column-major n x ncols (out[c*n + i]
 * = X(i, cols[c])). Same recurrence as above, one column at a time. */
ORACLE_API int64_t oracle_tril_inverse_columns(int64_t n, const double *L, int64_t ldl, int32_t unit,
                                               const int64_t *cols, int64_t ncols, double *out) {
  int64_t bad = first_zero_diag(n, L, ldl, 1, unit);
  if (bad) return bad;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < ncols; ++c) crit_column(n, L, ldl, 1, unit, cols[c], out + c * n);
  return 0;
}

/*
 * Chain-sum (combinatorial) inverse, Theorem Combinatorix (Section 3): for
 * unit upper T, S(i,j) is the sum over every increasing index chain
 * i = a_1 < a_2 < ... < a_l = j (the Hopscotch series H(i,j), Definition in
 * Section 3; 2^(j-i-1) chains, Proposition corrTranlation) of
 * (-1)^(l-1) * prod_t T(a_t, a_{t+1}).
 * Lower case (transpose): X(i,j), i > j, sums over chains j = c_1 < ... < c_l = i
 * of (-1)^(l-1) prod_t L(c_{t+1}, c_t). Non-unit case through L = D T with
 * D = diag(L) (Section 4): every factor is divided by the diagonal of its row
 * and the whole chain term by L(j,j), i.e. by the product of L(v,v) over all
 * chain members v. Brute force, O(2^n): only meant for n <= 20.
 * Returns -1 if n is too large, else as oracle_tril_inverse.
 */
ORACLE_API int64_t oracle_chain_sum_inverse(int64_t n, const double *L, int64_t ldl, int32_t unit,
                                            double *X, int64_t ldx) {
  if (n > 24) return -1;
  int64_t bad = first_zero_diag(n, L, ldl, 1, unit);
  if (bad) return bad;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) X[i * ldx + j] = 0.0;
  for (int64_t j = 0; j < n; ++j) X[j * ldx + j] = unit ? 1.0 : 1.0 / L[j * ldl + j];
  for (int64_t i = 1; i < n; ++i) {
    for (int64_t j = 0; j < i; ++j) {
      int64_t m = i - j - 1; /* interior indices j+1 .. i-1 */
      double total = 0.0;
      for (uint64_t mask = 0; mask < ((uint64_t)1 << m); ++mask) {
        double prod = 1.0;
        int64_t prev = j, len = 1;
        double dprod = unit ? 1.0 : L[j * ldl + j];
        for (int64_t b = 0; b < m; ++b) {
          if (mask & ((uint64_t)1 << b)) {
            int64_t v = j + 1 + b;
            prod *= L[v * ldl + prev];
            if (!unit) dprod *= L[v * ldl + v];
            prev = v;
            ++len;
          }
        }
        prod *= L[i * ldl + prev];
        if (!unit) dprod *= L[i * ldl + i];
        ++len;
        double sign = ((len - 1) % 2 == 0) ? 1.0 : -1.0;
        total += sign * prod / dprod;
      }
      X[i * ldx + j] = total;
    }
  }
  return 0;
}

/* Number of chains in H(a, b) counted by enumeration (for the pin of
 * Proposition corrTranlation, 2^(b-a-1) for a < b). */
ORACLE_API int64_t oracle_chain_count(int64_t a, int64_t b) {
  if (b <= a) return 0;
  int64_t m = b - a - 1, count = 0;
  for (uint64_t mask = 0; mask < ((uint64_t)1 << m); ++mask) ++count;
  return count;
}

/*
 * Crout decomposition without pivoting, the factorization part of algorithm
 * SKUL (Section 5): A = L U with L lower triangular (general diagonal) and U
 * unit upper triangular, formed row by row as the algorithm does: row i of L
 * (columns 1..i), then row i of U (columns i+1..n):
 *   L(i, j) = A(i, j) - sum_{k<j} L(i, k) U(k, j)               (j <= i)
 *   U(i, j) = (A(i, j) - sum_{k<i} L(i, k) U(k, j)) / L(i, i)    (j > i)
 * L and U are n x n row-major with leading dimension n, zero outside their
 * triangles. Returns 0, or the 1-based index of the first zero L(i, i).
 */
ORACLE_API int64_t oracle_crout_lu(int64_t n, const double *A, int64_t lda, double *L, double *U) {
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      L[i * n + j] = 0.0;
      U[i * n + j] = (i == j) ? 1.0 : 0.0;
    }
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j <= i; ++j) {
      double s = A[i * lda + j];
      for (int64_t k = 0; k < j; ++k) s -= L[i * n + k] * U[k * n + j];
      L[i * n + j] = s;
    }
    if (L[i * n + i] == 0.0) return i + 1;
    for (int64_t j = i + 1; j < n; ++j) {
      double s = A[i * lda + j];
      for (int64_t k = 0; k < i; ++k) s -= L[i * n + k] * U[k * n + j];
      U[i * n + j] = s / L[i * n + i];
    }
  }
  return 0;
}

/*
 * Factored inverse (Section 5, SKUL: from L U = A, S K = A^{-1} with
 * S = U^{-1}, K = L^{-1}). Linv = L^{-1}; Uinv = U^{-1} obtained as the
 * transpose of (U^T)^{-1}, U^T being lower; Ainv = Uinv * Linv by the plain
 * triple loop (skipped if Ainv is NULL). Only the lower triangle of L and the
 * upper triangle of U are read. Returns 0, the 1-based index of a zero
 * diagonal of L, or minus the 1-based index of a zero diagonal of U.
 */
ORACLE_API int64_t oracle_factored_inverse(int64_t n, const double *L, int64_t ldl, int32_t l_unit,
                                           const double *U, int64_t ldu, int32_t u_unit,
                                           double *Linv, double *Uinv, double *Ainv) {
  int64_t bad = tril_inverse_strided(n, L, ldl, 1, l_unit, Linv, n);
  if (bad) return bad;
  double *Ut_inv = (double *)malloc(sizeof(double) * (size_t)(n * n > 0 ? n * n : 1));
  /* U^T viewed as lower: element (i, j) of U^T is U[j * ldu + i]. */
  bad = tril_inverse_strided(n, U, 1, ldu, u_unit, Ut_inv, n);
  if (bad) {
    free(Ut_inv);
    return -bad;
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) Uinv[i * n + j] = Ut_inv[j * n + i];
  free(Ut_inv);
  if (Ainv) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int64_t k = 0; k < n; ++k) s += Uinv[i * n + k] * Linv[k * n + j];
        Ainv[i * n + j] = s;
      }
  }
  return 0;
}

/*
 * Gradient of f(L) = sum(G .* L^{-1}) with respect to the lower entries of L:
 * with X = L^{-1}, dX = -X dL X, so df/dL = -X^T G X^T, restricted to the
 * lower triangle: grad = -tril(X^T G X^T). X is computed here by the column
 * recurrence from L (no value from any other implementation); the two
 * products are plain full triple loops, G is used in full.
 * grad is row-major n x n with leading dimension n; its strict upper is 0.
 */
ORACLE_API int64_t oracle_tril_inverse_backward(int64_t n, const double *L, int64_t ldl, const double *G,
                                                int64_t ldg, double *grad) {
  size_t nn = (size_t)(n * n > 0 ? n * n : 1);
  double *X = (double *)malloc(sizeof(double) * nn);
  double *M = (double *)malloc(sizeof(double) * nn);
  int64_t bad = tril_inverse_strided(n, L, ldl, 1, 0, X, n);
  if (bad) {
    free(X);
    free(M);
    return bad;
  }
  /* M = X^T G */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = 0; k < n; ++k) {
      double s = 0.0;
      for (int64_t l = 0; l < n; ++l) s += X[l * n + i] * G[l * ldg + k];
      M[i * n + k] = s;
    }
  /* grad = -tril(M X^T) */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0;
      if (j <= i)
        for (int64_t k = 0; k < n; ++k) s += M[i * n + k] * X[j * n + k];
      grad[i * n + j] = (j <= i) ? -s : 0.0;
    }
  free(X);
  free(M);
  return 0;
}

/* Selected rows of the same gradient: out is nrows x n row-major. X is
 * computed in full from L, then row i of M = X^T G and row i of grad. */
ORACLE_API int64_t oracle_tril_inverse_backward_rows(int64_t n, const double *L, int64_t ldl,
                                                     const double *G, int64_t ldg, const int64_t *rows,
                                                     int64_t nrows, double *out) {
  size_t nn = (size_t)(n * n > 0 ? n * n : 1);
  double *X = (double *)malloc(sizeof(double) * nn);
  int64_t bad = tril_inverse_strided(n, L, ldl, 1, 0, X, n);
  if (bad) {
    free(X);
    return bad;
  }
#pragma omp parallel
  {
    double *m = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
      int64_t i = rows[r];
      for (int64_t k = 0; k < n; ++k) {
        double s = 0.0;
        for (int64_t l = 0; l < n; ++l) s += X[l * n + i] * G[l * ldg + k];
        m[k] = s;
      }
      for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        if (j <= i)
          for (int64_t k = 0; k < n; ++k) s += m[k] * X[j * n + k];
        out[r * n + j] = (j <= i) ? -s : 0.0;
      }
    }
    free(m);
  }
  free(X);
  return 0;
}

/*
 * Residual metrics of a candidate inverse X of lower L (L read as tril(L),
 * X read in full, so a non-zero strict upper in X shows up):
 *   out[0] = ||L X - I||_F, out[1] = ||X L - I||_F,
 *   out[2] = ||tril(L)||_F, out[3] = ||X||_F.
 * The relative residual is out[0] / (out[2] * out[3]).
 */
ORACLE_API void oracle_residuals(int64_t n, const double *L, int64_t ldl, const double *X, int64_t ldx,
                                 double *out) {
  double r_lx = 0.0, r_xl = 0.0, nl = 0.0, nx = 0.0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : r_lx, r_xl, nl, nx)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0; /* (L X)(i,j) = sum_{k <= i} L(i,k) X(k,j) */
      for (int64_t k = 0; k <= i; ++k) s += L[i * ldl + k] * X[k * ldx + j];
      double e = s - (i == j ? 1.0 : 0.0);
      r_lx += e * e;
      double t = 0.0; /* (X L)(i,j) = sum_{k >= j} X(i,k) L(k,j) */
      for (int64_t k = j; k < n; ++k) t += X[i * ldx + k] * L[k * ldl + j];
      double f = t - (i == j ? 1.0 : 0.0);
      r_xl += f * f;
      nx += X[i * ldx + j] * X[i * ldx + j];
      if (j <= i) nl += L[i * ldl + j] * L[i * ldl + j];
    }
  }
  out[0] = sqrt(r_lx);
  out[1] = sqrt(r_xl);
  out[2] = sqrt(nl);
  out[3] = sqrt(nx);
}

/* The residual matrix itself: out(i, j) = [i == j] - sum_{k <= i} L(i, k) X(k, j)
 * (tril(L) read, X read in full; out n x n, leading dimension n), ascending k. */
ORACLE_API void oracle_residual_matrix(int64_t n, const double *L, int64_t ldl, const double *X, int64_t ldx,
                                       double *out) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; ++i) {
    /* row i of L X: every entry sums L(i, k) X(k, j) over k = 0 .. i in
     * ascending k, one row of X at a time */
    double *o = out + i * n;
    for (int64_t j = 0; j < n; ++j) o[j] = 0.0;
    for (int64_t k = 0; k <= i; ++k) {
      const double l = L[i * ldl + k];
      const double *x = X + k * ldx;
      for (int64_t j = 0; j < n; ++j) o[j] += l * x[j];
    }
    for (int64_t j = 0; j < n; ++j) o[j] = (i == j ? 1.0 : 0.0) - o[j];
  }
}

/* Squared column norms of L X - I for selected columns (for matrices too
 * large for the full residual): out[c] = ||(L X - I)(:, cols[c])||_2^2. */
ORACLE_API void oracle_residual_columns(int64_t n, const double *L, int64_t ldl, const double *X,
                                        int64_t ldx, const int64_t *cols, int64_t ncols, double *out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < ncols; ++c) {
    int64_t j = cols[c];
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int64_t k = 0; k <= i; ++k) s += L[i * ldl + k] * X[k * ldx + j];
      double e = s - (i == j ? 1.0 : 0.0);
      acc += e * e;
    }
    out[c] = acc;
  }
}

/*
 * Algorithm SQR (Section 5): modified Gram-Schmidt QR of A (A = Q R, Q with
 * orthonormal columns, R upper triangular with positive diagonal) with
 * S = R^{-1} grown one column at a time beside R. For column j (0-based):
 *   q^ = v_j;  for i < j: R(i, j) = q^ . q_i,  q^ -= R(i, j) q_i   (in order);
 *   R(j, j) = ||q^||_2  (zero -> stop);  D(j, j) = 1 / R(j, j);  q_j = D(j, j) q^;
 *   S'(j, j) = 1;  S'(i, j) = -(1 / R(j, j)) sum_{k=i}^{j-1} S'(i, k) R(k, j)  (i < j);
 * and at the end S = D S' (row i of S' times D(i, i)). The column of S' uses
 * R(j, j) of the same column, so it is formed once R(j, j) is known (S' is
 * then the inverse of R D, whose diagonal is 1, and D S' = (R D D^{-1})^{-1}).
 * Q, R, S are n x n row-major with leading dimension n; R and S are zero
 * below the diagonal. Returns 0, or the 1-based index j + 1 of the first
 * column with R(j, j) = 0 (the outputs are then incomplete).
 */
ORACLE_API int64_t oracle_sqr(int64_t n, const double *A, int64_t lda, double *Q, double *R, double *S) {
  double *qh = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n * n; ++i) {
    Q[i] = 0.0;
    R[i] = 0.0;
    S[i] = 0.0;
  }
  int64_t bad = 0;
  for (int64_t j = 0; j < n && !bad; ++j) {
    for (int64_t r = 0; r < n; ++r) qh[r] = A[r * lda + j];
    for (int64_t i = 0; i < j; ++i) {
      double dot = 0.0;
      for (int64_t r = 0; r < n; ++r) dot += qh[r] * Q[r * n + i];
      R[i * n + j] = dot;
      for (int64_t r = 0; r < n; ++r) qh[r] -= dot * Q[r * n + i];
    }
    double nrm = 0.0;
    for (int64_t r = 0; r < n; ++r) nrm += qh[r] * qh[r];
    nrm = sqrt(nrm);
    R[j * n + j] = nrm;
    if (nrm == 0.0) {
      bad = j + 1;
      break;
    }
    d[j] = 1.0 / nrm;
    for (int64_t r = 0; r < n; ++r) Q[r * n + j] = d[j] * qh[r];
    S[j * n + j] = 1.0;
    for (int64_t i = 0; i < j; ++i) {
      double s = 0.0;
      for (int64_t k = i; k < j; ++k) s += S[i * n + k] * R[k * n + j];
      S[i * n + j] = -s / nrm;
    }
  }
  if (!bad)
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = i; j < n; ++j) S[i * n + j] *= d[i];
  free(qh);
  free(d);
  return bad;
}

/*
 * A^{-1} by its textbook construction: Gauss-Jordan elimination with partial
 * pivoting on [A | I]. For column c: pick the row p >= c with the largest
 * |a(p, c)|, swap rows p and c of both halves, divide row c by the pivot,
 * then subtract a(r, c) times row c from every other row r. The right half is
 * then A^{-1}. X is n x n row-major with leading dimension n. Returns 0, or
 * c + 1 for the first column without a nonzero pivot (X is then incomplete).
 */
ORACLE_API int64_t oracle_inverse(int64_t n, const double *A, int64_t lda, double *X) {
  size_t nn = (size_t)(n * n > 0 ? n * n : 1);
  double *W = (double *)malloc(sizeof(double) * nn);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      W[i * n + j] = A[i * lda + j];
      X[i * n + j] = (i == j) ? 1.0 : 0.0;
    }
  int64_t bad = 0;
  for (int64_t c = 0; c < n; ++c) {
    int64_t p = c;
    for (int64_t r = c + 1; r < n; ++r)
      if (fabs(W[r * n + c]) > fabs(W[p * n + c])) p = r;
    if (W[p * n + c] == 0.0) {
      bad = c + 1;
      break;
    }
    if (p != c)
      for (int64_t j = 0; j < n; ++j) {
        double t = W[p * n + j];
        W[p * n + j] = W[c * n + j];
        W[c * n + j] = t;
        t = X[p * n + j];
        X[p * n + j] = X[c * n + j];
        X[c * n + j] = t;
      }
    const double piv = W[c * n + c];
    for (int64_t j = 0; j < n; ++j) {
      W[c * n + j] /= piv;
      X[c * n + j] /= piv;
    }
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = W[r * n + c];
      if (f == 0.0) continue;
      for (int64_t j = 0; j < n; ++j) {
        W[r * n + j] -= f * W[c * n + j];
        X[r * n + j] -= f * X[c * n + j];
      }
    }
  }
  free(W);
  return bad;
}

/* Threads OpenMP will use (for the CPU-baseline report). */
ORACLE_API int32_t oracle_num_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}
