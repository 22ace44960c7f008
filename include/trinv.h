/*
 * trinv.h -- C ABI of the MI355X (gfx950) triangular-inverse library.
 *
 * The operation (Riahi, "Combinatorial and Recurrent Approaches for Efficient
 * Matrix Inversion", 2023): invert a non-singular triangular matrix
 * (Section 2, eq. defT; the paper states the unit upper case and obtains the
 * lower case by transposition and the non-unit case through a diagonal
 * factor R = D T, Section 4) by recursive 2x2 block splitting (Section 4.1,
 * algorithm COMBRIT with beta = 2):
 *
 *     [ A  0 ]^-1   [  A^-1           0    ]
 *     [ C  B ]    = [ -B^-1 C A^-1    B^-1 ]
 *
 * with the diagonal blocks inverted recursively and the smallest ("leaf")
 * blocks inverted by the column recurrence CRIT (Section 4.2; any leaf method
 * is allowed, Remark rmkCOMBRIT). The off-diagonal block is formed as
 * T = C * A^-1 followed by X21 = -B^-1 * T, i.e. the product with the inverted
 * diagonal block first (COMBRIT's B_ij = iD_ii A_ij, then iA_ij = iB_ij iD_jj,
 * transposed to the lower case).
 *
 * Conventions shared by every call:
 *   - All matrix pointers are DEVICE pointers owned by the caller; the
 *     library never allocates, frees or keeps them. Matrices are row-major;
 *     element (i, j) of A with leading dimension lda is A[i * lda + j].
 *   - Only the lower triangle (j <= i) of an input L is read; the strict
 *     upper part is ignored whatever it holds. With opts->unit_diag the
 *     diagonal is taken as 1 and not read.
 *   - The output X = L^-1 is written in full: lower triangle = the inverse,
 *     strict upper part = +0.0.
 *   - X must not overlap L (or any other input).
 *   - Every call is ordered on the given stream (a hipStream_t; NULL means
 *     the legacy default stream) and returns without waiting for the GPU
 *     unless opts->blocking is set, or the mode needs a host decision (the
 *     refinement loop reads one 8-byte norm per iteration).
 *   - The workspace is caller-owned device memory of at least
 *     trinv_workspace_bytes(...) bytes, 256-byte aligned.
 *   - n == 0 (or batch == 0) is a no-op returning TRINV_OK.
 *
 * Errors: a negative size, ld < n, a NULL required pointer, overlapping input
 * and output, or an unsupported mode returns TRINV_ERR_ARG /
 * TRINV_ERR_UNSUPPORTED before anything is launched. A too-small workspace
 * returns TRINV_ERR_WORKSPACE. A HIP launch or runtime error returns
 * TRINV_ERR_HIP. An exactly zero diagonal entry (the paper stops only on an
 * exact zero pivot, algorithms SQR/SKUL) is reported as TRINV_ERR_SINGULAR
 * with info->first_bad_index = its 1-based index when the call waits for the
 * GPU (opts->blocking or the refine modes); X is unspecified then.
 */
#ifndef TRINV_H
#define TRINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A hipStream_t passed as an opaque pointer. */
typedef void *trinv_stream_t;

typedef enum {
  /* FP64 storage, FP64 leaves, FP64 MFMA products. */
  TRINV_F64 = 0,
  /* FP32 storage, FP32 leaves, FP32 MFMA products. */
  TRINV_F32 = 1,
  /* FP64 storage and FP64 leaves; off-diagonal products on BF16 MFMA with
   * FP32 accumulation; then Newton-Schulz refinement X <- X + X (I - L X)
   * (which keeps X lower triangular) until the relative residual
   * ||L X - I||_F / (||L||_F ||X||_F) <= opts->tol. The residual is
   * assembled, stored and reduced in FP64; its O(n^3) strictly-lower product
   * runs on split BF16 slices or on FP64 MFMA (opts->resid), and
   * info->resid_error_est estimates the error this leaves in the reported
   * residual. The first iterate keeps the FP64 diagonal 1 / L_ii
   * and holds BF16 values below it (the values its products read); with
   * max_iter = 0 that iterate is what X holds on return. */
  TRINV_BF16_REFINE = 2,
  /* As TRINV_BF16_REFINE with FP16 slices (power-of-two scaled rows and
   * columns to keep them in FP16 range); the first iterate holds FP16 values
   * times one power-of-two scale below its diagonal. */
  TRINV_F16_REFINE = 3
} trinv_mode;

typedef enum {
  TRINV_OK = 0,
  TRINV_ERR_ARG = 1,
  TRINV_ERR_SINGULAR = 2,
  TRINV_ERR_NONFINITE = 3,
  TRINV_ERR_NOT_CONVERGED = 4,
  TRINV_ERR_HIP = 5,
  TRINV_ERR_UNSUPPORTED = 6,
  TRINV_ERR_WORKSPACE = 7
} trinv_status;

typedef struct {
  int32_t leaf;      /* leaf block order; 0 = the mode's default (tuned) */
  int32_t unit_diag; /* 1: the diagonal is taken as 1 and not read */
  int32_t upper;     /* 1: the input is UPPER triangular; the upper inverse is
                        returned (computed through the transposed view) */
  int32_t max_iter;  /* refine modes: most Newton-Schulz corrections (default 4) */
  double tol;        /* refine modes: target relative residual (default 1e-12) */
  int32_t blocking;  /* 1: wait for the GPU and fill *info (status, residual) */
  int32_t check;     /* 1 (with blocking): also compute the FP64 relative
                        residual of the result into info->rel_residual */
  int32_t beta;      /* block grid of the top level, algorithm COMBRIT
                        (Section 4.1): 0 or 2 = the binary recursion; 3..16 =
                        beta x beta blocks of order n / beta at the top (F64 /
                        F32, lower, n divisible by beta, ldl == ldx, else
                        TRINV_ERR_ARG / TRINV_ERR_UNSUPPORTED), the diagonal
                        blocks by the binary recursion */
  int32_t resid;     /* refine modes: precision of the residual's O(n^3)
                        product, one of trinv_resid_prec (default AUTO) */
} trinv_opts;

/* Precision of the refinement residual's strictly-lower product N_L N_X
 * (the O(n^2) diagonal terms are always exact FP64). */
typedef enum {
  /* SPLIT when its estimated error (info->resid_error_est) is at most
   * tol / 2, else FP64; decided once, from the first iterate's norms. */
  TRINV_RESID_AUTO = 0,
  /* Low-precision slices hi + lo of both factors, three MFMA products
   * (two for the first iterate, whose strictly lower part one slice holds
   * exactly), FP32 accumulation. */
  TRINV_RESID_SPLIT = 1,
  /* FP64 MFMA. */
  TRINV_RESID_FP64 = 2
} trinv_resid_prec;

typedef struct {
  double rel_residual;     /* ||L X - I||_F / (||L||_F ||X||_F), or -1 if not computed */
  /* Refine modes: the estimated error of rel_residual, from a random-walk
   * model of the split product's rounding errors (errors of the ~n terms of
   * an entry add like independent random signs):
   *   (0.5 u^2 + 2^-24 sqrt(n) / 8) ||N_L||_F ||N_X||_F / (sqrt(n) ||L||_F ||X||_F),
   * u = 2^-8 (BF16) or 2^-11 (FP16): the slices' rounding, then the FP32
   * accumulation and FP16 subnormals; the constants are about twice the
   * ones measured on the seeded test matrices. It is an estimate, not a
   * bound: the stopping rule is rel_residual + resid_error_est <= tol. For
   * the FP64 product: 2^-53 ||N_L||_F ||N_X||_F / (||L||_F ||X||_F). */
  double resid_error_est;
  /* Refine modes: a worst-case bound on the same error (every rounding at
   * its largest, in the same direction): slices (3u^2 + 3u^3), FP32
   * accumulation gamma_m = m 2^-23 / (1 - m 2^-23) over the m = nsplit n
   * products of an entry, FP64 assembly, FP16 underflow. It holds without
   * assumptions and is usually orders of magnitude above the actual error,
   * too loose to certify a residual of 1e-12 at these orders. */
  double resid_error_bound;
  int32_t iterations;      /* refine modes: corrections applied */
  int64_t first_bad_index; /* 1-based index of the first zero diagonal, 0 = none */
} trinv_info;

/* Fills *opts with the defaults (leaf 0, unit_diag 0, upper 0, max_iter 4,
 * tol 1e-12, blocking 0, check 0, beta 0, resid AUTO). Passing opts == NULL
 * to any call means these defaults. */
void trinv_default_opts(trinv_opts *opts);

/* Human-readable name of a status code (static storage). */
const char *trinv_status_string(int status);

/* Bytes of workspace trinv_tril_inverse needs for (mode, n, opts); 0 for
 * n <= 0 and for refine-mode orders above 2^23 - 128 (unsupported: the
 * low-precision products keep 32-bit byte offsets within 256 rows of a
 * plane). */
size_t trinv_workspace_bytes(int mode, int64_t n, const trinv_opts *opts);

/*
 * X = L^-1 for one n x n triangular matrix (lower by default; with
 * opts->upper an upper input, whose upper inverse is returned, zeros below
 * the diagonal: every mode computes it as the transpose of the lower inverse
 * of U^T, Section 2).
 * mode: a trinv_mode. L: device, FP64 for F64/BF16_REFINE/F16_REFINE, FP32
 * for F32; ldl >= n. X: device, same element type, ldx >= n, written in
 * full. ws/ws_bytes: workspace (see trinv_workspace_bytes). info: nullable.
 * Status: with opts->blocking (F64 / F32) or always (refine modes),
 * TRINV_ERR_SINGULAR for an exact zero diagonal entry and
 * TRINV_ERR_NONFINITE when X holds a NaN or an infinity (a non-finite
 * input, or overflow); the refine modes also return
 * TRINV_ERR_NOT_CONVERGED after opts->max_iter corrections (X then holds
 * the last iterate, info its residual). Refine modes stop when
 * info->rel_residual + info->resid_error_est <= opts->tol.
 */
int trinv_tril_inverse(int mode, int64_t n, const void *L, int64_t ldl, void *X, int64_t ldx,
                       const trinv_opts *opts, void *ws, size_t ws_bytes, trinv_stream_t stream,
                       trinv_info *info);

/* Bytes of workspace trinv_tril_inverse_batched needs for this batch: 4 bytes
 * per matrix plus a queue counter (n_host and opts are not needed for the
 * size and may be NULL). */
size_t trinv_batched_workspace_bytes(int mode, int64_t batch, const int32_t *n_host,
                                     const trinv_opts *opts);

/*
 * X_i = L_i^-1 for `batch` independent lower-triangular matrices, uniform or
 * of uneven order, packed back to back. Independent diagonal blocks can be
 * inverted concurrently (Section 4.1, algorithm COMBRIT and its complexity
 * remark); each matrix runs the same recursion as trinv_tril_inverse (leaves
 * of 32 or 64 by the column recurrence of Section 4.2, then the 2 x 2 block
 * levels).
 * mode: TRINV_F32 or TRINV_F64.
 *   n_host / n_dev: the orders n_i (host copy for validation, device copy read
 *     by the kernels; identical contents), 1 <= n_i <= 1024, batch < 2^31.
 *   off_host / off_dev: int64 element offsets of matrix i in L_packed and
 *     X_packed; matrix i is dense n_i x n_i row-major with leading dimension
 *     n_i (only its lower triangle is read; all of X_i is written, zeros
 *     above the diagonal). Gaps between matrices are not touched. The L and X
 *     ranges must not overlap (TRINV_ERR_ARG).
 *   status_dev: device int32[batch]; status_dev[i] = 0, or the 1-based index
 *     of the first zero diagonal of matrix i (X_i then holds non-finite
 *     values), or -1 if n_dev[i] is outside [1, 1024], or -2 if X_i holds a
 *     NaN or an infinity (a non-finite input entry, or overflow).
 *   opts: leaf 0 (tuned or default), 32 or 64 (else TRINV_ERR_ARG); unit_diag honoured;
 *     upper: the matrices are UPPER triangular (only their upper triangles
 *     are read) and X_i = U_i^-1 is upper (zeros below the diagonal),
 *     through the transpose, (U^T)^-1 = (U^-1)^T (Section 2); blocking: wait
 *     and return TRINV_ERR_SINGULAR if any matrix is singular, else
 *     TRINV_ERR_NONFINITE if any status is -2.
 *   ws: at least trinv_batched_workspace_bytes bytes (which depends on
 *     opts->upper), caller-owned.
 * Two launches on `stream`: a one-workgroup plan kernel (sorts the matrices
 * by order, largest first, and resets the queue counter in ws) and one
 * persistent kernel whose workgroups take whole matrices from that queue.
 * With upper, three more: the dense offsets, the transposes U_i^T into ws
 * (packed back to back), and X_i as the transposes of their lower inverses
 * (also held in ws).
 * No memset and no host synchronisation (unless blocking), so the call can be
 * captured in a graph and replayed.
 */
int trinv_tril_inverse_batched(int mode, int64_t batch, const int32_t *n_host, const int32_t *n_dev,
                               const int64_t *off_host, const int64_t *off_dev, const void *L_packed,
                               void *X_packed, int32_t *status_dev, const trinv_opts *opts, void *ws,
                               size_t ws_bytes, trinv_stream_t stream);

/*
 * For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same inversion
 * as trinv_tril_inverse_batched, always by the persistent launch, with its
 * plan and queue counter in a per-device scratch array of the library
 * (65536 matrix indices plus the counter, about 256 KB, held by each device
 * the library runs on until the process ends) instead of a workspace. No
 * device memory is allocated or freed, by the library or anything it calls.
 * Arguments, status values and errors as trinv_tril_inverse_batched, without
 * ws / ws_bytes; batch > 65536 gives TRINV_ERR_ARG, and opts->upper
 * TRINV_ERR_UNSUPPORTED (its transposed staging needs a workspace). Every call on one device
 * shares that device's scratch (the plan kernel rewrites the plan and resets
 * the counter at the start of each call), so calls that overlap on one
 * device -- on different streams, or from different threads -- race and
 * must be serialised by the caller.
 */
int trinv_tril_inverse_batched_noalloc(int mode, int64_t batch, const int32_t *n_host, const int32_t *n_dev,
                                       const int64_t *off_host, const int64_t *off_dev, const void *L_packed,
                                       void *X_packed, int32_t *status_dev, const trinv_opts *opts,
                                       trinv_stream_t stream);

/* A configuration of the persistent batched launch. */
typedef struct {
  int32_t leaf;         /* leaf order, the recursion's cut-off: 32 or 64 (the
                           diagonal blocks inverted by the column recurrence
                           before the 2 x 2 levels) */
  int32_t wgs_per_cu;   /* resident workgroups per CU (0 = the occupancy limit;
                           0 in autotune output of the level path) */
  float ms;             /* time of one launch pair with it; -1 if not timed */
  int32_t tile;         /* largest tile of the level products, 64 or 128
                           (0 = 128): each level uses min(h, tile) squares */
} trinv_batched_config;

/*
 * Autotuner of trinv_tril_inverse_batched (not in the paper): times the
 * persistent launch with every candidate configuration (leaf in {32, 64},
 * or opts->leaf if set; tile in {64, 128}; wgs_per_cu from 1 up to the
 * occupancy limit in powers of two, and that limit) on the caller's buffers and stream, one untimed
 * launch and the fastest of three each, and keeps the fastest for this
 * batch's order signature (mode, count, sum of n_i, sum of n_i^2, largest n_i)
 * for the rest of the process: later trinv_tril_inverse_batched calls with
 * the same signature use it (the default is leaf 64 for FP32, 32 for FP64,
 * and the occupancy limit). opts->upper gives TRINV_ERR_UNSUPPORTED: the
 * configuration tuned on the lower form serves upper calls with the same
 * orders. Arguments and errors as
 * trinv_tril_inverse_batched. On return X_packed and status_dev hold the
 * result of the chosen configuration; `out` (nullable) receives it. Uniform
 * batches that take the level path have nothing to tune (out->ms = -1).
 * Synchronises `stream` (not for graph capture: tune first, then capture).
 * If the environment variable TRINV_TUNE_CACHE names a file, every result is
 * appended to it as a line "device mode count sum sum_sq largest leaf
 * wgs_per_cu tile ms" (device: architecture name / CU count), and the first
 * lookup of a process loads that file's lines for the current device, so a
 * later process reuses them without tuning (a missing or unreadable file is
 * ignored).
 */
int trinv_batched_autotune(int mode, int64_t batch, const int32_t *n_host, const int32_t *n_dev,
                           const int64_t *off_host, const int64_t *off_dev, const void *L_packed,
                           void *X_packed, int32_t *status_dev, const trinv_opts *opts, void *ws,
                           size_t ws_bytes, trinv_stream_t stream, trinv_batched_config *out);

/* Sets the configuration later trinv_tril_inverse_batched calls use for
 * batches with this order signature (as trinv_batched_autotune would), e.g.
 * one an earlier process found. cfg->leaf 32 or 64, cfg->wgs_per_cu >= 0 (0
 * or above the occupancy limit: that limit), cfg->tile 0, 64 or 128; else
 * TRINV_ERR_ARG. */
int trinv_batched_set_config(int mode, int64_t batch, const int32_t *n_host, const trinv_batched_config *cfg);

/* The configuration the next trinv_tril_inverse_batched call with this
 * order signature would use (set, tuned in this process, or loaded from the
 * TRINV_TUNE_CACHE file; otherwise the default leaf, wgs_per_cu = 0 and
 * tile 128); cfg->ms = -1. TRINV_ERR_ARG for batch <= 0, a null pointer or an order
 * outside 1..1024; TRINV_ERR_UNSUPPORTED for modes other than F64 / F32. */
int trinv_batched_get_config(int mode, int64_t batch, const int32_t *n_host, trinv_batched_config *cfg);

/*
 * Adjoint of X = L^-1 for a strided batch of lower-triangular matrices:
 *     gradL = -tril(X^T G X^T)
 * (from dX = -X dL X; not part of the paper). X is the forward's output
 * (lower, strict upper read as zero), G the gradient with respect to X (only
 * its lower triangle contributes), gradL the gradient with respect to the
 * lower entries of L (strict upper written as 0). mode: TRINV_F32 or
 * TRINV_F64. Matrix b starts at element b * stride of each array; all have
 * leading dimension n. ws: workspace of trinv_backward_workspace_bytes.
 */
size_t trinv_backward_workspace_bytes(int mode, int64_t batch, int64_t n);
int trinv_tril_inverse_backward(int mode, int64_t batch, int64_t n, const void *X, const void *G,
                                void *gradL, int64_t stride, void *ws, size_t ws_bytes,
                                trinv_stream_t stream);

/*
 * Factored inverse from given triangular factors A = L U (Section 5,
 * algorithm SKUL's output statement: with S = U^-1 and K = L^-1,
 * S K = A^-1): Linv = L^-1 (lower), Uinv = U^-1 (upper, computed through the
 * transposed view of U; L and U^T are inverted together as a batch of two),
 * and, if Ainv != NULL, Ainv = Uinv * Linv (dense).
 * L (lower, only its lower triangle read) and U (upper, only its upper
 * triangle read): device, leading dimensions ldl, ldu >= n. l_unit /
 * u_unit: take that factor's diagonal as 1. Linv, Uinv, Ainv: device
 * outputs written in full (zeros outside the triangles of Linv and Uinv),
 * leading dimensions ldli, ldui, ldai >= n (ldai ignored when Ainv is NULL);
 * no output may overlap an input or another output (TRINV_ERR_ARG).
 * mode: TRINV_F64 or TRINV_F32. ws: at least trinv_factored_workspace_bytes
 * bytes. With opts->blocking: an exact zero diagonal entry gives
 * TRINV_ERR_SINGULAR with info->first_bad_index = the smallest 1-based i at
 * which L_ii or U_ii is zero; a NaN or an infinity in an output gives
 * TRINV_ERR_NONFINITE. info: nullable.
 */
size_t trinv_factored_workspace_bytes(int mode, int64_t n, const trinv_opts *opts);
int trinv_factored_inverse(int mode, int64_t n, const void *L, int64_t ldl, int32_t l_unit, const void *U,
                           int64_t ldu, int32_t u_unit, void *Linv, int64_t ldli, void *Uinv, int64_t ldui,
                           void *Ainv, int64_t ldai, const trinv_opts *opts, void *ws, size_t ws_bytes,
                           trinv_stream_t stream, trinv_info *info);

/*
 * Algorithm SKUL (Section 5): the Crout factorization A = L U (L lower with
 * general diagonal, U unit upper; no pivoting, so A must admit it, e.g. be
 * diagonally dominant or symmetric positive definite) together with
 * S = U^-1 and K = L^-1, so that S K = A^-1; optionally Ainv = S K.
 * mode: TRINV_F64 or TRINV_F32. A: device n x n row-major (leading dimension
 * n), read only; L, U, S, K (and Ainv if not NULL): device n x n outputs,
 * written in full, none overlapping A or each other (else TRINV_ERR_ARG).
 * opts: leaf (the triangular inverses), blocking; upper / unit_diag / beta > 2
 * give TRINV_ERR_UNSUPPORTED. ws: trinv_skul_workspace_bytes bytes (holds a
 * working copy of A). A zero pivot L(i, i) makes the outputs non-finite and,
 * with blocking, returns TRINV_ERR_SINGULAR with info->first_bad_index = i
 * (1-based). info: nullable.
 */
size_t trinv_skul_workspace_bytes(int mode, int64_t n, const trinv_opts *opts);
int trinv_skul(int mode, int64_t n, const void *A, void *L, void *U, void *S, void *K, void *Ainv,
               const trinv_opts *opts, void *ws, size_t ws_bytes, trinv_stream_t stream, trinv_info *info);

/*
 * Algorithm SQR (Section 5): modified Gram-Schmidt A = Q R (Q with
 * orthonormal columns, R upper triangular with positive diagonal) together
 * with S = R^-1, so that S Q^T = A^-1; optionally Ainv = S Q^T.
 * mode: TRINV_F64 or TRINV_F32; n <= 4096 (else TRINV_ERR_UNSUPPORTED).
 * A: device n x n row-major (leading dimension n), read only; Q, R, S (and
 * Ainv if not NULL): device n x n outputs written in full (R and S zero below
 * the diagonal), none overlapping A or each other (else TRINV_ERR_ARG).
 * opts: leaf (the triangular inverse), blocking; upper / unit_diag / beta > 2
 * give TRINV_ERR_UNSUPPORTED. ws: trinv_sqr_workspace_bytes bytes (holds a
 * working copy of A). A column whose orthogonalized part is exactly zero
 * (rank deficiency) makes the outputs non-finite and, with blocking, returns
 * TRINV_ERR_SINGULAR with info->first_bad_index = that column (1-based).
 * info: nullable.
 */
size_t trinv_sqr_workspace_bytes(int mode, int64_t n, const trinv_opts *opts);
int trinv_sqr(int mode, int64_t n, const void *A, void *Q, void *R, void *S, void *Ainv,
              const trinv_opts *opts, void *ws, size_t ws_bytes, trinv_stream_t stream, trinv_info *info);

/*
 * General inverse by BRSI with gamma = 2 (Section 5, Steps of BRSI and the
 * gamma = 2 derivation): with S11 = A11^-1, S22 = A22^-1, S12 = -S11 A12 S22
 * and W = (I + S12 A21)^-1, all inverses by the same recursion,
 *   A^-1 = [[W S11, W S12], [-S22 A21 W S11, S22 - S22 A21 W S12]].
 * No pivoting: every diagonal block met by the recursion must be invertible
 * (e.g. A symmetric positive definite or diagonally dominant). The order is
 * padded internally to b 2^k (b <= 128) with an identity tail.
 * mode: TRINV_F64 or TRINV_F32. A: device n x n, leading dimension lda >= n,
 * read only; Ainv: device n x n, leading dimension ldx >= n, not overlapping
 * A (else TRINV_ERR_ARG). opts: blocking; upper / unit_diag / beta > 2 give
 * TRINV_ERR_UNSUPPORTED. ws: trinv_brsi_workspace_bytes bytes (about 4 n^2
 * elements). A zero pivot in a bottom-level block makes the output
 * non-finite and, with blocking, returns TRINV_ERR_SINGULAR with
 * info->first_bad_index = the 1-based position of that pivot inside its
 * bottom-level block (the blocks are copies, so no global index exists).
 * info: nullable.
 */
size_t trinv_brsi_workspace_bytes(int mode, int64_t n, const trinv_opts *opts);
int trinv_brsi(int mode, int64_t n, const void *A, int64_t lda, void *Ainv, int64_t ldx,
               const trinv_opts *opts, void *ws, size_t ws_bytes, trinv_stream_t stream, trinv_info *info);

/*
 * Measurement helper (not part of the method): FP64 relative residual of a
 * candidate inverse, computed on the GPU with FP64 MFMA products:
 *   out_host[0] = ||L X - I||_F, [1] = ||tril(L)||_F, [2] = ||X||_F.
 * mode selects the element type of L and X (F64 or F32; the arithmetic is
 * FP64 in both cases). Waits for the GPU. ws: trinv_residual_workspace_bytes.
 */
size_t trinv_residual_workspace_bytes(int mode, int64_t n);
int trinv_residual(int mode, int64_t n, const void *L, int64_t ldl, const void *X, int64_t ldx,
                   void *ws, size_t ws_bytes, trinv_stream_t stream, double *out_host);

/*
 * The refinement's residual product on its own (not part of the paper; the
 * residual R = I - L X of TRINV_BF16_REFINE / TRINV_F16_REFINE): R is
 * assembled in FP64 from the exact diagonal terms and the strictly-lower
 * product N_L N_X formed from low-precision slices of both factors (nsplit =
 * 3: hi*hi + hi*lo + lo*hi; nsplit = 2: hi*hi + lo*hi, valid only when every
 * strictly-lower entry of X, times the FP16 scale, is exactly representable
 * in the low-precision type, as in the refinement's first iterate) with FP32
 * accumulation, the same kernels and epilogue the refinement runs.
 * mode: TRINV_BF16_REFINE or TRINV_F16_REFINE (FP16: L and X scaled by powers
 * of two from max |L| and max |X|). L, X: device FP64, lower triangles read,
 * ldl, ldx >= n. R: device FP32, ldr >= n; its lower triangle receives R
 * (R is lower triangular); inside the 256 x 256 diagonal tiles the strict
 * upper part is written as 0, elsewhere it is not touched. No overlap of R
 * with L or X (TRINV_ERR_ARG). out_host (host, 5 doubles): ||R||_F,
 * ||tril(L)||_F, ||tril(X)||_F, the estimated error of ||R|| / (||L|| ||X||)
 * and its worst-case bound (as trinv_info's resid_error_est and
 * resid_error_bound). ws: trinv_refine_residual_workspace_bytes bytes.
 * Waits for the GPU. Orders above 2^23 - 128 give TRINV_ERR_UNSUPPORTED (the
 * workspace query returns 0 for them).
 */
size_t trinv_refine_residual_workspace_bytes(int mode, int64_t n);
int trinv_refine_residual(int mode, int64_t n, const void *L, int64_t ldl, const void *X, int64_t ldx,
                          int32_t nsplit, float *R, int64_t ldr, void *ws, size_t ws_bytes,
                          trinv_stream_t stream, double *out_host);

/*
 * Measurement helpers (not part of the method). When profiling is enabled,
 * every profiled launch of the library carries two HIP events on its kernel
 * dispatches (start of the first kernel, end of the last; hipExtLaunchKernel,
 * on the stream the launch uses), and is filed under its kernel class with the
 * launch's algorithmic flops and bytes (the work the method must do, not the
 * work the tiles execute). trinv_profile_enable(1) starts a new profile
 * (dropping the old one), trinv_profile_enable(0) stops recording.
 * trinv_profile_read waits for the recorded events and writes up to
 * max_entries per-class totals into out (host memory); it returns the number
 * of classes, or a negative status on a HIP error.
 */
typedef struct {
  char name[32];      /* kernel class */
  int64_t launches;   /* launches recorded */
  double total_ms;    /* summed event-to-event time of those launches */
  double flops;       /* summed algorithmic flops */
  double bytes;       /* summed algorithmic HBM bytes */
} trinv_profile_entry;

int trinv_profile_enable(int on);
int trinv_profile_read(trinv_profile_entry *out, int max_entries);

/*
 * Restricts recording to the kernel classes named in `classes` (host string,
 * comma-separated, copied; NULL or "" records every class). A timed launch
 * ends with the writes its completion event needs made visible, which costs
 * a few microseconds after it; restricting the classes keeps that cost off
 * the others. Returns TRINV_OK.
 */
int trinv_profile_select(const char *classes);

#ifdef __cplusplus
}
#endif

#endif /* TRINV_H */
