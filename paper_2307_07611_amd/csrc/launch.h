// Host-side launchers of the library's kernels (internal; not the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trinv {

// ---------------------------------------------------------------- leaves
// Inverts the diagonal leaf blocks of order `leaf` (the last one may be
// shorter) of a strided batch of lower matrices. If Xlp / Xlpt are non-null,
// a BF16 (lp_is_f16 = 0) or FP16 (1) copy of each leaf block is stored there
// too, row-major / transposed (leading dimension ldxl, same batch stride),
// of the values times lp_scale (a power of two). first_bad: atomic minimum of
// the 1-based indices of exact zero pivots (init to all ones); one word for
// the whole call, or one per matrix (per_matrix_status = 1). round_x (needs
// Xlp): X receives the copy's values (divided by lp_scale) off the diagonal.
template <typename T>
hipError_t launch_leaf(int64_t n, const T* L, int64_t ldl, T* X, int64_t ldx, int64_t stride, int64_t batch,
                       int leaf, int unit, void* Xlp, void* Xlpt, int lp_is_f16, int64_t ldxl, double lp_scale,
                       uint64_t* first_bad, int per_matrix_status, hipStream_t s, int round_x = 0,
                       int zero_upper = 0);

// ---------------------------------------------------------------- tile products
// A tile product D = alpha * op(A) * op(B) over a set of output tiles
// (TM x TN = 128 x 128) with a K range per tile that skips the zero
// triangles of triangular operands. The caller states the K range rule, the
// tile set and the order in which tiles are dispatched (heaviest first).
enum KLo { kLoZero = 0, kLoN0 = 1, kLoM0 = 2, kLoMax = 3 };   // k >= 0 | n0 | m0 | max(m0, n0)
enum KHi { kHiK = 0, kHiM1 = 1, kHiN1 = 2 };                   // k < K | m0 + TM | n0 + TN
// Low-precision products of lower tiles over panel-blocked planes, each tile
// over its own range n0 .. m0 + TM (with kHiM1); the operands must hold zeros
// wherever that range leaves their triangles.
enum { kLoN0Pb = 5 };
enum Tiles { kAllTiles = 0, kLowerTiles = 1 };                  // all tiles | tiles with it >= jt
enum Order {
  kColAsc = 0,   // all tiles, tile column ascending (work shrinks with the column)
  kRowDesc = 1,  // all tiles, tile row descending (work grows with the row)
  kDiagDesc = 2, // lower tiles, it - jt descending
  kRowAsc = 3,   // lower tiles, tile row ascending
  kColDesc = 4   // lower tiles, tile column descending
};
// Element masks applied when an operand tile is staged (indices inside the
// product): 0 none, 1 lower, 2 strict lower, 3 upper; for A(m, k) lower
// means k <= m, for B(k, n) lower means k >= n.
struct GemmBatch {
  int64_t nmerge;                  // products per batch entry (merges of a level)
  int64_t nbatch;                  // independent batch entries
  int64_t M, N, K;                 // sizes of every product but the last merge
  int64_t M_last, N_last, K_last;  // sizes of the last merge of each batch entry
};

// Element (i, j) of merge z of batch entry b is
//   base[b * bstride2 + z * bstride + i * ld + j]   (or [.. + j * ld + i] if transposed).
template <typename T>
struct Operand {
  T* base;
  int64_t ld;
  int64_t bstride;
  int64_t bstride2;
};

template <typename TI>
struct GemmArgs {
  Operand<const TI> A, B;
  Operand<TI> D;        // base null: D is not stored
  Operand<TI> Zmirror;  // optional: zero the transposed position of each tile
  Operand<void> Dlp;    // optional: BF16 (lp_is_f16 = 0) / FP16 (1) copy of D
  int lp_is_f16;
  double alpha;
  int a_trans, b_trans;   // operand read transposed: A(m,k) = A[k*ld + m]
  int amask, bmask;
  int tiles, order, klo, khi;
  int out_lower;          // store 0 where col > row
  int mirror_skip_diag;   // do not zero the mirror of a diagonal tile
  int subtract_identity;  // D = alpha*A*B - I (row == col inside the product)
  double* tile_sq;        // optional: per-tile sum of squares of D (FP64)
  GemmBatch bt;
  // Refinement residual epilogue (FP64 product of the strictly lower parts
  // N_L N_X): R = I - L X assembled in FP64 from acc and the diagonals,
  // stored as FP32 (R32, ldr) and as a transposed low-precision copy (Rt,
  // ldrt, BF16 or FP16 by lp_is_f16); per-tile sums of R^2 (tile_sq) and of
  // X^2 (tile_sqx) over the lower triangle.
  const TI* Lfull;
  int64_t ldl;
  const TI* Xfull;
  int64_t ldx;
  const double* dL;
  const double* dX;
  float* R32;
  int64_t ldr;
  void* Rt;
  int64_t ldrt;
  double* tile_sqx;
  int refine_resid;
  int accumulate;  // D = alpha * A B + D
};

template <typename TI, typename TC>
hipError_t launch_gemm(const GemmArgs<TI>& a, hipStream_t s);
int64_t gemm_tiles(const GemmBatch& bt, int tiles);

// ---------------------------------------------------------------- elementwise
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t count, hipStream_t s);
// out[0] = sum of squares of tril(A) (lower = 1) or A (lower = 0).
template <typename T>
hipError_t launch_sumsq(const T* A, int64_t n, int64_t lda, int lower, int unit, double* partial,
                        int64_t npartial, double* out, hipStream_t s);
hipError_t launch_reduce_sum(const double* partial, int64_t count, double* out, hipStream_t s);
// out[0] = sum of v[i]^2 (one block, fixed order).
hipError_t launch_sumsq_vec(const double* v, int64_t count, double* out, hipStream_t s);
// out[0] = max |A(i, j)| over the lower triangle (or all of A), diagonal
// taken as 1 if unit; partial: npartial doubles of scratch.
template <typename T>
hipError_t launch_maxabs(const T* A, int64_t n, int64_t lda, int lower, int unit, double* partial, int64_t npartial,
                         double* out, hipStream_t s);
// Diagonal-block step of the blocked Crout factorization (skul.hip): factors
// W[0:nb, 0:nb] (nb <= 128) into the L block (lower) and the U block (unit
// upper) at L / U (leading dimension ld) and writes their inverses K = L^-1,
// S = U^-1 at K / S (leading dimension ldk); zero pivots -> *bad (row0 + p + 1).
// A batch of `count` blocks at strides sw (W), slu (L, U) and sk (K, S) runs
// in one launch, one workgroup per block.
template <typename T>
hipError_t launch_crout_diag(const T* W, int64_t ldw, int64_t sw, int nb, T* L, T* U, int64_t ld, int64_t slu, T* K,
                             T* S, int64_t ldk, int64_t sk, int64_t count, int64_t row0, uint64_t* bad,
                             hipStream_t s);
// Zero bytes [p, p + bytes) (a multiple of 4) with a kernel (no memset node).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// out[0] = min over blocks b of (b * m + words[b]) over the set words (all ones = unset).
hipError_t launch_fold_status(const uint64_t* words, int64_t count, int64_t m, uint64_t* out, hipStream_t s);
// A(i, i) = v for i < n.
template <typename T>
hipError_t launch_set_diag(T* A, int64_t ld, int64_t n, T v, hipStream_t s);
// dst block b = alpha * src block b for nblocks m x m blocks (block b of src at
// src + b sstride, leading dimension lds; likewise dst).
template <typename T>
hipError_t launch_block_copy(const T* src, int64_t lds, int64_t sstride, T* dst, int64_t ldd, int64_t dstride,
                             int64_t m, int64_t nblocks, T alpha, hipStream_t s);
// Panel step of blocked modified Gram-Schmidt (sqr.hip): orthogonalizes the
// columns p0 .. p0 + w - 1 of V (n x n, leading dimension ld, n <= 4096,
// w <= mgs_panel_width(n)) among themselves in one workgroup, writing those
// columns of Q and the block R[p0 : p0 + w, p0 : p0 + w]; a zero norm sends
// p0 + j + 1 to *bad.
int mgs_panel_width(int64_t n);
template <typename T>
hipError_t launch_mgs_panel(const T* V, T* Q, T* R, int64_t ld, int64_t n, int64_t p0, int w, uint64_t* bad,
                            hipStream_t s);
// dst block b (m x m) = [[src block b (n x n), 0], [0, I]] for n <= m (src
// null: the identity), blocks at strides sstride / dstride.
template <typename T>
hipError_t launch_embed(const T* src, int64_t lds, int64_t sstride, int64_t n, T* dst, int64_t ldd, int64_t dstride,
                        int64_t m, int64_t nblocks, hipStream_t s);
// dst (rows x cols) = sum over c < count of src + c stride, in order of c.
template <typename T>
hipError_t launch_sum_blocks(const T* src, int64_t lds, int64_t stride, int64_t count, int64_t rows, int64_t cols,
                             T* dst, int64_t ldd, hipStream_t s);
// status[i] = first_bad[i] == all ones ? 0 : first_bad[i]  (int32 per matrix).
hipError_t launch_status_to_i32(const uint64_t* first_bad, int32_t* status, int64_t count, hipStream_t s);
// B = A^T for an n x n matrix.
template <typename T>
hipError_t launch_transpose(const T* A, int64_t lda, T* B, int64_t ldb, int64_t n, hipStream_t s);
// A = A^T in place for an n x n matrix.
template <typename T>
hipError_t launch_transpose_inplace(T* A, int64_t lda, int64_t n, hipStream_t s);
// off[i] = sum_{j < i} n_j^2 over the batch's orders (outside 1..1024: 0)
hipError_t launch_dense_offsets(const int32_t* n_dev, int64_t batch, int64_t* off, hipStream_t s);
// B_i = A_i^T for every matrix of a packed batch (skips orders outside
// 1..1024 and B ranges ending beyond capb elements)
template <typename T>
hipError_t launch_transpose_packed(int64_t batch, const int32_t* n_dev, const int64_t* offa, const T* A,
                                   const int64_t* offb, T* B, int64_t capb, hipStream_t s);
// *flag |= 1 if the n x n matrix A holds a NaN or an infinity (flag: a
// device word the caller clears).
template <typename T>
hipError_t launch_nonfinite(const T* A, int64_t n, int64_t lda, unsigned* flag, hipStream_t s);
// status[b] = -2 where status[b] == 0 and the n x n matrix b (leading
// dimension n, at element b * stride of X) holds a NaN or an infinity.
template <typename T>
hipError_t launch_nonfinite_status(const T* X, int64_t n, int64_t stride, int64_t batch, int32_t* status,
                                   hipStream_t s);

// Uneven batch in one persistent launch (persistent.hip): a plan kernel sorts
// the matrices by order into `order` (batch entries) and resets `queue`, then
// `grid` workgroups invert whole matrices taken from the queue (leaves of
// order `leaf`, 32 or 64, by the column recurrence; then the 2 x 2 levels on
// MFMA tiles).
// status[i]: 0, the 1-based index of the first zero diagonal, -1 for an
// order outside [1, 1024], or -2 if a NaN or an infinity was stored into X_i.
template <typename T>
hipError_t launch_batched(int64_t batch, const int32_t* n_dev, const int64_t* off_dev, const T* L, T* X,
                          int32_t* status, int32_t* order, uint32_t* queue, int unit, int grid, int leaf,
                          int tmax, hipStream_t s);
// Device scratch of the allocation-free batched entry point (a file-scope
// device array, one copy per device): room for the plan of kNoAllocMaxBatch
// matrices and the queue counter. Returns this device's addresses (looked up
// once per device).
constexpr int64_t kNoAllocMaxBatch = 65536;
constexpr int kMaxDevices = 64;
hipError_t batched_scratch(int32_t** order, uint32_t** queue);
// Resident workgroups of the persistent kernel (leaf order 32 or 64) per CU
// (occupancy) and, in *cus, the device's CU count.
template <typename T>
int batched_occupancy(int leaf, int* cus);
// Persistent grid size: per_cu workgroups per CU (the occupancy if per_cu is
// 0 or above it), at most batch.
template <typename T>
int batched_grid(int64_t batch, int leaf, int per_cu);

}  // namespace trinv
