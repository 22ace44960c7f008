// Mixed-precision (BF16 / FP16 MFMA, FP32 accumulation) kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.h"

namespace trinv {

// Which fused epilogue a low-precision product runs.
enum LpEpilogue {
  kLpEpT = 0,      // store alpha*acc transposed (low precision): T for the next product
  kLpEpX21 = 1,    // X21 = alpha*acc: FP64 X, low-precision row-major and transposed copies
                   // (the FP64 X12 block is zeroed by the leaf launch)
  kLpEpResid = 2,  // R = I - L X assembled in FP64 from alpha*acc = N_L N_X (lower tiles):
                   // FP32 R, low-precision transposed R (if Rt is set), per-tile
                   // ||R||^2 and ||X||^2
  kLpEpCorr = 3    // X <- X + D_X R + alpha*acc (alpha*acc = N_X R), lower tiles, in place
};

// All operands in element units of their own type. Low-precision operands:
// A row-major [m][k]; B stored transposed, Bt[n][k] = B(k, n), so both are
// k-contiguous. Every low-precision buffer must have at least 8 readable
// padding columns past the last column a product uses. The refinement
// products (klo = kLoN0Pb) read panel-blocked planes instead, and lda / ldb
// are then their K blocks per panel; their residual epilogue writes Rt
// panel-blocked too (ldrt = K blocks per panel).
struct LpGemmArgs {
  const void* A_hi;
  const void* A_lo;  // second slice (3-product split) or null
  int64_t lda, a_bstride;
  const void* Bt_hi;
  const void* Bt_lo;
  int64_t ldb, b_bstride;
  GemmBatch bt;  // nbatch must be 1
  double alpha;
  // epilogue operands
  void* Ot;  // kLpEpT: transposed output
  int64_t ldot, ot_bstride;
  double* X;  // kLpEpX21: X21 block base; kLpEpResid / kLpEpCorr: X
  int64_t ldx, x_bstride;
  void* Xlp;        // kLpEpX21: row-major low-precision copy of X21
  int64_t ldxlp, xlp_bstride;
  void* Xlpt;  // kLpEpX21: transposed low-precision copy (element (r,c) -> [c][r])
  int64_t ldxlpt, xlpt_bstride;
  int x_round;  // kLpEpX21: the FP64 X21 holds the low-precision copy's values (divided by lp_scale)
  const double* L;  // kLpEpResid
  int64_t ldl;
  const double* dL;  // diag(L) (kLpEpResid)
  const double* dX;  // diag(X) before this call (kLpEpResid, kLpEpCorr)
  float* R32;        // kLpEpResid: written; kLpEpCorr: read
  int64_t ldr;
  void* Rt;  // kLpEpResid: transposed low-precision R
  int64_t ldrt;
  double* tile_sq;   // kLpEpResid: per-tile sum of R^2
  double* tile_sqx;  // kLpEpResid: per-tile sum of X^2 (lower triangle)
  // Power-of-two factor applied to the values before they are stored in low
  // precision (kLpEpX21 copies, kLpEpResid's Rt); the accumulator itself is
  // scaled by alpha in every epilogue.
  double lp_scale;
  // kLpEpCorr, BF16, interior tiles only (optional): the slices of the updated
  // X that the next residual reads, as the split would write them (strictly
  // lower part, hi / lo in the transposed B role, panel-blocked with kbx K
  // blocks), and its FP64 diagonal (dXn). Neither may be read by the same call.
  void* Xn_tb_hi;
  void* Xn_tb_lo;
  double* dXn;
  int64_t kbx;
};

struct LpConfig {
  int f16;     // 0: BF16, 1: FP16
  int nsplit;  // 1: hi*hi, 2: hi*hi + lo*hi (B exact in hi), 3: hi*hi + hi*lo + lo*hi
  int amask, bmask;
  int tiles, order, klo, khi;
  int epi;
};

hipError_t launch_gemm_lp(const LpGemmArgs& a, const LpConfig& c, hipStream_t s);
int64_t gemm_lp_tiles(const GemmBatch& bt, int tiles);

// Panel-blocked plane (the operands of the refinement products): rows in
// panels of 256, K in blocks of 16; the 256 x 16 block of panel p and K block b
// is 8 KB of contiguous memory at element ((p kb + b) 4096), row-major (32-byte
// rows), with the two 16-byte halves of a row exchanged in rows whose bit 3 is
// set. A stage of a product is then a contiguous range per operand tile, which
// direct global -> LDS loads copy as is: the half exchange is the LDS bank
// swizzle of the fragment reads. kb = K blocks per panel.
__host__ __device__ inline int64_t pb_index(int64_t r, int64_t k, int64_t kb) {
  const int64_t rr = r & 255, kk = k & 15;
  return (((r >> 8) * kb + (k >> 4)) << 12) + (rr << 4) + ((((kk >> 3) ^ ((rr >> 3) & 1))) << 3) + (kk & 7);
}
// K blocks per panel for order n: the splits write whole 64-wide tiles (up
// to the next multiple of 64), and the last stage of a product may read up to
// 31 elements past the last column (masked in LDS, but inside the plane).
inline int64_t pb_kblocks(int64_t n) { return (n + 63) / 64 * 4 + 2; }
inline size_t pb_elems(int64_t n) { return (size_t)((n + 255) / 256) * (size_t)pb_kblocks(n) * 4096; }

// Outputs of a split (any may be null): row-major hi / lo and transposed
// hi_t / lo_t with leading dimension ldo; panel-blocked hi_b / lo_b (element
// (i, j) at row i, k = j) and hi_tb / lo_tb (element (i, j) at row j, k = i)
// with kb K blocks per panel.
struct SplitOut {
  unsigned short *hi, *lo, *hi_t, *lo_t;
  int64_t ldo;
  unsigned short *hi_b, *lo_b, *hi_tb, *lo_tb;
  int64_t kb;
  // optional, one double per 64 x 64 tile of the lower triangle (split_tiles):
  // the sum of squares of the values read (lower triangle, diagonal included,
  // before scaling) and of the diagonal values alone
  double *sq, *dsq;
};
// Tiles (workgroups) of one split of order n.
inline int64_t split_tiles(int64_t n) {
  const int64_t t = (n + 63) / 64;
  return t * (t + 1) / 2;
}

// Low-precision slices of a lower-triangular FP64 matrix times a power-of-two
// scale (64 x 64 tiles of the lower triangle; elements above the diagonal are
// written as 0 inside diagonal tiles and not at all elsewhere):
//   hi = round(scale v), lo = round(scale v - hi) (round-to-nearest-even in
// the target type). diag (optional) receives the unscaled diagonal. strict:
// the slices hold the strictly lower part (zero diagonal).
hipError_t launch_split(const double* S, int64_t lds, int64_t n, int f16, const SplitOut& o, double* diag, int unit,
                        int strict, double scale, hipStream_t s);
// The same from an FP32 lower-triangular matrix (no diagonal output).
// The same split (strict, no unit diagonal) of a matrix whose strictly lower
// values are exactly a row-major low-precision copy divided by the
// power-of-two `scale` (lp, leading dimension ldlp): those values are read
// from the copy (2 bytes instead of 8), the diagonal from S. Panel-blocked
// hi slices only (hi_b, hi_tb); the lo slices of such a matrix are zero.
hipError_t launch_split_lp_source(const double* S, int64_t lds, const void* lp, int64_t ldlp, int64_t n, int f16,
                                  const SplitOut& o, double* diag, double scale, hipStream_t s);
hipError_t launch_split_f32(const float* S, int64_t lds, int64_t n, int f16, const SplitOut& o, double scale,
                            hipStream_t s);
// Zeros in a band of `band` columns (multiple of 8) beside the tiles the split
// writes, in `count` (<= 8) panel-blocked planes in one launch: to the right
// of each 64-row strip's diagonal tile (right[i] = 1, planes holding a lower
// triangle) or to its left (right[i] = 0, transposed planes). The refinement
// products read each panel up to the end of its diagonal 256 x 256 block and
// need these zeros.
hipError_t launch_zero_band_pb(void* const* planes, const int* right, int count, int64_t kb, int64_t n, int64_t band,
                               hipStream_t s);

}  // namespace trinv
