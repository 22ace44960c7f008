// Mixed-precision (BF16 / FP16 MFMA, FP32 accumulation) kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.h"

namespace trinv {

// Which fused epilogue a low-precision product runs.
enum LpEpilogue {
  kLpEpT = 0,      // store alpha*acc transposed (low precision): T for the next product
  kLpEpX21 = 1,    // X21 = alpha*acc: FP64 X, low-precision row-major and transposed copies,
                   // zero the FP64 X12 block
  kLpEpResid = 2,  // R = I - L X assembled in FP64 from alpha*acc = N_L N_X (lower tiles):
                   // FP32 R, low-precision transposed R (if Rt is set), per-tile
                   // ||R||^2 and ||X||^2
  kLpEpCorr = 3    // X <- X + D_X R + alpha*acc (alpha*acc = N_X R), lower tiles, in place
};

// All operands in element units of their own type. Low-precision operands:
// A row-major [m][k]; B stored transposed, Bt[n][k] = B(k, n), so both are
// k-contiguous. Every low-precision buffer must have at least 8 readable
// padding columns past the last column a product uses.
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
  double* Xmirror;  // kLpEpX21: X12 block base (FP64 zeros)
  void* Xlp;        // kLpEpX21: row-major low-precision copy of X21
  int64_t ldxlp, xlp_bstride;
  void* Xlpt;  // kLpEpX21: transposed low-precision copy (element (r,c) -> [c][r])
  int64_t ldxlpt, xlpt_bstride;
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
};

struct LpConfig {
  int f16;     // 0: BF16, 1: FP16
  int nsplit;  // 1: hi*hi, 3: hi*hi + hi*lo + lo*hi
  int amask, bmask;
  int tiles, order, klo, khi;
  int epi;
};

hipError_t launch_gemm_lp(const LpGemmArgs& a, const LpConfig& c, hipStream_t s);
int64_t gemm_lp_tiles(const GemmBatch& bt, int tiles);

// Low-precision slices of a lower-triangular FP64 matrix times a power-of-two
// scale (64 x 64 tiles of the lower triangle; elements above the diagonal are
// written as 0 inside diagonal tiles and not at all elsewhere):
//   hi = round(scale v), lo = round(scale v - hi) (round-to-nearest-even in
// the target type); each output is optional; "t" outputs are transposed
// (element (i,j) at [j][i]). diag (optional) receives the unscaled diagonal.
// strict: the slices hold the strictly lower part (zero diagonal).
hipError_t launch_split(const double* S, int64_t lds, int64_t n, int f16, void* hi, void* lo, void* hi_t, void* lo_t,
                        int64_t ldo, double* diag, int unit, int strict, double scale, hipStream_t s);
// The transposed hi slice only, from an FP32 lower-triangular matrix.
hipError_t launch_split_f32(const float* S, int64_t lds, int64_t n, int f16, void* hi_t, int64_t ldo, double scale,
                            hipStream_t s);
// Zeros in a band of `band` columns beside the tiles the split writes: to the
// right of each 64-row strip's diagonal tile (right = 1, row-major lower
// planes) or to its left (right = 0, transposed planes). Low-precision planes
// read over block-union K ranges need these zeros.
hipError_t launch_zero_band(void* P, int64_t ldo, int64_t n, int64_t band, int right, hipStream_t s);

}  // namespace trinv
