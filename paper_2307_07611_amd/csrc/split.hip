// Staging casts of the mixed-precision path: a lower-triangular FP64 (or FP32)
// matrix, times a power-of-two scale s, is cut into low-precision slices
// hi = round(s v) and lo = round(s v - hi) (round-to-nearest-even in BF16 or
// FP16; s v and s v - hi are exact in FP64), written row-major and/or
// transposed (through a 64 x 64 LDS tile so both stores are coalesced), plus
// the unscaled FP64 diagonal. HBM-bound: one read of the lower triangle,
// 2 bytes written per requested slice and element.
#include "common.h"
#include "lowp.h"

namespace trinv {

namespace {
typedef unsigned short u16;

template <int F16>
__device__ __forceinline__ u16 lp_bits(double v, double* back) {
  if (F16) {
    const _Float16 h = (_Float16)v;
    *back = (double)h;
    return __builtin_bit_cast(u16, h);
  }
  const __bf16 h = (__bf16)v;
  *back = (double)(float)h;
  return __builtin_bit_cast(u16, h);
}
}  // namespace

// Grid: one block per 64 x 64 tile of the lower triangle (tile row it >= tile col jt).
template <int F16, typename TS>
__global__ __launch_bounds__(256) void k_split(const TS* __restrict__ S, int64_t lds, int64_t n,
                                               u16* __restrict__ hi, u16* __restrict__ lo, u16* __restrict__ hi_t,
                                               u16* __restrict__ lo_t, int64_t ldo, double* __restrict__ diag,
                                               int unit, int strict, double scale) {
  __shared__ u16 th[64][66];
  __shared__ u16 tl[64][66];
  const int64_t q = blockIdx.x;
  int64_t it = (int64_t)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
  while (it * (it + 1) / 2 > q) --it;
  while ((it + 1) * (it + 2) / 2 <= q) ++it;
  const int64_t jt = q - it * (it + 1) / 2;
  const int64_t i0 = it * 64, j0 = jt * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  for (int r = ty; r < 64; r += 4) {
    const int64_t i = i0 + r, j = j0 + tx;
    u16 h = 0, l = 0;
    if (i < n && j < n) {
      double v = (j <= i) ? (double)S[i * lds + j] : 0.0;
      if (unit && i == j) v = 1.0;
      if (i == j && diag) diag[i] = v;
      if (strict && i == j) v = 0.0;  // slices of the strictly lower part
      v *= scale;
      double hb;
      h = lp_bits<F16>(v, &hb);
      double lb;
      l = lp_bits<F16>(v - hb, &lb);
      if (hi) hi[i * ldo + j] = h;
      if (lo) lo[i * ldo + j] = l;
    }
    th[r][tx] = h;
    tl[r][tx] = l;
  }
  if (!hi_t && !lo_t) return;
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t c = j0 + r, rr = i0 + tx;  // transposed element (c, rr) = S(rr, c)
    if (c < n && rr < n) {
      if (hi_t) hi_t[c * ldo + rr] = th[tx][r];
      if (lo_t) lo_t[c * ldo + rr] = tl[tx][r];
    }
  }
}

template <typename TS>
static hipError_t split_t(const TS* S, int64_t lds, int64_t n, int f16, void* hi, void* lo, void* hi_t, void* lo_t,
                          int64_t ldo, double* diag, int unit, int strict, double scale, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t T = (n + 63) / 64, blocks = T * (T + 1) / 2;
  if (f16)
    hipLaunchKernelGGL((k_split<1, TS>), dim3((unsigned)blocks), dim3(256), 0, s, S, lds, n, (u16*)hi, (u16*)lo,
                       (u16*)hi_t, (u16*)lo_t, ldo, diag, unit, strict, scale);
  else
    hipLaunchKernelGGL((k_split<0, TS>), dim3((unsigned)blocks), dim3(256), 0, s, S, lds, n, (u16*)hi, (u16*)lo,
                       (u16*)hi_t, (u16*)lo_t, ldo, diag, unit, strict, scale);
  return hipGetLastError();
}

hipError_t launch_split(const double* S, int64_t lds, int64_t n, int f16, void* hi, void* lo, void* hi_t, void* lo_t,
                        int64_t ldo, double* diag, int unit, int strict, double scale, hipStream_t s) {
  return split_t<double>(S, lds, n, f16, hi, lo, hi_t, lo_t, ldo, diag, unit, strict, scale, s);
}

hipError_t launch_split_f32(const float* S, int64_t lds, int64_t n, int f16, void* hi_t, int64_t ldo, double scale,
                            hipStream_t s) {
  return split_t<float>(S, lds, n, f16, nullptr, nullptr, hi_t, nullptr, ldo, nullptr, 0, 0, scale, s);
}

// Zeros in a band of `band` columns next to the 64 x 64 tiles the split
// writes: for rows in 64-row strip q, columns [(q + 1) 64, (q + 1) 64 + band)
// (right = 1, row-major lower planes) or [q 64 - band, q 64) (right = 0,
// transposed planes), clipped to [0, ldo). One block per strip.
__global__ __launch_bounds__(256) void k_zero_band(u16* __restrict__ P, int64_t ldo, int64_t n, int64_t band,
                                                   int right) {
  const int64_t q = blockIdx.x;
  const int64_t c0 = right ? (q + 1) * 64 : q * 64 - band;
  const int64_t lo = c0 < 0 ? 0 : c0, hi = (c0 + band < ldo) ? c0 + band : ldo;
  if (hi <= lo) return;
  const int64_t w = hi - lo;
  for (int64_t r = 0; r < 64; ++r) {
    const int64_t i = q * 64 + r;
    if (i >= n) break;
    for (int64_t j = threadIdx.x; j < w; j += 256) P[i * ldo + lo + j] = 0;
  }
}

hipError_t launch_zero_band(void* P, int64_t ldo, int64_t n, int64_t band, int right, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_band, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, (u16*)P, ldo, n, band, right);
  return hipGetLastError();
}

}  // namespace trinv
