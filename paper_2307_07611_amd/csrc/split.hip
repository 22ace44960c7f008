// Staging casts of the mixed-precision path: a lower-triangular FP64 (or FP32)
// matrix, times a power-of-two scale s, is cut into low-precision slices
// hi = round(s v) and lo = round(s v - hi) (round-to-nearest-even in BF16 or
// FP16; s v and s v - hi are exact in FP64), written row-major and/or
// transposed, in the row-major or the panel-blocked plane layout (through a
// 64 x 64 LDS tile, so every store is a run of consecutive elements), plus the
// unscaled FP64 diagonal. HBM-bound: one read of the lower triangle, 2 bytes
// written per requested slice and element.
#include "common.h"
#include "lowp.h"

namespace trinv {

namespace {
typedef unsigned short u16;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

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

// 8 consecutive elements of one row of an LDS tile, or of one column (t = 1).
__device__ __forceinline__ u32x4 pack8(const u16 (*t)[66], int r, int c, int transposed) {
  u16 v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = transposed ? t[c + e][r] : t[r][c + e];
  u32x4 o;
#pragma unroll
  for (int e = 0; e < 4; ++e) o[e] = (unsigned)v[2 * e] | ((unsigned)v[2 * e + 1] << 16);
  return o;
}
}  // namespace

// Grid: one block per 64 x 64 tile of the lower triangle (tile row it >= tile col jt).
template <int F16, typename TS>
__global__ __launch_bounds__(256) void k_split(const TS* __restrict__ S, int64_t lds, int64_t n, SplitOut o,
                                               double* __restrict__ diag, int unit, int strict, double scale) {
  __shared__ u16 th[64][66];
  __shared__ u16 tl[64][66];
  __shared__ double red[2][4];
  const int64_t q = blockIdx.x;
  int64_t it = (int64_t)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
  while (it * (it + 1) / 2 > q) --it;
  while ((it + 1) * (it + 2) / 2 <= q) ++it;
  const int64_t jt = q - it * (it + 1) / 2;
  const int64_t i0 = it * 64, j0 = jt * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  double sq = 0.0, dsq = 0.0;
  for (int r = ty; r < 64; r += 4) {
    const int64_t i = i0 + r, j = j0 + tx;
    u16 h = 0, l = 0;
    if (i < n && j < n) {
      double v = (j <= i) ? (double)S[i * lds + j] : 0.0;
      if (unit && i == j) v = 1.0;
      sq += v * v;
      dsq += (i == j) ? v * v : 0.0;
      if (i == j && diag) diag[i] = v;
      if (strict && i == j) v = 0.0;  // slices of the strictly lower part
      v *= scale;
      double hb;
      h = lp_bits<F16>(v, &hb);
      double lb;
      l = lp_bits<F16>(v - hb, &lb);
      if (o.hi) o.hi[i * o.ldo + j] = h;
      if (o.lo) o.lo[i * o.ldo + j] = l;
    }
    th[r][tx] = h;
    tl[r][tx] = l;
  }
  if (o.sq) {  // uniform: this tile's sums of squares (fixed order)
    for (int m = 32; m >= 1; m >>= 1) {
      sq += __shfl_xor(sq, m, 64);
      dsq += __shfl_xor(dsq, m, 64);
    }
    if (tx == 0) {
      red[0][ty] = sq;
      red[1][ty] = dsq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      o.sq[q] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
      o.dsq[q] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
  }
  const bool rm_t = o.hi_t || o.lo_t;
  const bool pb = o.hi_b || o.lo_b || o.hi_tb || o.lo_tb;
  if (!rm_t && !pb) return;
  __syncthreads();
  if (rm_t) {
    for (int r = ty; r < 64; r += 4) {
      const int64_t c = j0 + r, rr = i0 + tx;  // transposed element (c, rr) = S(rr, c)
      if (c < n && rr < n) {
        if (o.hi_t) o.hi_t[c * o.ldo + rr] = th[tx][r];
        if (o.lo_t) o.lo_t[c * o.ldo + rr] = tl[tx][r];
      }
    }
  }
  if (pb) {
    // 16-byte chunks: 64 rows x 8 chunks per output; chunk (r, c) holds
    // elements c .. c + 7 of row r of the (possibly transposed) tile.
    for (int e = threadIdx.x; e < 512; e += 256) {
      const int r = e >> 3, c = (e & 7) * 8;
      const int64_t gi = i0 + r, gk = j0 + c;  // A role: row of S, k = column of S
      if (gi < n) {
        if (o.hi_b) *(u32x4*)(o.hi_b + pb_index(gi, gk, o.kb)) = pack8(th, r, c, 0);
        if (o.lo_b) *(u32x4*)(o.lo_b + pb_index(gi, gk, o.kb)) = pack8(tl, r, c, 0);
      }
      const int64_t gr = j0 + r, gc = i0 + c;  // B role: row = column of S, k = row of S
      if (gr < n) {
        if (o.hi_tb) *(u32x4*)(o.hi_tb + pb_index(gr, gc, o.kb)) = pack8(th, r, c, 1);
        if (o.lo_tb) *(u32x4*)(o.lo_tb + pb_index(gr, gc, o.kb)) = pack8(tl, r, c, 1);
      }
    }
  }
}

template <typename TS>
static hipError_t split_t(const TS* S, int64_t lds, int64_t n, int f16, const SplitOut& o, double* diag, int unit,
                          int strict, double scale, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (o.sq && !o.dsq) return hipErrorInvalidValue;
  const int64_t blocks = split_tiles(n);
  if (f16)
    TRINV_LAUNCH((k_split<1, TS>), dim3((unsigned)blocks), dim3(256), 0, s, S, lds, n, o, diag, unit, strict,
                       scale);
  else
    TRINV_LAUNCH((k_split<0, TS>), dim3((unsigned)blocks), dim3(256), 0, s, S, lds, n, o, diag, unit, strict,
                       scale);
  return hipGetLastError();
}

hipError_t launch_split(const double* S, int64_t lds, int64_t n, int f16, const SplitOut& o, double* diag, int unit,
                        int strict, double scale, hipStream_t s) {
  return split_t<double>(S, lds, n, f16, o, diag, unit, strict, scale, s);
}

hipError_t launch_split_f32(const float* S, int64_t lds, int64_t n, int f16, const SplitOut& o, double scale,
                            hipStream_t s) {
  return split_t<float>(S, lds, n, f16, o, nullptr, 0, 0, scale, s);
}

// Zeros in a band of `band` columns (a multiple of 8) beside the 64 x 64
// tiles the split writes, in up to 8 panel-blocked planes at once
// (blockIdx.y selects the plane): for rows in 64-row strip q, columns
// [(q + 1) 64, (q + 1) 64 + band) (right = 1, planes holding a lower triangle)
// or [q 64 - band, q 64) (right = 0, transposed planes), clipped to
// [0, 16 kb). One block per strip and plane, 16-byte stores.
struct BandPlanes {
  u16* p[8];
  int right[8];
};

__global__ __launch_bounds__(256) void k_zero_band_pb(BandPlanes bp, int64_t kb, int64_t n, int64_t band) {
  const int64_t q = blockIdx.x;
  u16* P = bp.p[blockIdx.y];
  const int right = bp.right[blockIdx.y];
  const int64_t c0 = right ? (q + 1) * 64 : q * 64 - band;
  const int64_t lo = c0 < 0 ? 0 : c0, hi = (c0 + band < 16 * kb) ? c0 + band : 16 * kb;
  if (hi <= lo) return;
  const int64_t chunks = (hi - lo) / 8;
  for (int64_t e = threadIdx.x; e < 64 * chunks; e += 256) {
    const int64_t i = q * 64 + e / chunks, k = lo + 8 * (e % chunks);
    if (i < n) *(u32x4*)(P + pb_index(i, k, kb)) = u32x4{0u, 0u, 0u, 0u};
  }
}

hipError_t launch_zero_band_pb(void* const* planes, const int* right, int count, int64_t kb, int64_t n, int64_t band,
                               hipStream_t s) {
  if (n <= 0 || count <= 0) return hipSuccess;
  if (count > 8) return hipErrorInvalidValue;
  BandPlanes bp{};
  for (int i = 0; i < count; ++i) {
    bp.p[i] = (u16*)planes[i];
    bp.right[i] = right[i];
  }
  TRINV_LAUNCH(k_zero_band_pb, dim3((unsigned)((n + 63) / 64), (unsigned)count), dim3(256), 0, s, bp, kb, n,
                     band);
  return hipGetLastError();
}

}  // namespace trinv
