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
__device__ __forceinline__ double lp_value(u16 bits) {
  return F16 ? (double)__builtin_bit_cast(_Float16, bits) : (double)(float)__builtin_bit_cast(__bf16, bits);
}

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
// SRC 0: one element of S per load; SRC 2: two consecutive elements of S
// per load (S aligned to two elements, lds even); LPSRC (SRC 1): the
// strictly lower values are read from a row-major low-precision copy
// (value = copy / scale, exactly, for a power-of-two scale) and only the
// diagonal from S.
template <int F16, typename TS, int SRC>
__global__ __launch_bounds__(256) void k_split(const TS* __restrict__ S, int64_t lds, int64_t n, SplitOut o,
                                               double* __restrict__ diag, int unit, int strict, double scale,
                                               const u16* __restrict__ lp, int64_t ldlp) {
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
  constexpr int LPSRC = SRC == 1;
  const double inv = LPSRC ? 1.0 / scale : 1.0;
  double sq = 0.0, dsq = 0.0;
  if constexpr (LPSRC) {
    // Strictly lower values: the copy over scale (a power of two: multiplying
    // by inv divides exactly), so scale v is the copy itself: hi = its bits,
    // lo = 0. The FP64 diagonal enters the norms and diag only (strict
    // slices). Two 16-byte loads per thread: row e / 8 of the tile, columns
    // 8 (e % 8) .. + 7, e = tid, tid + 256 (the copy's rows are padded to at
    // least n + 8 elements, so a chunk starting below n stays in its row).
    u32x4 raw[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = (int)threadIdx.x + 256 * u, r = e >> 3, c = (e & 7) * 8;
      const int64_t i = i0 + r;
      raw[u] = (i < n && j0 + c < n) ? *(const u32x4*)(lp + i * ldlp + j0 + c) : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = (int)threadIdx.x + 256 * u, r = e >> 3, c = (e & 7) * 8;
      const int64_t i = i0 + r;
      unsigned packed[4];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int64_t j = j0 + c + t;
        const bool low = i < n && j < i;
        const u16 bits = low ? (u16)(raw[u][t >> 1] >> (16 * (t & 1))) : (u16)0;
        const bool dg = i < n && j == i;
        const double v = low ? lp_value<F16>(bits) * inv : (dg ? (double)S[i * lds + i] : 0.0);
        sq += v * v;
        dsq += dg ? v * v : 0.0;
        if (dg && diag) diag[i] = v;
        if (t & 1)
          packed[t >> 1] |= (unsigned)bits << 16;
        else
          packed[t >> 1] = bits;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) *(unsigned*)&th[r][c + 2 * t] = packed[t];
    }
  } else if constexpr (SRC == 2) {
    // Eight loads of two consecutive elements per thread, issued together:
    // row e / 32 of the tile, columns 2 (e % 32) and + 1, e = tid + 256 u
    // (a pair reaching column n is loaded as its first element alone).
    typedef TS ts2 __attribute__((ext_vector_type(2)));
    ts2 raw[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = (int)threadIdx.x + 256 * u, r = e >> 5, c = (e & 31) * 2;
      const int64_t i = i0 + r, j = j0 + c;
      if (i < n && j + 1 < n) {
        raw[u] = *(const ts2*)(S + i * lds + j);
      } else {
        raw[u][0] = (i < n && j < n) ? S[i * lds + j] : (TS)0;
        raw[u][1] = (TS)0;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = (int)threadIdx.x + 256 * u, r = e >> 5, c = (e & 31) * 2;
      const int64_t i = i0 + r;
      u16 h[2] = {0, 0}, l[2] = {0, 0};
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int64_t j = j0 + c + t;
        if (i < n && j < n) {
          double v = (j <= i) ? (double)raw[u][t] : 0.0;
          if (unit && i == j) v = 1.0;
          sq += v * v;
          dsq += (i == j) ? v * v : 0.0;
          if (i == j && diag) diag[i] = v;
          if (strict && i == j) v = 0.0;  // slices of the strictly lower part
          v *= scale;
          double hb;
          h[t] = lp_bits<F16>(v, &hb);
          double lb;
          l[t] = lp_bits<F16>(v - hb, &lb);
        }
      }
      const int64_t j = j0 + c;
      if (i < n && j < n) {
        if (o.hi) {
          u16* d = o.hi + i * o.ldo + j;
          if (j + 1 < n && (((uintptr_t)d) & 3) == 0) {
            *(unsigned*)d = (unsigned)h[0] | ((unsigned)h[1] << 16);
          } else {
            d[0] = h[0];
            if (j + 1 < n) d[1] = h[1];
          }
        }
        if (o.lo) {
          u16* d = o.lo + i * o.ldo + j;
          if (j + 1 < n && (((uintptr_t)d) & 3) == 0) {
            *(unsigned*)d = (unsigned)l[0] | ((unsigned)l[1] << 16);
          } else {
            d[0] = l[0];
            if (j + 1 < n) d[1] = l[1];
          }
        }
      }
      *(unsigned*)&th[r][c] = (unsigned)h[0] | ((unsigned)h[1] << 16);
      *(unsigned*)&tl[r][c] = (unsigned)l[0] | ((unsigned)l[1] << 16);
    }
  } else {
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

template <typename TS, int SRC>
static hipError_t split_t(const TS* S, int64_t lds, int64_t n, int f16, const SplitOut& o, double* diag, int unit,
                          int strict, double scale, const u16* lp, int64_t ldlp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (o.sq && !o.dsq) return hipErrorInvalidValue;
  const int64_t blocks = split_tiles(n);
  if (f16)
    TRINV_LAUNCH((k_split<1, TS, SRC>), dim3((unsigned)blocks), dim3(256), 0, s, S, lds, n, o, diag, unit,
                 strict, scale, lp, ldlp);
  else
    TRINV_LAUNCH((k_split<0, TS, SRC>), dim3((unsigned)blocks), dim3(256), 0, s, S, lds, n, o, diag, unit,
                 strict, scale, lp, ldlp);
  return hipGetLastError();
}

// Pairs of elements per load where S is aligned to two elements and lds is even.
template <typename TS>
static hipError_t split_any(const TS* S, int64_t lds, int64_t n, int f16, const SplitOut& o, double* diag, int unit,
                            int strict, double scale, hipStream_t s) {
  if ((((uintptr_t)S) % (2 * sizeof(TS))) == 0 && lds % 2 == 0)
    return split_t<TS, 2>(S, lds, n, f16, o, diag, unit, strict, scale, nullptr, 0, s);
  return split_t<TS, 0>(S, lds, n, f16, o, diag, unit, strict, scale, nullptr, 0, s);
}

hipError_t launch_split(const double* S, int64_t lds, int64_t n, int f16, const SplitOut& o, double* diag, int unit,
                        int strict, double scale, hipStream_t s) {
  return split_any<double>(S, lds, n, f16, o, diag, unit, strict, scale, s);
}

hipError_t launch_split_lp_source(const double* S, int64_t lds, const void* lp, int64_t ldlp, int64_t n, int f16,
                                  const SplitOut& o, double* diag, double scale, hipStream_t s) {
  int e = 0;
  if (!lp || ldlp < n || !(scale > 0.0) || std::frexp(scale, &e) != 0.5) return hipErrorInvalidValue;
  if (o.hi || o.lo || o.lo_b || o.lo_tb || o.hi_t || o.lo_t) return hipErrorInvalidValue;  // hi slices only
  if ((((uintptr_t)lp) & 15) != 0 || ldlp % 8 != 0 || ldlp < n + 8) return hipErrorInvalidValue;  // 16-byte rows
  return split_t<double, 1>(S, lds, n, f16, o, diag, 0, 1, scale, (const u16*)lp, ldlp, s);
}

hipError_t launch_split_f32(const float* S, int64_t lds, int64_t n, int f16, const SplitOut& o, double scale,
                            hipStream_t s) {
  return split_any<float>(S, lds, n, f16, o, nullptr, 0, 0, scale, s);
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
