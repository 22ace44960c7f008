// Leaf inversion: the diagonal b x b blocks of L are inverted independently
// (one workgroup each) by the column recurrence CRIT (Section 4.2, algorithm
// CRIT, transposed to the lower case):
//     X(j,j) = 1 / L(j,j),
//     X(i,j) = -( sum_{k=j}^{i-1} L(i,k) X(k,j) ) / L(i,i),   i > j.
// X is held in registers and built right-looking, one pivot row at a time
// (see k_leaf_inverse); L^T of the leaf sits in LDS (a 128 x 128 FP64 leaf
// takes 130 KB of the 160 KB).
#include "common.h"
#include "launch.h"

namespace trinv {

// grid: (leaves per matrix, batch). Matrix `bz` starts at element bz*stride.
// Leaf l covers rows/cols [l*b, min(n, l*b + b)).
//
// Thread (ty, tx) of a 16 x 16 grid owns the elements (ty + 16 a, tx + 16 c),
// a, c < B / 16, of the leaf's X in registers; column p of L is read from an
// LDS copy of L^T. Pivot p = 16 P + q, in order:
//   the owners of row p divide it by L(p, p): X(p, :) final, broadcast through
//   LDS (double buffered, one barrier per pivot);
//   every row i > p takes X(i, :) -= L(i, p) X(p, :).
// Starting from X = I this gives X(i, j) = -(sum_{k=j}^{i-1} L(i, k) X(k, j))
// / L(i, i), the sums taken in ascending k, as the column recurrence forms them.
template <typename T, int B, int P>
__device__ __forceinline__ void leaf_phase(T (&v)[B / 16][B / 16], int bs, int tx, int ty, const T* __restrict__ Lt,
                                           T* __restrict__ rowb, int unit, int64_t r0, int64_t* first_bad) {
  constexpr int NS = B / 16, LS = B + 1;
  for (int q = 0; q < 16; ++q) {
    const int p = 16 * P + q;
    if (p >= bs) return;
    T* rb = rowb + (p & 1) * B;
    if (ty == q) {
      const T d = unit ? T(1) : Lt[p * LS + p];
#pragma unroll
      for (int c = 0; c <= P; ++c) {
        if (tx + 16 * c <= p) v[P][c] = v[P][c] / d;  // right of the diagonal stays an exact 0
        rb[tx + 16 * c] = v[P][c];
      }
      if (tx == q && !unit && d == T(0) && first_bad)
        atomicMin((unsigned long long*)first_bad, (unsigned long long)(r0 + p + 1));
    }
    __syncthreads();
    T l[NS], x[NS];
#pragma unroll
    for (int a = P; a < NS; ++a) l[a] = Lt[p * LS + ty + 16 * a];
#pragma unroll
    for (int c = 0; c <= P; ++c) x[c] = rb[tx + 16 * c];
#pragma unroll
    for (int a = P; a < NS; ++a) {
      const bool below = a > P || ty > q;
#pragma unroll
      for (int c = 0; c <= P; ++c) v[a][c] = below ? v[a][c] - l[a] * x[c] : v[a][c];
    }
  }
}

template <typename T, typename TL, int B>
__global__ __launch_bounds__(256) void k_leaf_inverse(int64_t n, const T* __restrict__ L, int64_t ldl,
                                                      T* __restrict__ X, int64_t ldx, int64_t stride,
                                                      int unit, TL* __restrict__ Xlp, TL* __restrict__ Xlpt,
                                                      int64_t ldxl, double lp_scale, int64_t* __restrict__ first_bad,
                                                      int per_matrix_status, int round_x, int zero_wgs) {
  constexpr int NS = B / 16, LS = B + 1;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  T* Lt = (T*)smem;           // L^T of the leaf: Lt[k * LS + i] = L(i, k), zero outside
  T* rowb = Lt + B * LS;      // two broadcast rows
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  if (zero_wgs > 0 && (int)blockIdx.x >= (int)gridDim.x - zero_wgs) {
    // The last zero_wgs workgroups write the zeros of X above the leaf blocks
    // (row i, columns from the next leaf boundary to n - 1), rows w,
    // w + zero_wgs, ...; they run on the CUs the leaves leave idle.
    const int w = (int)blockIdx.x - ((int)gridDim.x - zero_wgs);
    T* Xm = X + (int64_t)blockIdx.y * stride;
    // FP64 rows start 16-byte aligned (B is even) when X is and ldx is even:
    // 16-byte stores, the odd last element alone
    const bool pairs = sizeof(T) == 8 && ((((uintptr_t)Xm) | (uintptr_t)(ldx * 8)) & 15) == 0;
    for (int64_t i = w; i < n; i += zero_wgs) {
      T* row = Xm + i * ldx;
      const int64_t c0 = (i / B + 1) * B;
      if (pairs) {
        typedef T t2 __attribute__((ext_vector_type(2)));
        for (int64_t c = c0 + 2 * tid; c + 1 < n; c += 512) __builtin_nontemporal_store((t2){(T)0, (T)0}, (t2*)(row + c));
        if (tid == 0 && c0 < n && ((n - c0) & 1)) row[n - 1] = (T)0;
      } else {
        for (int64_t c = c0 + tid; c < n; c += 256) row[c] = (T)0;
      }
    }
    return;
  }
  const int64_t r0 = (int64_t)blockIdx.x * B;
  const int bs = (int)imin64(B, n - r0);
  if (bs <= 0) return;
  const T* Lb = L + (int64_t)blockIdx.y * stride + r0 * ldl + r0;
  T* Xb = X + (int64_t)blockIdx.y * stride + r0 * ldx + r0;
  int64_t* fb = first_bad ? first_bad + (per_matrix_status ? blockIdx.y : 0) : nullptr;

  // Stage L^T (row-major reads, coalesced); the strict upper part of L is not read.
  for (int idx = tid; idx < B * B; idx += 256) {
    const int i = idx / B, k = idx % B;
    Lt[k * LS + i] = (i < bs && k <= i) ? Lb[(int64_t)i * ldl + k] : T(0);
  }
  T v[NS][NS];
#pragma unroll
  for (int a = 0; a < NS; ++a)
#pragma unroll
    for (int c = 0; c < NS; ++c) v[a][c] = (ty + 16 * a == tx + 16 * c) ? T(1) : T(0);
  __syncthreads();
  leaf_phase<T, B, 0>(v, bs, tx, ty, Lt, rowb, unit, r0, fb);
  if constexpr (NS > 1) leaf_phase<T, B, 1>(v, bs, tx, ty, Lt, rowb, unit, r0, fb);
  if constexpr (NS > 2) {
    leaf_phase<T, B, 2>(v, bs, tx, ty, Lt, rowb, unit, r0, fb);
    leaf_phase<T, B, 3>(v, bs, tx, ty, Lt, rowb, unit, r0, fb);
  }
  if constexpr (NS > 4) {
    leaf_phase<T, B, 4>(v, bs, tx, ty, Lt, rowb, unit, r0, fb);
    leaf_phase<T, B, 5>(v, bs, tx, ty, Lt, rowb, unit, r0, fb);
    leaf_phase<T, B, 6>(v, bs, tx, ty, Lt, rowb, unit, r0, fb);
    leaf_phase<T, B, 7>(v, bs, tx, ty, Lt, rowb, unit, r0, fb);
  }

  // Write the full leaf block of X (exact zeros above the diagonal) and the
  // optional row-major low-precision copy. round_x: the off-diagonal entries
  // of X are stored as the copy's values (divided by lp_scale), the diagonal
  // as computed.
#pragma unroll
  for (int a = 0; a < NS; ++a)
#pragma unroll
    for (int c = 0; c < NS; ++c) {
      const int i = ty + 16 * a, jj = tx + 16 * c;
      if (i < bs && jj < bs) {
        const TL lp = (TL)(float)((double)v[a][c] * lp_scale);
        Xb[(int64_t)i * ldx + jj] = (round_x && i != jj) ? (T)((double)(float)lp / lp_scale) : v[a][c];
        if (Xlp) Xlp[(int64_t)blockIdx.y * stride + (r0 + i) * ldxl + r0 + jj] = lp;
      }
    }
  // Transposed low-precision copy, staged through LDS so that consecutive
  // threads write consecutive elements.
  if (Xlpt) {
    __syncthreads();  // every wave is done with Lt
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
      for (int c = 0; c < NS; ++c) Lt[(tx + 16 * c) * LS + ty + 16 * a] = v[a][c];
    __syncthreads();
    for (int idx = tid; idx < bs * bs; idx += 256) {
      const int jj = idx / bs, i = idx % bs;
      Xlpt[(int64_t)blockIdx.y * stride + (r0 + jj) * ldxl + r0 + i] = (TL)(float)((double)Lt[jj * LS + i] * lp_scale);
    }
  }
}

template <typename T, typename TL, int B>
static hipError_t go_leaf(dim3 grid, hipStream_t s, int64_t n, const T* L, int64_t ldl, T* X, int64_t ldx,
                          int64_t stride, int unit, TL* Xlp, TL* Xlpt, int64_t ldxl, double lp_scale, int64_t* fb,
                          int per_matrix_status, int round_x, int zero_wgs) {
  const size_t lds = sizeof(T) * ((size_t)B * (B + 1) + 2 * B);
  auto k = k_leaf_inverse<T, TL, B>;
  static bool attr_set = false;  // per instantiation
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  TRINV_LAUNCH(k, grid, dim3(256), lds, s, n, L, ldl, X, ldx, stride, unit, Xlp, Xlpt, ldxl, lp_scale, fb,
               per_matrix_status, round_x, zero_wgs);
  return hipGetLastError();
}

template <typename T, typename TL>
static hipError_t launch_leaf_t(int64_t n, const T* L, int64_t ldl, T* X, int64_t ldx, int64_t stride,
                                int64_t batch, int leaf, int unit, TL* Xlp, TL* Xlpt, int64_t ldxl, double lp_scale,
                                uint64_t* first_bad, int per_matrix_status, int round_x, int zero_upper,
                                hipStream_t s) {
  const int64_t nleaves = (n + leaf - 1) / leaf;
  if (nleaves <= 0 || batch <= 0) return hipSuccess;
  // zero_upper: extra workgroups zero X above the leaf blocks, on the CUs the
  // leaves leave idle and then on those they free (one workgroup per CU)
  const int zw = (zero_upper && nleaves > 1) ? (int)(nleaves >= 256 ? 128 : 512 - nleaves) : 0;
  dim3 grid((unsigned)(nleaves + zw), (unsigned)batch);
  int64_t* fb = (int64_t*)first_bad;
  switch (leaf) {
    case 16: return go_leaf<T, TL, 16>(grid, s, n, L, ldl, X, ldx, stride, unit, Xlp, Xlpt, ldxl, lp_scale, fb, per_matrix_status, round_x, zw);
    case 32: return go_leaf<T, TL, 32>(grid, s, n, L, ldl, X, ldx, stride, unit, Xlp, Xlpt, ldxl, lp_scale, fb, per_matrix_status, round_x, zw);
    case 64: return go_leaf<T, TL, 64>(grid, s, n, L, ldl, X, ldx, stride, unit, Xlp, Xlpt, ldxl, lp_scale, fb, per_matrix_status, round_x, zw);
    case 128: return go_leaf<T, TL, 128>(grid, s, n, L, ldl, X, ldx, stride, unit, Xlp, Xlpt, ldxl, lp_scale, fb, per_matrix_status, round_x, zw);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_leaf(int64_t n, const T* L, int64_t ldl, T* X, int64_t ldx, int64_t stride, int64_t batch,
                       int leaf, int unit, void* Xlp, void* Xlpt, int lp_is_f16, int64_t ldxl, double lp_scale,
                       uint64_t* first_bad, int per_matrix_status, hipStream_t s, int round_x, int zero_upper) {
  if (round_x && !Xlp) return hipErrorInvalidValue;
  if (Xlp && lp_is_f16)
    return launch_leaf_t<T, _Float16>(n, L, ldl, X, ldx, stride, batch, leaf, unit, (_Float16*)Xlp, (_Float16*)Xlpt,
                                      ldxl, lp_scale, first_bad, per_matrix_status, round_x, zero_upper, s);
  return launch_leaf_t<T, __bf16>(n, L, ldl, X, ldx, stride, batch, leaf, unit, (__bf16*)Xlp, (__bf16*)Xlpt, ldxl,
                                  lp_scale, first_bad, per_matrix_status, round_x, zero_upper, s);
}

template hipError_t launch_leaf<double>(int64_t, const double*, int64_t, double*, int64_t, int64_t, int64_t, int,
                                        int, void*, void*, int, int64_t, double, uint64_t*, int, hipStream_t, int,
                                        int);
template hipError_t launch_leaf<float>(int64_t, const float*, int64_t, float*, int64_t, int64_t, int64_t, int, int,
                                       void*, void*, int, int64_t, double, uint64_t*, int, hipStream_t, int, int);

}  // namespace trinv
