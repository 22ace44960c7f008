// Leaf inversion: the diagonal b x b blocks of L are inverted independently
// (one workgroup each) by the column recurrence CRIT (Section 4.2, algorithm
// CRIT, transposed to the lower case):
//     X(j,j) = 1 / L(j,j),
//     X(i,j) = -( sum_{k=j}^{i-1} L(i,k) X(k,j) ) / L(i,i),   i > j.
// Rows are produced in order i = 1, 2, ...; all columns j < i of row i are
// computed at once, one column per group of P lanes (P = 256 / b), the P
// lanes splitting the k-sum and combining it with cross-lane shuffles. L and
// X live in LDS in packed lower storage (row i at offset i(i+1)/2), so a
// 128 x 128 FP64 leaf needs 2 x 66 KB of the 160 KB LDS.
#include "common.h"
#include "launch.h"

namespace trinv {

template <typename T>
__device__ __forceinline__ T shfl_xor_t(T v, int mask) {
  return __shfl_xor(v, mask, 64);
}

// grid: (leaves per matrix, batch). Matrix `bz` starts at element bz*stride.
// Leaf l covers rows/cols [l*b, min(n, l*b + b)).
template <typename T, typename TL, int B>
__global__ __launch_bounds__(256) void k_leaf_inverse(int64_t n, const T* __restrict__ L, int64_t ldl,
                                                      T* __restrict__ X, int64_t ldx, int64_t stride,
                                                      int unit, TL* __restrict__ Xlp, TL* __restrict__ Xlpt,
                                                      int64_t ldxl, double lp_scale, int64_t* __restrict__ first_bad,
                                                      int per_matrix_status) {
  constexpr int P = 256 / B;  // lanes per column
  constexpr int PACK = B * (B + 1) / 2;
  __shared__ T Lp[PACK];
  __shared__ T Xp[PACK];

  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * B;
  const int bs = (int)imin64(B, n - r0);
  if (bs <= 0) return;
  const T* Lb = L + (int64_t)blockIdx.y * stride + r0 * ldl + r0;
  T* Xb = X + (int64_t)blockIdx.y * stride + r0 * ldx + r0;

  // Stage the lower triangle of the leaf in LDS (row-major reads, coalesced).
  for (int idx = tid; idx < bs * bs; idx += 256) {
    const int i = idx / bs, j = idx % bs;
    if (j <= i) Lp[i * (i + 1) / 2 + j] = Lb[(int64_t)i * ldl + j];
  }
  __syncthreads();

  // Diagonal: X(i,i) = 1 / L(i,i); report the first exact zero pivot.
  if (tid < bs) {
    const T d = Lp[tid * (tid + 1) / 2 + tid];
    if (!unit && d == (T)0 && first_bad)
      atomicMin((unsigned long long*)(first_bad + (per_matrix_status ? blockIdx.y : 0)),
                (unsigned long long)(r0 + tid + 1));
    Xp[tid * (tid + 1) / 2 + tid] = unit ? (T)1 : (T)1 / d;
  }
  __syncthreads();

  const int j = tid / P;  // column handled by this lane group
  const int p = tid % P;  // part of the k-sum
  for (int i = 1; i < bs; ++i) {
    const int ri = i * (i + 1) / 2;
    T s = (T)0;
    if (j < i) {
      // k runs over [j, i); lanes of a group take k = j+p, j+p+P, ...
      for (int k = j + p; k < i; k += P) s += Lp[ri + k] * Xp[k * (k + 1) / 2 + j];
    }
#pragma unroll
    for (int m = 1; m < P; m <<= 1) s += shfl_xor_t(s, m);
    if (j < i && p == 0) Xp[ri + j] = unit ? -s : -s / Lp[ri + i];
    __syncthreads();
  }

  // Write the full leaf block of X (zeros above the diagonal).
  for (int idx = tid; idx < bs * bs; idx += 256) {
    const int i = idx / bs, jj = idx % bs;
    const T v = (jj <= i) ? Xp[i * (i + 1) / 2 + jj] : (T)0;
    Xb[(int64_t)i * ldx + jj] = v;
    if (Xlp) Xlp[(int64_t)blockIdx.y * stride + (r0 + i) * ldxl + r0 + jj] = (TL)(float)((double)v * lp_scale);
  }
  // Transposed low-precision copy: element (i, jj) of the leaf at [jj][i],
  // written with consecutive threads along i (coalesced).
  if (Xlpt) {
    for (int idx = tid; idx < bs * bs; idx += 256) {
      const int jj = idx / bs, i = idx % bs;
      const T v = (jj <= i) ? Xp[i * (i + 1) / 2 + jj] : (T)0;
      Xlpt[(int64_t)blockIdx.y * stride + (r0 + jj) * ldxl + r0 + i] = (TL)(float)((double)v * lp_scale);
    }
  }
}

template <typename T, typename TL>
static hipError_t launch_leaf_t(int64_t n, const T* L, int64_t ldl, T* X, int64_t ldx, int64_t stride,
                                int64_t batch, int leaf, int unit, TL* Xlp, TL* Xlpt, int64_t ldxl, double lp_scale,
                                uint64_t* first_bad, int per_matrix_status, hipStream_t s) {
  const int64_t nleaves = (n + leaf - 1) / leaf;
  if (nleaves <= 0 || batch <= 0) return hipSuccess;
  dim3 grid((unsigned)nleaves, (unsigned)batch), block(256);
  int64_t* fb = (int64_t*)first_bad;
  switch (leaf) {
    case 16: hipLaunchKernelGGL((k_leaf_inverse<T, TL, 16>), grid, block, 0, s, n, L, ldl, X, ldx, stride, unit, Xlp, Xlpt, ldxl, lp_scale, fb, per_matrix_status); break;
    case 32: hipLaunchKernelGGL((k_leaf_inverse<T, TL, 32>), grid, block, 0, s, n, L, ldl, X, ldx, stride, unit, Xlp, Xlpt, ldxl, lp_scale, fb, per_matrix_status); break;
    case 64: hipLaunchKernelGGL((k_leaf_inverse<T, TL, 64>), grid, block, 0, s, n, L, ldl, X, ldx, stride, unit, Xlp, Xlpt, ldxl, lp_scale, fb, per_matrix_status); break;
    case 128: hipLaunchKernelGGL((k_leaf_inverse<T, TL, 128>), grid, block, 0, s, n, L, ldl, X, ldx, stride, unit, Xlp, Xlpt, ldxl, lp_scale, fb, per_matrix_status); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_leaf(int64_t n, const T* L, int64_t ldl, T* X, int64_t ldx, int64_t stride, int64_t batch,
                       int leaf, int unit, void* Xlp, void* Xlpt, int lp_is_f16, int64_t ldxl, double lp_scale,
                       uint64_t* first_bad, int per_matrix_status, hipStream_t s) {
  if (Xlp && lp_is_f16)
    return launch_leaf_t<T, _Float16>(n, L, ldl, X, ldx, stride, batch, leaf, unit, (_Float16*)Xlp, (_Float16*)Xlpt,
                                      ldxl, lp_scale, first_bad, per_matrix_status, s);
  return launch_leaf_t<T, __bf16>(n, L, ldl, X, ldx, stride, batch, leaf, unit, (__bf16*)Xlp, (__bf16*)Xlpt, ldxl,
                                  lp_scale, first_bad, per_matrix_status, s);
}

template hipError_t launch_leaf<double>(int64_t, const double*, int64_t, double*, int64_t, int64_t, int64_t, int,
                                        int, void*, void*, int, int64_t, double, uint64_t*, int, hipStream_t);
template hipError_t launch_leaf<float>(int64_t, const float*, int64_t, float*, int64_t, int64_t, int64_t, int, int,
                                       void*, void*, int, int64_t, double, uint64_t*, int, hipStream_t);

}  // namespace trinv
