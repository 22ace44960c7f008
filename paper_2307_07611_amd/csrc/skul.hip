// Diagonal-block step of the blocked form of algorithm SKUL (Section 5): the
// Crout factors A = L U (L lower triangular with general diagonal, U unit upper
// triangular, no pivoting) together with K = L^-1 and S = U^-1, all grown in
// one pass over the pivots as SKUL grows them beside the Crout loop.
#include "common.h"
#include "launch.h"

namespace trinv {

namespace {
constexpr int kMaxNb = 128;
constexpr int kLuStride = kMaxNb + 1;

// Pivots p = 16 P + q, q = 0 .. 15, of one phase. Thread (ty, tx) of a 16 x 16
// grid owns the elements (ty + 16 a, tx + 16 b), a, b = 0 .. 7, in registers;
// slot v[a][b] holds, for element (i, j) after step p:
//   i > p and j > p : the trailing entry of the right-looking elimination;
//   i > j, j <= p   : K(i, j) (the column of L has already been retired);
//   i <= p, j > i   : S(i, j) (the row of U has already been retired);
//   i == j <= p     : K(i, i) = 1 / L(i, i).
// Step p broadcasts column p (L(i, p) below the pivot, S(i, p) above it) and
// row p (U(p, j) W(p, p) to the right, K(p, j) W(p, p) to the left) through
// LDS, then every slot takes one rank-1 contribution:
//   i > p : v -= L(i, p) c_j, starting from 0 in column p (K(i, p) = -L(i, p) / L(p, p));
//   i = p : v = c_j (j <= p: row p of K is final) or -c_j (j > p: S(p, j) = -U(p, j));
//   i < p : v -= S(i, p) U(p, j) for j > p;
// with c_j = row_j / L(p, p). Slots with a < P and b < P are final in this
// phase and skipped at compile time. L(:, p) and U(p, :) are copied to the LDS
// array LU as they retire.
template <typename T, int P>
__device__ __forceinline__ void crout_phase(T (&v)[8][8], int nb, int tx, int ty, T* __restrict__ buf,
                                            T* __restrict__ LU, int64_t row0, uint64_t* bad) {
  for (int q = 0; q < 16; ++q) {
    const int p = 16 * P + q;
    if (p >= nb) return;
    T* colb = buf + (p & 1) * 2 * kMaxNb;
    T* rowb = colb + kMaxNb;
    if (tx == q) {
#pragma unroll
      for (int a = 0; a < 8; ++a) colb[ty + 16 * a] = v[a][P];
    }
    if (ty == q) {
#pragma unroll
      for (int b = 0; b < 8; ++b) rowb[tx + 16 * b] = (b == P && tx == q) ? T(1) : v[P][b];
    }
    __syncthreads();
    const T piv = colb[p];
    if (threadIdx.x == 0 && piv == T(0)) atomicMin((unsigned long long*)bad, (unsigned long long)(row0 + p + 1));
    const T inv = T(1) / piv;
    T r[8], c[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) r[a] = colb[ty + 16 * a];
#pragma unroll
    for (int b = 0; b < 8; ++b) c[b] = rowb[tx + 16 * b] * inv;
    if (tx == q) {
#pragma unroll
      for (int a = P; a < 8; ++a)
        if (a > P || ty >= q) LU[(ty + 16 * a) * kLuStride + p] = v[a][P];
    }
    if (ty == q) {
#pragma unroll
      for (int b = P; b < 8; ++b)
        if (b > P || tx > q) LU[p * kLuStride + tx + 16 * b] = c[b];
    }
#pragma unroll
    for (int a = 0; a < 8; ++a) {
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        if (a < P && b < P) continue;
        T& x = v[a][b];
        if (a > P) {
          if (b == P)
            x = (tx == q ? T(0) : x) - r[a] * c[b];
          else
            x -= r[a] * c[b];
        } else if (a < P) {
          if (b > P)
            x -= r[a] * c[b];
          else
            x -= (tx > q ? r[a] : T(0)) * c[b];
        } else {
          const bool jgt = b > P || (b == P && tx > q);
          const bool jeq = b == P && tx == q;
          const T lt = jgt ? x - r[a] * c[b] : x;
          const T eq = jgt ? -c[b] : c[b];
          const T gt = (jeq ? T(0) : x) - r[a] * c[b];
          x = ty < q ? lt : (ty == q ? eq : gt);
        }
      }
    }
  }
}
}  // namespace

// One workgroup of 256 threads per block (blockIdx.x selects the block of a
// strided batch) factors the block W[0:nb, 0:nb] (nb <= 128, leading
// dimension ldw) and writes: L (lower, diagonal included) and U (unit
// upper) of the block, zeros elsewhere, at leading dimension ld; K = L^-1
// (lower, zeros above) and S = U^-1 (unit upper, zeros below) at leading
// dimension ldk. The 1-based index row0 + p + 1 of the first zero pivot goes to
// *bad (atomic minimum); the factors are then not finite.
template <typename T>
__global__ __launch_bounds__(256) void k_crout_diag(const T* __restrict__ W, int64_t ldw, int64_t sw, int nb,
                                                    T* __restrict__ L, T* __restrict__ U, int64_t ld, int64_t slu,
                                                    T* __restrict__ K, T* __restrict__ S, int64_t ldk, int64_t sk,
                                                    int64_t row0, uint64_t* bad) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  W += blockIdx.x * sw;
  L += blockIdx.x * slu;
  U += blockIdx.x * slu;
  K += blockIdx.x * sk;
  S += blockIdx.x * sk;
  T* LU = (T*)smem;
  T* buf = LU + kMaxNb * kLuStride;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  T v[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int i = ty + 16 * a, j = tx + 16 * b;
      v[a][b] = (i < nb && j < nb) ? W[(int64_t)i * ldw + j] : T(0);
    }
  }
  crout_phase<T, 0>(v, nb, tx, ty, buf, LU, row0, bad);
  crout_phase<T, 1>(v, nb, tx, ty, buf, LU, row0, bad);
  crout_phase<T, 2>(v, nb, tx, ty, buf, LU, row0, bad);
  crout_phase<T, 3>(v, nb, tx, ty, buf, LU, row0, bad);
  crout_phase<T, 4>(v, nb, tx, ty, buf, LU, row0, bad);
  crout_phase<T, 5>(v, nb, tx, ty, buf, LU, row0, bad);
  crout_phase<T, 6>(v, nb, tx, ty, buf, LU, row0, bad);
  crout_phase<T, 7>(v, nb, tx, ty, buf, LU, row0, bad);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int i = ty + 16 * a, j = tx + 16 * b;
      if (i < nb && j < nb) {
        K[(int64_t)i * ldk + j] = i >= j ? v[a][b] : T(0);
        S[(int64_t)i * ldk + j] = i < j ? v[a][b] : (i == j ? T(1) : T(0));
      }
    }
  }
  __syncthreads();
  for (int r = ty; r < nb; r += 16) {
    for (int c = tx; c < nb; c += 16) {
      const T x = LU[r * kLuStride + c];
      L[(int64_t)r * ld + c] = c <= r ? x : T(0);
      U[(int64_t)r * ld + c] = c > r ? x : (c == r ? T(1) : T(0));
    }
  }
}

template <typename T>
hipError_t launch_crout_diag(const T* W, int64_t ldw, int64_t sw, int nb, T* L, T* U, int64_t ld, int64_t slu, T* K,
                             T* S, int64_t ldk, int64_t sk, int64_t count, int64_t row0, uint64_t* bad,
                             hipStream_t s) {
  if (nb <= 0 || count <= 0) return hipSuccess;
  if (count > 0x7fffffff) return hipErrorInvalidValue;
  if (nb > kMaxNb || ldk < nb) return hipErrorInvalidValue;
  const size_t lds = sizeof(T) * ((size_t)kMaxNb * kLuStride + 4 * kMaxNb);
  static bool attr_set = false;  // per instantiation
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_crout_diag<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  TRINV_LAUNCH(k_crout_diag<T>, dim3((unsigned)count), dim3(256), lds, s, W, ldw, sw, nb, L, U, ld, slu, K, S,
                     ldk, sk, row0, bad);
  return hipGetLastError();
}

template hipError_t launch_crout_diag<double>(const double*, int64_t, int64_t, int, double*, double*, int64_t, int64_t,
                                              double*, double*, int64_t, int64_t, int64_t, int64_t, uint64_t*,
                                              hipStream_t);
template hipError_t launch_crout_diag<float>(const float*, int64_t, int64_t, int, float*, float*, int64_t, int64_t,
                                             float*, float*, int64_t, int64_t, int64_t, int64_t, uint64_t*,
                                             hipStream_t);

}  // namespace trinv
