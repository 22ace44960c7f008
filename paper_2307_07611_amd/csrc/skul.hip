// Diagonal-block step of the blocked Crout factorization of algorithm SKUL
// (Section 5): A = L U with L lower triangular (general diagonal) and U unit
// upper triangular, no pivoting.
#include "common.h"
#include "launch.h"

namespace trinv {

namespace {
constexpr int kMaxNb = 128;
}

// One workgroup factors the block W[0:nb, 0:nb] (order nb <= 128, leading
// dimension ldw) in LDS, right-looking, pivot by pivot:
//   U(p, j) = W(p, j) / W(p, p) (j > p),   W(i, j) -= W(i, p) U(p, j) (i, j > p),
// which gives the same factors as the row-by-row recurrence of SKUL. Writes
// the block's L (lower, diagonal included) and U (unit upper) with zeros
// elsewhere; the 1-based index row0 + p + 1 of the first zero pivot goes to
// *bad (atomic minimum).
template <typename T>
__global__ __launch_bounds__(256) void k_crout_diag(const T* __restrict__ W, int64_t ldw, int nb, T* __restrict__ L,
                                                    T* __restrict__ U, int64_t ld, int64_t row0, uint64_t* bad) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  T* B = (T*)smem;
  const int S = nb + 1;  // LDS row stride
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) B[(e / nb) * S + e % nb] = W[(int64_t)(e / nb) * ldw + e % nb];
  __syncthreads();
  for (int p = 0; p < nb; ++p) {
    const T piv = B[p * S + p];
    if (tid == 0 && piv == T(0)) atomicMin((unsigned long long*)bad, (unsigned long long)(row0 + p + 1));
    for (int j = p + 1 + tid; j < nb; j += 256) B[p * S + j] = B[p * S + j] / piv;
    __syncthreads();
    const int m = nb - p - 1;
    for (int e = tid; e < m * m; e += 256) {
      const int i = p + 1 + e / m, j = p + 1 + e % m;
      B[i * S + j] -= B[i * S + p] * B[p * S + j];
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) {
    const int r = e / nb, c = e % nb;
    const T v = B[r * S + c];
    L[(int64_t)r * ld + c] = (c <= r) ? v : T(0);
    U[(int64_t)r * ld + c] = (c > r) ? v : (c == r ? T(1) : T(0));
  }
}

template <typename T>
hipError_t launch_crout_diag(const T* W, int64_t ldw, int nb, T* L, T* U, int64_t ld, int64_t row0, uint64_t* bad,
                             hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  if (nb > kMaxNb) return hipErrorInvalidValue;
  const size_t lds = sizeof(T) * (size_t)nb * (nb + 1);
  static bool attr_set = false;  // per instantiation
  if (!attr_set) {
    const int maxb = (int)(sizeof(T) * kMaxNb * (kMaxNb + 1));
    hipError_t e = hipFuncSetAttribute((const void*)k_crout_diag<T>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_crout_diag<T>, dim3(1), dim3(256), lds, s, W, ldw, nb, L, U, ld, row0, bad);
  return hipGetLastError();
}

template hipError_t launch_crout_diag<double>(const double*, int64_t, int, double*, double*, int64_t, int64_t,
                                              uint64_t*, hipStream_t);
template hipError_t launch_crout_diag<float>(const float*, int64_t, int, float*, float*, int64_t, int64_t, uint64_t*,
                                             hipStream_t);

}  // namespace trinv
