// Panel step of the blocked form of algorithm SQR (Section 5): modified
// Gram-Schmidt over up to 16 (or 8) consecutive columns of the working matrix V,
// column by column as the algorithm orthogonalizes them.
#include "common.h"
#include "launch.h"

namespace trinv {

namespace {
constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
}  // namespace

// Panel width for order n: 16 columns while a thread holds one row, 8 beyond
// (a wave of a 1024-thread workgroup has 128 VGPRs).
int mgs_panel_width(int64_t n) { return n <= kThreads ? 16 : 8; }

// One workgroup of 1024 threads holds the panel V[:, p0 : p0 + w] (w <= PW)
// in registers, thread t owning rows t + 1024 i (i < RPT, n <= 1024 RPT). For
// column j of the panel, in order:
//   d_c = v_j . v_c (c >= j, one block reduction for all of them),
//   R(j, j) = sqrt(d_j), q_j = v_j / R(j, j),
//   R(j, c) = d_c / R(j, j) = q_j . v_c and v_c -= R(j, c) q_j (c > j),
// which is the projection sequence of modified Gram-Schmidt (each later
// column loses its q_j component while q_j is formed). Writes Q[:, p0 : p0 + w]
// and R[p0 : p0 + w, p0 : p0 + w] (upper part; the lower part is not
// touched). A zero R(j, j) sends p0 + j + 1 to *bad (atomic minimum).
template <typename T, int RPT, int kPw>
__global__ __launch_bounds__(kThreads) void k_mgs_panel(const T* __restrict__ V, T* __restrict__ Q,
                                                        T* __restrict__ R, int64_t ld, int64_t n, int64_t p0, int w,
                                                        uint64_t* bad) {
  __shared__ double part[kWaves][16];
  __shared__ double tot[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  T v[RPT][kPw];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int64_t r = tid + (int64_t)kThreads * i;
#pragma unroll
    for (int c = 0; c < kPw; ++c) v[i][c] = (r < n && c < w) ? V[r * ld + p0 + c] : T(0);
  }
  static_for<0, kPw>([&](auto J) {
    constexpr int j = decltype(J)::value;
    if (j >= w) return;
    double d[kPw];
#pragma unroll
    for (int c = j; c < kPw; ++c) {
      double a = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) a += (double)v[i][j] * (double)v[i][c];
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) a += __shfl_xor(a, m, 64);
      d[c] = a;
    }
    if (lane == 0) {
#pragma unroll
      for (int c = j; c < kPw; ++c) part[wave][c] = d[c];
    }
    __syncthreads();
    if (wave == 0) {  // lane l sums waves 4 (l / 16) .. + 3 of column l % 16
      const int c = lane & 15, g = lane >> 4;
      double a = 0.0;
      if (c >= j && c < kPw) {
#pragma unroll
        for (int q = 0; q < 4; ++q) a += part[4 * g + q][c];
      }
      a += __shfl_xor(a, 16, 64);
      a += __shfl_xor(a, 32, 64);
      if (lane < 16) tot[lane] = a;
    }
    __syncthreads();
    const double nrm = sqrt(tot[j]);
    if (tid == 0 && nrm == 0.0) atomicMin((unsigned long long*)bad, (unsigned long long)(p0 + j + 1));
    const double inv = 1.0 / nrm;
#pragma unroll
    for (int i = 0; i < RPT; ++i) v[i][j] = (T)((double)v[i][j] * inv);
#pragma unroll
    for (int c = j + 1; c < kPw; ++c) {
      const T rjc = (T)(tot[c] * inv);
#pragma unroll
      for (int i = 0; i < RPT; ++i) v[i][c] -= rjc * v[i][j];
    }
    if (tid < w && tid >= j) R[(p0 + j) * ld + p0 + tid] = (T)(tid == j ? nrm : tot[tid] * inv);
    // the next column's partial sums go to `part` only after every wave has
    // read `tot` of this one (the barrier of the next reduction orders it)
  });
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int64_t r = tid + (int64_t)kThreads * i;
    if (r < n) {
#pragma unroll
      for (int c = 0; c < kPw; ++c)
        if (c < w) Q[r * ld + p0 + c] = v[i][c];
    }
  }
}

template <typename T>
hipError_t launch_mgs_panel(const T* V, T* Q, T* R, int64_t ld, int64_t n, int64_t p0, int w, uint64_t* bad,
                            hipStream_t s) {
  if (w <= 0) return hipSuccess;
  if (w > mgs_panel_width(n) || n > 4 * kThreads || p0 + w > n) return hipErrorInvalidValue;
  if (n <= kThreads)
    TRINV_LAUNCH((k_mgs_panel<T, 1, 16>), dim3(1), dim3(kThreads), 0, s, V, Q, R, ld, n, p0, w, bad);
  else if (n <= 2 * kThreads)
    TRINV_LAUNCH((k_mgs_panel<T, 2, 8>), dim3(1), dim3(kThreads), 0, s, V, Q, R, ld, n, p0, w, bad);
  else
    TRINV_LAUNCH((k_mgs_panel<T, 4, 8>), dim3(1), dim3(kThreads), 0, s, V, Q, R, ld, n, p0, w, bad);
  return hipGetLastError();
}

template hipError_t launch_mgs_panel<double>(const double*, double*, double*, int64_t, int64_t, int64_t, int, uint64_t*,
                                             hipStream_t);
template hipError_t launch_mgs_panel<float>(const float*, float*, float*, int64_t, int64_t, int64_t, int, uint64_t*,
                                            hipStream_t);

}  // namespace trinv
