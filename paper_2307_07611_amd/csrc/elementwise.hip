// Small HBM-bound helpers: flag initialisation and deterministic FP64
// reductions (sums of squares for Frobenius norms).
#include "common.h"
#include "launch.h"

namespace trinv {

__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = (count + 255) / 256;
  TRINV_LAUNCH(k_fill_u64, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

// Block-wide sum of one double per thread (256 threads), fixed order.
__device__ __forceinline__ double block_sum_256(double v) {
  __shared__ double red[4];
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// One block per group of rows; partial[b] = sum of squares of its rows.
template <typename T>
__global__ __launch_bounds__(256) void k_sumsq(const T* A, int64_t n, int64_t lda, int lower, int unit,
                                               int64_t rows_per_block, double* partial) {
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = imin64(n, r0 + rows_per_block);
  double s = 0.0;
  for (int64_t i = r0; i < r1; ++i) {
    const int64_t jmax = lower ? i + 1 : n;
    for (int64_t j = threadIdx.x; j < jmax; j += 256) {
      double v = (double)A[i * lda + j];
      if (unit && j == i) v = 1.0;
      s += v * v;
    }
  }
  s = block_sum_256(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Block-wide maximum of one double per thread (256 threads).
__device__ __forceinline__ double block_max_256(double v) {
  __shared__ double red[4];
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return r;
}

template <typename T>
__global__ __launch_bounds__(256) void k_maxabs(const T* A, int64_t n, int64_t lda, int lower, int unit,
                                                int64_t rows_per_block, double* partial) {
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = imin64(n, r0 + rows_per_block);
  double m = 0.0;
  for (int64_t i = r0; i < r1; ++i) {
    const int64_t jmax = lower ? i + 1 : n;
    for (int64_t j = threadIdx.x; j < jmax; j += 256) {
      double v = fabs((double)A[i * lda + j]);
      if (unit && j == i) v = 1.0;
      m = fmax(m, v);
    }
  }
  m = block_max_256(m);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(256) void k_reduce_max(const double* partial, int64_t count, double* out) {
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) m = fmax(m, partial[i]);
  m = block_max_256(m);
  if (threadIdx.x == 0) out[0] = m;
}

template <typename T>
hipError_t launch_maxabs(const T* A, int64_t n, int64_t lda, int lower, int unit, double* partial, int64_t npartial,
                         double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t rpb = (n + npartial - 1) / npartial;
  const int64_t blocks = (n + rpb - 1) / rpb;
  TRINV_LAUNCH((k_maxabs<T>), dim3((unsigned)blocks), dim3(256), 0, s, A, n, lda, lower, unit, rpb, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  TRINV_LAUNCH(k_reduce_max, dim3(1), dim3(256), 0, s, partial, blocks, out);
  return hipGetLastError();
}
template hipError_t launch_maxabs<double>(const double*, int64_t, int64_t, int, int, double*, int64_t, double*,
                                          hipStream_t);
template hipError_t launch_maxabs<float>(const float*, int64_t, int64_t, int, int, double*, int64_t, double*,
                                         hipStream_t);

// Thread t adds entries t, t + 256, t + 512, ... in ascending order; the
// loads are issued 16 at a time so that their latencies overlap.
__global__ __launch_bounds__(256) void k_reduce_sum(const double* partial, int64_t count, double* out) {
  double s = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 15 * 256 < count; i += 16 * 256) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = partial[i + u * 256];
#pragma unroll
    for (int u = 0; u < 16; ++u) s += v[u];
  }
  for (; i < count; i += 256) s += partial[i];
  s = block_sum_256(s);
  if (threadIdx.x == 0) out[0] = s;
}

__global__ __launch_bounds__(256) void k_sumsq_vec(const double* v, int64_t count, double* out) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) s += v[i] * v[i];
  s = block_sum_256(s);
  if (threadIdx.x == 0) out[0] = s;
}

hipError_t launch_sumsq_vec(const double* v, int64_t count, double* out, hipStream_t s) {
  TRINV_LAUNCH(k_sumsq_vec, dim3(1), dim3(256), 0, s, v, count, out);
  return hipGetLastError();
}

hipError_t launch_reduce_sum(const double* partial, int64_t count, double* out, hipStream_t s) {
  TRINV_LAUNCH(k_reduce_sum, dim3(1), dim3(256), 0, s, partial, count, out);
  return hipGetLastError();
}

__global__ void k_zero_u32(uint32_t* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t count = (int64_t)(bytes / 4);
  if (count <= 0) return hipSuccess;
  const int64_t blocks = (count + 255) / 256;
  TRINV_LAUNCH(k_zero_u32, dim3((unsigned)(blocks < 16384 ? blocks : 16384)), dim3(256), 0, s, (uint32_t*)p,
                     count);
  return hipGetLastError();
}

// out[0] = min over blocks b of (b * m + words[b]) for words that are set
// (an all-ones word means no zero pivot in that block).
__global__ void k_fold_status(const uint64_t* words, int64_t count, int64_t m, uint64_t* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t v = ~0ull;
  for (int64_t b = 0; b < count; ++b)
    if (words[b] != ~0ull && (uint64_t)(b * m) + words[b] < v) v = (uint64_t)(b * m) + words[b];
  out[0] = v;
}

hipError_t launch_fold_status(const uint64_t* words, int64_t count, int64_t m, uint64_t* out, hipStream_t s) {
  TRINV_LAUNCH(k_fold_status, dim3(1), dim3(64), 0, s, words, count, m, out);
  return hipGetLastError();
}

// dst block b = alpha * src block b (m x m blocks at strides sstride / dstride).
template <typename T>
__global__ void k_block_copy(const T* src, int64_t lds, int64_t sstride, T* dst, int64_t ldd, int64_t dstride,
                             int64_t m, int64_t nblocks, T alpha) {
  const int64_t total = nblocks * m * m;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / (m * m), r = (e / m) % m, c = e % m;
    dst[b * dstride + r * ldd + c] = alpha * src[b * sstride + r * lds + c];
  }
}

template <typename T>
hipError_t launch_block_copy(const T* src, int64_t lds, int64_t sstride, T* dst, int64_t ldd, int64_t dstride,
                             int64_t m, int64_t nblocks, T alpha, hipStream_t s) {
  if (m <= 0 || nblocks <= 0) return hipSuccess;
  const int64_t total = nblocks * m * m, blocks = (total + 255) / 256;
  TRINV_LAUNCH((k_block_copy<T>), dim3((unsigned)(blocks < 16384 ? blocks : 16384)), dim3(256), 0, s, src, lds,
                     sstride, dst, ldd, dstride, m, nblocks, alpha);
  return hipGetLastError();
}
template hipError_t launch_block_copy<double>(const double*, int64_t, int64_t, double*, int64_t, int64_t, int64_t,
                                              int64_t, double, hipStream_t);
template hipError_t launch_block_copy<float>(const float*, int64_t, int64_t, float*, int64_t, int64_t, int64_t,
                                             int64_t, float, hipStream_t);

// A(i, i) = v for i < n (leading dimension ld).
template <typename T>
__global__ void k_set_diag(T* A, int64_t ld, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    A[i * ld + i] = v;
}

template <typename T>
hipError_t launch_set_diag(T* A, int64_t ld, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  TRINV_LAUNCH((k_set_diag<T>), dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, A, ld, n, v);
  return hipGetLastError();
}
template hipError_t launch_set_diag<double>(double*, int64_t, int64_t, double, hipStream_t);
template hipError_t launch_set_diag<float>(float*, int64_t, int64_t, float, hipStream_t);

// dst block b (m x m) = [[src block b (n x n), 0], [0, I]] (n <= m; src null:
// the identity), blocks at strides sstride / dstride.
template <typename T>
__global__ void k_embed(const T* src, int64_t lds, int64_t sstride, int64_t n, T* dst, int64_t ldd, int64_t dstride,
                        int64_t m, int64_t nblocks) {
  const int64_t total = nblocks * m * m;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / (m * m), r = (e / m) % m, c = e % m;
    T v = (r == c) ? T(1) : T(0);
    if (src && r < n && c < n) v = src[b * sstride + r * lds + c];
    dst[b * dstride + r * ldd + c] = v;
  }
}

template <typename T>
hipError_t launch_embed(const T* src, int64_t lds, int64_t sstride, int64_t n, T* dst, int64_t ldd, int64_t dstride,
                        int64_t m, int64_t nblocks, hipStream_t s) {
  if (m <= 0 || nblocks <= 0) return hipSuccess;
  if (n > m) return hipErrorInvalidValue;
  const int64_t total = nblocks * m * m, blocks = (total + 255) / 256;
  TRINV_LAUNCH((k_embed<T>), dim3((unsigned)(blocks < 16384 ? blocks : 16384)), dim3(256), 0, s, src, lds,
                     sstride, n, dst, ldd, dstride, m, nblocks);
  return hipGetLastError();
}
template hipError_t launch_embed<double>(const double*, int64_t, int64_t, int64_t, double*, int64_t, int64_t, int64_t,
                                         int64_t, hipStream_t);
template hipError_t launch_embed<float>(const float*, int64_t, int64_t, int64_t, float*, int64_t, int64_t, int64_t,
                                        int64_t, hipStream_t);

// dst (rows x cols, leading dimension ldd) = sum over c < count of the
// matrices src + c stride (leading dimension lds), summed in order of c.
template <typename T>
__global__ void k_sum_blocks(const T* __restrict__ src, int64_t lds, int64_t stride, int64_t count, int64_t rows,
                             int64_t cols, T* __restrict__ dst, int64_t ldd) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e % cols;
    T v = T(0);
    for (int64_t b = 0; b < count; ++b) v += src[b * stride + r * lds + c];
    dst[r * ldd + c] = v;
  }
}

template <typename T>
hipError_t launch_sum_blocks(const T* src, int64_t lds, int64_t stride, int64_t count, int64_t rows, int64_t cols,
                             T* dst, int64_t ldd, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int64_t total = rows * cols, blocks = (total + 255) / 256;
  TRINV_LAUNCH((k_sum_blocks<T>), dim3((unsigned)(blocks < 16384 ? blocks : 16384)), dim3(256), 0, s, src, lds,
                     stride, count, rows, cols, dst, ldd);
  return hipGetLastError();
}
template hipError_t launch_sum_blocks<double>(const double*, int64_t, int64_t, int64_t, int64_t, int64_t, double*,
                                              int64_t, hipStream_t);
template hipError_t launch_sum_blocks<float>(const float*, int64_t, int64_t, int64_t, int64_t, int64_t, float*,
                                             int64_t, hipStream_t);

__global__ void k_status_to_i32(const uint64_t* first_bad, int32_t* status, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    status[i] = first_bad[i] == ~0ull ? 0 : (int32_t)first_bad[i];
}

hipError_t launch_status_to_i32(const uint64_t* first_bad, int32_t* status, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = (count + 255) / 256;
  TRINV_LAUNCH(k_status_to_i32, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, s, first_bad,
                     status, count);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sumsq(const T* A, int64_t n, int64_t lda, int lower, int unit, double* partial, int64_t npartial,
                        double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t rpb = (n + npartial - 1) / npartial;
  const int64_t blocks = (n + rpb - 1) / rpb;
  TRINV_LAUNCH((k_sumsq<T>), dim3((unsigned)blocks), dim3(256), 0, s, A, n, lda, lower, unit, rpb, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_sum(partial, blocks, out, s);
}
template hipError_t launch_sumsq<double>(const double*, int64_t, int64_t, int, int, double*, int64_t, double*, hipStream_t);
template hipError_t launch_sumsq<float>(const float*, int64_t, int64_t, int, int, double*, int64_t, double*, hipStream_t);

// B = A^T through a 32 x 32 LDS tile (coalesced reads and writes).
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T* A, int64_t lda, T* B, int64_t ldb, int64_t n) {
  __shared__ T tile[32][33];
  const int64_t bi = (int64_t)blockIdx.y * 32, bj = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi + r, j = bj + tx;
    if (i < n && j < n) tile[r][tx] = A[i * lda + j];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bj + r, j = bi + tx;  // B(i, j) = A(j, i)
    if (i < n && j < n) B[i * ldb + j] = tile[tx][r];
  }
}

template <typename T>
hipError_t launch_transpose(const T* A, int64_t lda, T* B, int64_t ldb, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned g = (unsigned)((n + 31) / 32);
  TRINV_LAUNCH((k_transpose<T>), dim3(g, g), dim3(256), 0, s, A, lda, B, ldb, n);
  return hipGetLastError();
}
template hipError_t launch_transpose<double>(const double*, int64_t, double*, int64_t, int64_t, hipStream_t);
template hipError_t launch_transpose<float>(const float*, int64_t, float*, int64_t, int64_t, hipStream_t);

// A = A^T in place: one block per pair of mirrored 32 x 32 tiles (tile row
// it >= tile column jt), both staged in LDS before either is written.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose_inplace(T* A, int64_t lda, int64_t n) {
  __shared__ T t1[32][33];
  __shared__ T t2[32][33];
  const int64_t q = blockIdx.x;
  int64_t it = (int64_t)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
  while (it * (it + 1) / 2 > q) --it;
  while ((it + 1) * (it + 2) / 2 <= q) ++it;
  const int64_t jt = q - it * (it + 1) / 2;
  const int64_t bi = it * 32, bj = jt * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    if (bi + r < n && bj + tx < n) t1[r][tx] = A[(bi + r) * lda + bj + tx];
    if (it != jt && bj + r < n && bi + tx < n) t2[r][tx] = A[(bj + r) * lda + bi + tx];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    if (bj + r < n && bi + tx < n) A[(bj + r) * lda + bi + tx] = t1[tx][r];  // (bj + r, bi + tx) <- (bi + tx, bj + r)
    if (it != jt && bi + r < n && bj + tx < n) A[(bi + r) * lda + bj + tx] = t2[tx][r];
  }
}

template <typename T>
hipError_t launch_transpose_inplace(T* A, int64_t lda, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t t = (n + 31) / 32;
  TRINV_LAUNCH((k_transpose_inplace<T>), dim3((unsigned)(t * (t + 1) / 2)), dim3(256), 0, s, A, lda, n);
  return hipGetLastError();
}
template hipError_t launch_transpose_inplace<double>(double*, int64_t, int64_t, hipStream_t);
template hipError_t launch_transpose_inplace<float>(float*, int64_t, int64_t, hipStream_t);

// Dense offsets of a packed batch, off[i] = sum_{j < i} n_j^2 (orders
// outside 1..1024 count as 0): one workgroup, 256-element chunks, each an
// inclusive scan in LDS plus the running total.
__global__ __launch_bounds__(256) void k_dense_offsets(const int32_t* __restrict__ n, int64_t batch,
                                                       int64_t* __restrict__ off) {
  __shared__ int64_t part[256];
  const int t = threadIdx.x;
  int64_t carry = 0;
  for (int64_t base = 0; base < batch; base += 256) {
    const int64_t i = base + t;
    const int32_t ni = i < batch ? n[i] : 0;
    const int64_t v = (ni >= 1 && ni <= 1024) ? (int64_t)ni * ni : 0;
    part[t] = v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
      const int64_t add = t >= d ? part[t - d] : 0;
      __syncthreads();
      part[t] += add;
      __syncthreads();
    }
    if (i < batch) off[i] = carry + part[t] - v;
    carry += part[255];
    __syncthreads();
  }
}

hipError_t launch_dense_offsets(const int32_t* n_dev, int64_t batch, int64_t* off, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  TRINV_LAUNCH(k_dense_offsets, dim3(1), dim3(256), 0, s, n_dev, batch, off);
  return hipGetLastError();
}

// B_i = A_i^T for every matrix of a packed batch (order n_dev[i], A_i at
// offset offa[i], B_i at offb[i], leading dimension n_i): block (i, c) moves
// the 32 x 32 tiles c, c + gridDim.y, ... of matrix i through LDS. Matrices
// of an order outside 1..1024, or whose B range would end beyond capb
// elements, are skipped.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose_packed(const int32_t* __restrict__ n_dev,
                                                          const int64_t* __restrict__ offa, const T* __restrict__ A,
                                                          const int64_t* __restrict__ offb, T* __restrict__ B,
                                                          int64_t capb) {
  __shared__ T tile[32][33];
  const int64_t m = blockIdx.x;
  const int n = n_dev[m];
  if (n < 1 || n > 1024 || offb[m] + (int64_t)n * n > capb) return;
  const T* a = A + offa[m];
  T* b = B + offb[m];
  const int nt = (n + 31) / 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int q = blockIdx.y; q < nt * nt; q += gridDim.y) {
    const int bi = (q / nt) * 32, bj = (q % nt) * 32;
    for (int r = ty; r < 32; r += 8)
      if (bi + r < n && bj + tx < n) tile[r][tx] = a[(int64_t)(bi + r) * n + bj + tx];
    __syncthreads();
    for (int r = ty; r < 32; r += 8)
      if (bj + r < n && bi + tx < n) b[(int64_t)(bj + r) * n + bi + tx] = tile[tx][r];  // B(bj+r, bi+tx) = A(bi+tx, bj+r)
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_transpose_packed(int64_t batch, const int32_t* n_dev, const int64_t* offa, const T* A,
                                   const int64_t* offb, T* B, int64_t capb, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (batch > 0x7fffffff) return hipErrorInvalidValue;
  TRINV_LAUNCH((k_transpose_packed<T>), dim3((unsigned)batch, 8), dim3(256), 0, s, n_dev, offa, A, offb, B,
                     capb);
  return hipGetLastError();
}
template hipError_t launch_transpose_packed<double>(int64_t, const int32_t*, const int64_t*, const double*,
                                                    const int64_t*, double*, int64_t, hipStream_t);
template hipError_t launch_transpose_packed<float>(int64_t, const int32_t*, const int64_t*, const float*,
                                                   const int64_t*, float*, int64_t, hipStream_t);

// *flag |= 1 if the n x n matrix A holds a NaN or an infinity.
template <typename T>
__global__ __launch_bounds__(256) void k_nonfinite(const T* __restrict__ A, int64_t n, int64_t lda, int64_t rpb,
                                                   unsigned* flag) {
  const int64_t r0 = (int64_t)blockIdx.x * rpb, r1 = r0 + rpb < n ? r0 + rpb : n;
  bool bad = false;
  for (int64_t i = r0; i < r1; ++i)
    for (int64_t j = threadIdx.x; j < n; j += 256) bad |= !isfinite(A[i * lda + j]);
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(flag, 1u);
}

template <typename T>
hipError_t launch_nonfinite(const T* A, int64_t n, int64_t lda, unsigned* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t rpb = (n + 4095) / 4096;
  TRINV_LAUNCH((k_nonfinite<T>), dim3((unsigned)((n + rpb - 1) / rpb)), dim3(256), 0, s, A, n, lda, rpb, flag);
  return hipGetLastError();
}
template hipError_t launch_nonfinite<double>(const double*, int64_t, int64_t, unsigned*, hipStream_t);

// status[b] = -2 where status[b] == 0 and matrix b (n x n at b * stride)
// holds a NaN or an infinity; grid (row blocks, batch).
template <typename T>
__global__ __launch_bounds__(256) void k_nonfinite_status(const T* __restrict__ X, int64_t n, int64_t stride,
                                                          int64_t rpb, int32_t* status) {
  const T* A = X + (int64_t)blockIdx.y * stride;
  const int64_t r0 = (int64_t)blockIdx.x * rpb, r1 = r0 + rpb < n ? r0 + rpb : n;
  bool bad = false;
  for (int64_t i = r0; i < r1; ++i)
    for (int64_t j = threadIdx.x; j < n; j += 256) bad |= !isfinite(A[i * n + j]);
  if (__syncthreads_or(bad) && threadIdx.x == 0 && status[blockIdx.y] == 0) status[blockIdx.y] = -2;
}

template <typename T>
hipError_t launch_nonfinite_status(const T* X, int64_t n, int64_t stride, int64_t batch, int32_t* status,
                                   hipStream_t s) {
  if (n <= 0 || batch <= 0) return hipSuccess;
  const int64_t rpb = (n + 63) / 64;
  TRINV_LAUNCH((k_nonfinite_status<T>), dim3((unsigned)((n + rpb - 1) / rpb), (unsigned)batch), dim3(256), 0,
                     s, X, n, stride, rpb, status);
  return hipGetLastError();
}
template hipError_t launch_nonfinite_status<double>(const double*, int64_t, int64_t, int64_t, int32_t*, hipStream_t);
template hipError_t launch_nonfinite_status<float>(const float*, int64_t, int64_t, int64_t, int32_t*, hipStream_t);
template hipError_t launch_nonfinite<float>(const float*, int64_t, int64_t, unsigned*, hipStream_t);

}  // namespace trinv
