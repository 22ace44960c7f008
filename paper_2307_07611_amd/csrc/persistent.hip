// Batched inversion of many lower-triangular matrices of uneven order
// (1 <= n_i <= 1024) in one persistent launch.
//
// The two diagonal halves of every merge are independent (Section 4.1,
// algorithm COMBRIT with beta = 2), and so are different matrices: each
// workgroup takes whole matrices from a device-side queue, largest first, and
// inverts each one on its own CU, so a matrix stays in that XCD's L2.
//
// Per matrix, in one workgroup of 256 threads (4 waves):
//   1. leaves: 16 x 16 diagonal blocks by the column recurrence (algorithm
//      CRIT, Section 4.2, transposed to the lower case), 16 leaves at a
//      time, one thread per column, the leaf staged in LDS;
//   2. levels h = 16, 32, 64, ... < n, all merges of a level together:
//        T   =  C * A^-1   written straight into the X21 block of X,
//        X21 = -B^-1 * T   in place, one 32-row band at a time from the
//                          bottom: output band r reads only rows <= r of T,
//                          so the bands above it are still intact;
//      X12 is written as zeros. Every product runs on 16 x 16 x 4 MFMAs
//      (FP32 or FP64): blocks below 128 in 32 x 32 wave tiles whose fragments
//      are loaded from global memory one K chunk ahead, larger ones in
//      128 x 128 workgroup tiles staged through LDS. K ranges are cut to the
//      triangles (T: k >= first column; X21: k <= last row).
// A plan kernel first sorts the matrices by order (counting sort, largest
// first) and resets the queue, so the pair needs no memset and can be
// captured in a graph.
#include <limits.h>

#include <mutex>

#include "common.h"
#include "launch.h"

namespace trinv {

// Scratch of the allocation-free batched entry point: the plan (kNoAllocMaxBatch
// matrix indices) followed by the queue counter. Each device holds its own copy
// for the life of the process; host code reaches it only through the address
// batched_scratch() obtains per device.
static __device__ __align__(256) int32_t scratch[kNoAllocMaxBatch + 64];

hipError_t batched_scratch(int32_t** order, uint32_t** queue) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *order = (int32_t*)addr[dev];
  *queue = (uint32_t*)((int32_t*)addr[dev] + kNoAllocMaxBatch);
  return hipSuccess;
}

namespace {

constexpr int kThreads = 256;
constexpr int WT = 32;  // wave tile (rows and columns)
constexpr int KC = 16;  // K per register chunk (4 MFMA k-steps)
constexpr int kLeaf = 16;  // leaf order

template <typename T>
struct PMma;
template <>
struct PMma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of result register r within a 16 x 16 block (measured layout)
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct PMma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// One wave: D[r0:r0+32, c0:c0+32] = alpha * A[r0:, klo:khi] * B[klo:khi, c0:]
// for row-major A (lda), B (ldb), D (ldd); rows >= M and columns >= N are
// neither read nor written (their inputs are taken as zero), and k >= khi
// reads as zero. Lane l supplies A(l%16, k + l/16) and B(k + l/16, l%16) per
// 16 x 16 x 4 step.
template <typename T>
__device__ __forceinline__ void wave_tile(const T* A, int lda, const T* B, int ldb,
                                          T* D, int ldd, int M, int N, int r0, int c0, int klo,
                                          int khi, T alpha, int lane, bool& nf) {
  typedef typename PMma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  const int li = lane & 15, lk = lane >> 4;
  int ar[2], bc[2];
  bool aok[2], bok[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int r = r0 + 16 * b + li, c = c0 + 16 * b + li;
    aok[b] = r < M;
    bok[b] = c < N;
    ar[b] = aok[b] ? r : 0;
    bc[b] = bok[b] ? c : 0;
  }
  T fa[2][4][2], fb[2][4][2];  // [buffer][k step][block]
  auto load = [&](int buf, int k0) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * s + lk;
      const bool kok = k < khi;
      const int kc = kok ? k : klo;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const T va = A[ar[b] * lda + kc];
        const T vb = B[kc * ldb + bc[b]];
        fa[buf][s][b] = (kok && aok[b]) ? va : T(0);
        fb[buf][s][b] = (kok && bok[b]) ? vb : T(0);
      }
    }
  };
  if (klo < khi) {
    load(0, klo);
    int buf = 0;
    for (int k0 = klo; k0 < khi; k0 += KC) {
      if (k0 + KC < khi) load(buf ^ 1, k0 + KC);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = PMma<T>::op(fa[buf][s][i], fb[buf][s][j], acc[i][j]);
      buf ^= 1;
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = c0 + 16 * j + li;
      if (c >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + 16 * i + PMma<T>::row(lane, r);
        const T v = alpha * acc[i][j][r];
        if (row < M) D[row * ldd + c] = v;
        nf |= !__builtin_isfinite(v);
      }
    }
}

// Leaves of order B (the last one may be shorter): 256 / B leaves per pass,
// thread (leaf, column j) runs the column recurrence
//   X(j, j) = 1 / L(j, j),  X(i, j) = -(sum_{k=j}^{i-1} L(i, k) X(k, j)) / L(i, i)
// with the leaf's L in LDS and its column in registers, in right-looking
// order: once X(k, j) is final it is added into the running sums of the rows
// below (the same ascending-k summation as the formula, so the same rounding),
// which keeps one register per row. The whole leaf block of X is written,
// zeros above the diagonal included.
template <typename T, int B>
__device__ __forceinline__ void leaves(const T* __restrict__ L, T* __restrict__ X, int n, int unit, T* lds, int* bad,
                                       bool& nf) {
  constexpr int G = kThreads / B;
  constexpr int S = B + 1;  // LDS row stride
  const int tid = threadIdx.x;
  const int nl = (n + B - 1) / B;
  for (int g0 = 0; g0 < nl; g0 += G) {
#pragma unroll 4
    for (int e = tid; e < G * B * B; e += kThreads) {
      const int li = e / (B * B), i = (e / B) % B, j = e % B;
      const int l = g0 + li;
      const int gi = l * B + i, gj = l * B + j;
      T v = T(0);
      if (l < nl && gi < n && j <= i) v = (unit && i == j) ? T(1) : L[gi * n + gj];
      lds[(li * B + i) * S + j] = v;
    }
    __syncthreads();
    const int li = tid / B, j = tid % B, l = g0 + li;
    const int base = l * B;
    const int bl = (l < nl) ? min(B, n - base) : 0;
    if (j < bl) {
      const T* Ll = lds + li * B * S;
      if (Ll[j * S + j] == T(0)) atomicMin(bad, base + j + 1);
      T x[B];  // running sum of row i, then X(i, j)
#pragma unroll
      for (int i = 0; i < B; ++i) x[i] = T(0);
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const T num = (k == j) ? T(1) : -x[k];
        x[k] = (k < j) ? T(0) : (unit ? num : num / Ll[k * S + k]);
#pragma unroll
        for (int i = k + 1; i < B; ++i) x[i] += Ll[i * S + k] * x[k];
        __builtin_amdgcn_sched_barrier(0);  // keep each step's loads in that step
      }
      T* Xl = X + base * n + base + j;
#pragma unroll
      for (int i = 0; i < B; ++i)
        if (i < bl) {
          Xl[i * n] = x[i];
          nf |= !__builtin_isfinite(x[i]);
        }
    }
    __syncthreads();
  }
}

// One workgroup: D[r0:r0+128, c0:c0+128] = alpha * A[r0:, klo:khi] * B[klo:khi, c0:]
// (same conventions as wave_tile). K advances 16 at a time through two LDS
// buffers (A stored [m][k], B stored [k][n], padded rows), the next chunk's
// global loads (16 consecutive k of a row of A, 128 consecutive columns of a
// row of B: full cache lines) in flight while the current one is multiplied;
// each wave owns a 64 x 64 quarter (4 x 4 MFMA blocks). All threads of the
// workgroup must call it together.
constexpr int GT = 128;
constexpr int GSA = KC + 1, GSB = GT + 2;
constexpr int GBUF = GT * GSA + KC * GSB;  // elements of one stage

template <typename T>
__device__ __forceinline__ void wg_tile(const T* A, int lda, const T* B, int ldb, T* D, int ldd, int M, int N, int r0, int c0,
                        int klo, int khi, T alpha, T* lds, bool& nf) {
  typedef typename PMma<T>::acc_t acc_t;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  // this thread's staging elements: A rows ra + 16 i at k offset ka; B row
  // kb + 2 i at column cb
  const int ka = tid & 15, ra = tid >> 4;
  const int cb = tid & 127, kb = tid >> 7;
  T va[8], vb[8];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = r0 + ra + 16 * i, k = k0 + ka;
      const bool ok = r < M && k < khi;
      const T v = A[(r < M ? r : 0) * lda + (k < khi ? k : klo)];
      va[i] = ok ? v : T(0);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = k0 + kb + 2 * i, c = c0 + cb;
      const bool ok = c < N && k < khi;
      const T v = B[(k < khi ? k : klo) * ldb + (c < N ? c : 0)];
      vb[i] = ok ? v : T(0);
    }
  };
  auto sstore = [&](int buf) {
    T* As = lds + buf * GBUF;
    T* Bs = As + GT * GSA;
#pragma unroll
    for (int i = 0; i < 8; ++i) As[(ra + 16 * i) * GSA + ka] = va[i];
#pragma unroll
    for (int i = 0; i < 8; ++i) Bs[(kb + 2 * i) * GSB + cb] = vb[i];
  };
  const int li = lane & 15, lk = lane >> 4;
  if (klo < khi) {
    gload(klo);
    sstore(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = klo; k0 < khi; k0 += KC) {
      const bool more = k0 + KC < khi;
      if (more) gload(k0 + KC);
      const T* As = lds + buf * GBUF;
      const T* Bs = As + GT * GSA;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        T fa[4], fb[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          fa[b] = As[(wm * 64 + 16 * b + li) * GSA + 4 * s + lk];
          fb[b] = Bs[(4 * s + lk) * GSB + wn * 64 + 16 * b + li];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = PMma<T>::op(fa[i], fb[j], acc[i][j]);
      }
      if (more) sstore(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + wn * 64 + 16 * j + li;
      if (c >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + wm * 64 + 16 * i + PMma<T>::row(lane, r);
        const T v = alpha * acc[i][j][r];
        if (row < M) D[row * ldd + c] = v;
        nf |= !__builtin_isfinite(v);
      }
    }
}

// All off-diagonal products of one matrix (see the file comment). Levels with
// blocks of at least wg_from (128 or more; chosen by the autotuner) use
// workgroup tiles of 128 (one tile at a time, so the in-place product only has
// to take its bands bottom-up); smaller levels use independent 32 x 32 wave
// tiles. Step -1 of a level is T = C A^-1 over
// all merges; step s >= 0 is band (bands - 1 - s) of X21 = -B^-1 T of every
// merge. Each tile routine has a single call site (keeps register use low).
template <typename T>
__device__ __forceinline__ void levels(const T* __restrict__ L, T* X, int n, int b, int wg_from, T* lds, bool& nf) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: tile parameters stay scalar
  constexpr int NW = kThreads / 64;
  for (int h = b; h < n; h *= 2) {
    const int span = 2 * h;
    const int nmerge = (n - h + span - 1) / span;
    const int hb_last = min(h, n - (nmerge - 1) * span - h);
    // X12 = 0
    for (int m = 0; m < nmerge; ++m) {
      const int o = m * span, hb = (m == nmerge - 1) ? hb_last : h;
      for (int e = tid; e < h * hb; e += kThreads) {
        const int i = e / hb, j = e % hb;
        X[(o + i) * n + o + h + j] = T(0);
      }
    }
    const bool big = h >= wg_from;
    const int TT = big ? GT : WT;
    const int tc = (h + TT - 1) / TT;                           // column tiles of T / X21
    const int tr_full = tc, tr_last = (hb_last + TT - 1) / TT;  // row tiles (bands)
    for (int s = -1; s < tr_full; ++s) {
      const int per_full = (s < 0) ? tr_full * tc : tc;
      const int per_last = (s < 0) ? tr_last * tc : (s < tr_last ? tc : 0);
      const int tiles = (nmerge - 1) * per_full + per_last;
      for (int t = big ? 0 : wave; t < tiles; t += big ? 1 : NW) {
        const int m = min(t / per_full, nmerge - 1);
        const int q = t - m * per_full;
        const int o = m * span, hb = (m == nmerge - 1) ? hb_last : h;
        T* D = X + (o + h) * n + o;  // T, then X21
        const T* A;
        const T* Bm;
        int r0, c0, klo, khi;
        T alpha;
        if (s < 0) {  // T = C * A^-1: k >= first column of the tile
          A = L + (o + h) * n + o;
          Bm = X + o * n + o;
          r0 = (q / tc) * TT;
          c0 = (q % tc) * TT;
          klo = c0;
          khi = h;
          alpha = T(1);
        } else {  // X21 = -B^-1 * T: k <= last row of the band
          const int rb = ((m == nmerge - 1) ? tr_last : tr_full) - 1 - s;
          A = X + (o + h) * n + o + h;
          Bm = D;
          r0 = rb * TT;
          c0 = q * TT;
          klo = 0;
          khi = min(hb, r0 + TT);
          alpha = T(-1);
        }
        if (big)
          wg_tile<T>(A, n, Bm, n, D, n, hb, h, r0, c0, klo, khi, alpha, lds, nf);
        else
          wave_tile<T>(A, n, Bm, n, D, n, hb, h, r0, c0, klo, khi, alpha, lane, nf);
      }
      __syncthreads();
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_batched(int64_t batch, const int32_t* __restrict__ n_dev,
                                                      const int64_t* __restrict__ off_dev, const T* __restrict__ L,
                                                      T* __restrict__ X, int32_t* __restrict__ status,
                                                      const int32_t* __restrict__ order, uint32_t* queue, int unit,
                                                      int wg_from) {
  // the leaf stage (256 / B leaves of B x (B + 1) elements) or the two
  // staging buffers of the workgroup tiles
  __shared__ T lds[kThreads * 33 > 2 * GBUF ? kThreads * 33 : 2 * GBUF];
  __shared__ int s_item, s_bad;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) {
      s_item = (int)atomicAdd(queue, 1u);
      s_bad = INT_MAX;
    }
    __syncthreads();
    // uniform across the workgroup: keep the matrix's scalars in SGPRs
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item >= batch) break;
    const int m = __builtin_amdgcn_readfirstlane(order[item]);
    const int n = __builtin_amdgcn_readfirstlane(n_dev[m]);
    const int64_t off = off_dev[m];
    const int64_t offu = ((int64_t)__builtin_amdgcn_readfirstlane((int)(off >> 32)) << 32) |
                         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)off);
    bool nf = false;  // a NaN or an infinity stored into this matrix's X (and its T blocks)
    if (n >= 1 && n <= 1024) {
      const T* Lm = L + offu;
      T* Xm = X + offu;
      leaves<T, kLeaf>(Lm, Xm, n, unit, lds, &s_bad, nf);
      levels<T>(Lm, Xm, n, kLeaf, wg_from, lds, nf);
    }
    nf = __syncthreads_or(nf);
    if (tid == 0) status[m] = (n < 1 || n > 1024) ? -1 : (s_bad != INT_MAX ? s_bad : (nf ? -2 : 0));
    __syncthreads();
  }
}

// Counting sort of the matrices by order, largest first (1024 bins, one per
// thread: thread t holds order 1024 - t), and queue reset.
__global__ __launch_bounds__(1024) void k_batched_plan(int64_t batch, const int32_t* __restrict__ n_dev,
                                                       int32_t* __restrict__ order, uint32_t* queue) {
  __shared__ int cnt[1024];
  __shared__ int wsum[16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  cnt[t] = 0;
  __syncthreads();
  auto bin = [](int v) { return 1024 - min(max(v, 1), 1024); };  // order v -> slot, descending
  for (int64_t i = t; i < batch; i += 1024) atomicAdd(&cnt[bin(n_dev[i])], 1);
  __syncthreads();
  // exclusive prefix sum over the 1024 slots
  const int c = cnt[t];
  int v = c;
#pragma unroll
  for (int d = 1; d < 64; d *= 2) {
    const int u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  if (lane == 63) wsum[w] = v;
  __syncthreads();
  int before = 0;
  for (int k = 0; k < w; ++k) before += wsum[k];
  const int start = before + v - c;
  __syncthreads();
  cnt[t] = start;
  __syncthreads();
  for (int64_t i = t; i < batch; i += 1024) {
    const int p = atomicAdd(&cnt[bin(n_dev[i])], 1);
    order[p] = (int32_t)i;
  }
  if (t == 0) *queue = 0u;
}

}  // namespace

template <typename T>
hipError_t launch_batched(int64_t batch, const int32_t* n_dev, const int64_t* off_dev, const T* L, T* X,
                          int32_t* status, int32_t* order, uint32_t* queue, int unit, int grid, int wg_from,
                          hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (wg_from < GT || grid < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_batched_plan, dim3(1), dim3(1024), 0, s, batch, n_dev, order, queue);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batched<T>, dim3((unsigned)grid), dim3(kThreads), 0, s, batch, n_dev, off_dev, L, X, status,
                     order, queue, unit, wg_from);
  return hipGetLastError();
}

template <typename T>
int batched_occupancy(int* cus_out) {
  static int per_cu = -1, cus = 0;
  if (per_cu < 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batched<T>, kThreads, 0) != hipSuccess || occ < 1) occ = 1;
    per_cu = occ;
  }
  if (cus_out) *cus_out = cus;
  return per_cu;
}

template <typename T>
int batched_grid(int64_t batch, int per_cu) {
  int cus = 0;
  const int occ = batched_occupancy<T>(&cus);
  const int k = (per_cu >= 1 && per_cu <= occ) ? per_cu : occ;
  const int64_t g = (int64_t)cus * k;
  return (int)(batch < g ? batch : g);
}

template hipError_t launch_batched<float>(int64_t, const int32_t*, const int64_t*, const float*, float*, int32_t*,
                                          int32_t*, uint32_t*, int, int, int, hipStream_t);
template hipError_t launch_batched<double>(int64_t, const int32_t*, const int64_t*, const double*, double*, int32_t*,
                                           int32_t*, uint32_t*, int, int, int, hipStream_t);
template int batched_occupancy<float>(int*);
template int batched_occupancy<double>(int*);
template int batched_grid<float>(int64_t, int);
template int batched_grid<double>(int64_t, int);

}  // namespace trinv
