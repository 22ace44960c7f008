// Batched inversion of many lower-triangular matrices of uneven order
// (1 <= n_i <= 1024) in one persistent launch.
//
// The two diagonal halves of every merge are independent (Section 4.1,
// algorithm COMBRIT with beta = 2), and so are different matrices: each
// workgroup takes whole matrices from a device-side queue, largest first, and
// inverts each one on its own CU.
//
// Per matrix, in one workgroup of 256 threads (4 waves):
//   1. leaves: the diagonal blocks of order LEAF (32 or 64, the recursion's
//      cut-off, chosen by the autotuner) by the column recurrence (algorithm
//      CRIT, Section 4.2, transposed to the lower case): each lane owns one
//      column of a leaf in registers and reads the leaf's L^T from LDS;
//      every wave inverts 64 / LEAF leaves at a time;
//   2. levels h = LEAF, 2 LEAF, ... < n, each in two steps over all merges of
//      the level:
//        T   =  C * A^-1   written straight into the X21 block of X,
//        X21 = -B^-1 * T   in place, bands of output rows from the bottom
//                          up: a band reads only the rows of T at or above
//                          it, which the bands below it do not write;
//      then X12 is written as zeros. The products run on 16 x 16 x 4 MFMAs
//      (FP32 or FP64) in TM x TM workgroup tiles (TM = min(h, tmax), tmax 64 or
//      128 chosen by the autotuner; each wave
//      owns a TM/2 x TM/2 quarter), K cut to the triangles (T: k >= first
//      column of the tile; X21: k < end of the band). All tiles of one step
//      form one stream of K stages through a four-stage LDS ring filled by
//      direct global -> LDS loads three stages ahead, across tile
//      boundaries, so the loads of the next tile overlap the products of the
//      current one (no tile of a step reads what an earlier tile of the same
//      step writes). A stage that reaches past the end of the K range is
//      filled by bounds-checked loads instead (zeros beyond K).
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

template <typename T>
struct BMma;
template <>
struct BMma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of result register r within a 16 x 16 block (measured layout)
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct BMma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// The LDS ring of the tile products: NS stages, each holding an A tile
// [TM rows][KC] (a 64-byte row piece per row: four 16-byte chunks, chunk c of
// row r at position c ^ ((r >> 2) & 3)) followed by a B tile [KC rows][TM]
// (row k in 16-byte chunks, chunk c at position c ^ swzb(k)). The stage size is
// that of the largest tile (TM = 128) whatever TM a step uses.
template <typename T>
struct Ring {
  static constexpr int KC = 64 / sizeof(T);  // K per stage
  static constexpr int KS = KC / 4;           // MFMA k steps per stage (lane group g holds k = g KS + s)
  static constexpr int EPC = 16 / sizeof(T);  // elements per 16-byte chunk (= KS)
  static constexpr int NS = 4;
  static constexpr int STAGE = 2 * 128 * 64;  // bytes
  static constexpr int BYTES = NS * STAGE;
  static_assert(EPC == KS, "a lane's chunk holds its k values of one stage");
};

// Position of B-tile chunk c in row k: FP32 rows of one lane group and the
// next one are read in the same half wave, so their chunks are moved 64 bytes
// apart (16 banks).
template <typename T>
__device__ __forceinline__ int swzb(int k) {
  return sizeof(T) == 4 ? ((k / Ring<T>::KS) & 1) * 4 : 0;
}

// One output tile of a product step: D[r0 : r0 + TM, c0 : c0 + TM] (rows < M
// stored) = alpha * A[r0 :, klo : khi] * B[klo : khi, c0 :], all row-major
// with element (i, j) at base[i * ld + j].
template <typename T>
struct TileDesc {
  const T* A;
  const T* B;
  T* D;
  const T* safe;  // the matrix's first element: a 16-byte load there stays inside it
  int ld;  // the matrix order: every operand lives in L or X of one matrix
  int M, r0, c0, klo, khi;
  T alpha;
};

// The tiles of the two product steps of level h: `kind` 0 is T = C A^-1
// (merge-major), 1 is X21 = -B^-1 T (bands from the bottom up, then merges).
template <typename T>
struct LevelTiles {
  const T* L;
  T* X;
  int n, h, nmerge, hb_last, TM;
  int kind;
  __device__ int count() const {
    const int R = h / TM, C = h / TM, rl = (hb_last + TM - 1) / TM;
    return ((nmerge - 1) * R + rl) * C;
  }
  __device__ TileDesc<T> operator()(int t) const {
    const int R = h / TM, C = h / TM, rl = (hb_last + TM - 1) / TM;
    int m, bi, bj;
    if (kind == 0) {
      m = t / (R * C);
      if (m > nmerge - 1) m = nmerge - 1;
      const int q = t - m * R * C;
      bi = q / C;
      bj = q % C;
    } else {
      // bands R-1 .. rl hold the full merges only, bands rl-1 .. 0 all merges
      const int A = (nmerge - 1) * C, B = nmerge * C;
      const int head = (R - rl) * A;
      int q;
      if (t < head) {
        bi = R - 1 - t / A;
        q = t % A;
      } else {
        bi = rl - 1 - (t - head) / B;
        q = (t - head) % B;
      }
      m = q / C;
      bj = q % C;
    }
    const int o = m * 2 * h, hb = (m == nmerge - 1) ? hb_last : h;
    TileDesc<T> d;
    d.safe = X;
    d.ld = n;
    d.M = hb;
    d.r0 = bi * TM;
    d.c0 = bj * TM;
    d.D = X + (o + h) * n + o;  // T, then X21
    if (kind == 0) {
      d.A = L + (o + h) * n + o;  // C
      d.B = X + o * n + o;        // A^-1
      d.klo = d.c0;               // A^-1(k, j) = 0 for k < j
      d.khi = h;
      d.alpha = T(1);
    } else {
      d.A = X + (o + h) * n + o + h;  // B^-1
      d.B = d.D;                      // T
      d.klo = 0;
      d.khi = min(hb, d.r0 + TM);  // B^-1(i, k) = 0 for k > i
      d.alpha = T(-1);
    }
    return d;
  }
};

// Waits until at most VM of this wave's vector memory operations are
// outstanding and for all its LDS operations, then a workgroup barrier (no
// memory fence: direct loads of later stages stay in flight across it).
template <int VM>
__device__ __forceinline__ void wait_barrier() {
  static_assert(VM >= 0 && VM < 64, "vmcnt range");
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt((VM & 15) | ((VM >> 4) << 14) | (7 << 4));
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Every memory operation of the workgroup complete and visible to all of its
// waves.
__device__ __forceinline__ void drain() {
  wait_barrier<0>();
  __syncthreads();
}

// All tiles of one product step as one stream of K stages (see the file
// comment). Every thread of the workgroup calls it with the same arguments.
// Returns whether this thread stored a NaN or an infinity.
template <typename T, int TM>
__device__ __forceinline__ bool run_step(const LevelTiles<T>& tiles, char* ring) {
  typedef Ring<T> R;
  typedef typename BMma<T>::acc_t acc_t;
  constexpr int KC = R::KC, KS = R::KS, EPC = R::EPC, NS = R::NS;
  constexpr int BI = TM / 32;             // 16 x 16 blocks per wave and dimension
  constexpr int LPS = TM / 32;            // direct loads per thread and stage
  constexpr int NA = TM / 16;             // 1 KB load blocks of the A tile (and of the B tile)
  constexpr int CPRB = TM * (int)sizeof(T) / 16;  // chunks per B-tile row
  constexpr int BOFF = TM * 64;           // byte offset of the B tile in a stage
  typedef __attribute__((address_space(3))) char lds_char;
  typedef T vec_t __attribute__((ext_vector_type(KS)));
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int ntiles = tiles.count();
  bool nf = false;
  if (ntiles <= 0) return nf;
  auto nstages = [&](const TileDesc<T>& d) { return (d.khi - d.klo + KC - 1) / KC; };
  // consume cursor: tile tc, its stage sc
  int tc = 0, sc = 0;
  TileDesc<T> dc = tiles(0);
  int nsc = nstages(dc);

  // Stage k0 of tile d into ring slot `slot` by direct loads (an edge stage
  // loads the matrix's first 16 bytes into every chunk: its data is replaced
  // before use, and it keeps the count of loads per stage).
  auto issue = [&](int slot, const TileDesc<T>& d, int k0) {
    const bool edge = k0 + KC > d.khi;
    lds_char* st = (lds_char*)ring + slot * R::STAGE;
#pragma unroll
    for (int i = 0; i < LPS; ++i) {
      const int b = wave + 4 * i;
      const T* src;
      lds_char* dst;
      if (b < NA) {
        const int p = b * 64 + lane, row = p >> 2, c = (p & 3) ^ ((row >> 2) & 3);
        const int gr = min(d.r0 + row, d.M - 1);
        src = d.A + gr * d.ld + k0 + c * EPC;
        dst = st + b * 1024;
      } else {
        const int p = (b - NA) * 64 + lane, krow = p / CPRB, c = (p % CPRB) ^ swzb<T>(krow);
        src = d.B + (k0 + krow) * d.ld + d.c0 + c * EPC;
        dst = st + BOFF + (b - NA) * 1024;
      }
      if (edge) src = d.safe;
      __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    }
  };
  // Bounds-checked fill of a stage that reaches past khi (zeros beyond it).
  auto guarded_fill = [&](int slot, const TileDesc<T>& d, int k0) {
    char* st = ring + slot * R::STAGE;
    for (int e = tid; e < TM * KC; e += kThreads) {
      const int row = e / KC, k = e % KC;
      const int gr = min(d.r0 + row, d.M - 1);
      const T v = (k0 + k < d.khi) ? d.A[gr * d.ld + k0 + k] : T(0);
      *(T*)(st + (row * 4 + ((k / EPC) ^ ((row >> 2) & 3))) * 16 + (k % EPC) * (int)sizeof(T)) = v;
    }
    for (int e = tid; e < KC * TM; e += kThreads) {
      const int krow = e / TM, col = e % TM;
      const T v = (k0 + krow < d.khi) ? d.B[(k0 + krow) * d.ld + d.c0 + col] : T(0);
      *(T*)(st + BOFF + (krow * CPRB + ((col / EPC) ^ swzb<T>(krow))) * 16 + (col % EPC) * (int)sizeof(T)) = v;
    }
  };

  acc_t acc[BI][BI];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BI; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  // Products of one stage: lane group g = lane / 16 supplies k = g KS + s in
  // k step s, for A (one 16-byte chunk per block row) and B alike. Block
  // (i, j) of the wave's quarter only needs k >= its first column (T = C A^-1,
  // A^-1 lower) or k < its last row + 1 (X21 = -B^-1 T, B^-1 lower): a stage
  // wholly outside that range skips the block's MFMAs (wave-uniform).
  auto compute = [&](int slot, int k0, int kind) {
    const char* st = ring + slot * R::STAGE;
    T a[BI][KS], b[BI][KS];
#pragma unroll
    for (int i = 0; i < BI; ++i) {
      const int row = wm * (TM / 2) + 16 * i + (lane & 15);
      const int pos = (lane >> 4) ^ ((row >> 2) & 3);
      const vec_t v = *(const vec_t*)(st + (row * 4 + pos) * 16);
#pragma unroll
      for (int s = 0; s < KS; ++s) a[i][s] = v[s];
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int krow = (lane >> 4) * KS + s;
#pragma unroll
      for (int j = 0; j < BI; ++j) {
        const int col = wn * (TM / 2) + 16 * j + (lane & 15);
        b[j][s] = *(const T*)(st + BOFF + (krow * CPRB + ((col / EPC) ^ swzb<T>(krow))) * 16 +
                              (col % EPC) * (int)sizeof(T));
      }
    }
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int j = 0; j < BI; ++j) {
        // tile-relative first column / last row of the block (both uniform)
        const bool need = kind == 0 ? (k0 + KC > dc.c0 + wn * (TM / 2) + 16 * j)
                                    : (k0 < dc.r0 + wm * (TM / 2) + 16 * i + 16);
        if (need) {
#pragma unroll
          for (int s = 0; s < KS; ++s) acc[i][j] = BMma<T>::op(a[i][s], b[j][s], acc[i][j]);
        }
      }
  };
  auto epilogue = [&](const TileDesc<T>& d) {
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int j = 0; j < BI; ++j) {
        const int col = d.c0 + wn * (TM / 2) + 16 * j + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = d.r0 + wm * (TM / 2) + 16 * i + BMma<T>::row(lane, r);
          const T v = d.alpha * acc[i][j][r];
          if (row < d.M) {
            d.D[row * d.ld + col] = v;
            nf |= !__builtin_isfinite(v);
          }
        }
        acc[i][j] = acc_t{0, 0, 0, 0};
      }
  };

  // issue cursor: tile ti, its stage si
  int ti = 0, si = 0, issued = 0;
  TileDesc<T> di = tiles(0);
  int nsi = nstages(di);
  auto issue_next = [&]() {
    issue(issued % NS, di, di.klo + si * KC);
    ++issued;
    if (++si >= nsi) {
      si = 0;
      if (++ti < ntiles) {
        di = tiles(ti);
        nsi = nstages(di);
      }
    }
  };
#pragma unroll
  for (int p = 0; p < NS - 1; ++p)
    if (ti < ntiles) issue_next();
  bool stores = false;  // epilogue stores outstanding: wait for everything
  for (int g = 0;; ++g) {
    const int ahead = issued - 1 - g;  // stages issued after stage g
    if (stores || ahead <= 0)
      wait_barrier<0>();
    else if (ahead == 1)
      wait_barrier<LPS>();
    else
      wait_barrier<2 * LPS>();
    stores = false;
    if (ti < ntiles) issue_next();  // into the slot read in the previous iteration
    const int k0 = dc.klo + sc * KC;
    if (k0 + KC > dc.khi) {
      guarded_fill(g % NS, dc, k0);
      __syncthreads();
    }
    compute(g % NS, k0, tiles.kind);
    if (++sc == nsc) {
      epilogue(dc);
      stores = true;
      if (++tc == ntiles) break;
      dc = tiles(tc);
      nsc = nstages(dc);
      sc = 0;
    }
  }
  drain();  // the step's stores visible to the workgroup's next loads
  return nf;
}

// Leaves of order LEAF (the last may be shorter): lane j of a wave (or of a
// half wave for LEAF = 32) owns column j of one leaf and runs the column
// recurrence
//   X(j, j) = 1 / L(j, j),  X(i, j) = -(sum_{k=j}^{i-1} L(i, k) X(k, j)) / L(i, i)
// right-looking in registers: once X(k, j) is final it is added into the
// running sums of the rows below (the same ascending-k summation as the
// formula, so the same rounding). The leaf's L^T sits in LDS (row k of L^T
// read as 16-byte pieces, the same address for every lane of the leaf); the
// finished X^T goes back to the same LDS rows and leaves for X in row
// pieces. The whole leaf block of X is written, zeros above the diagonal
// included. Returns whether this thread stored a NaN or an infinity.
template <typename T, int LEAF>
__device__ __forceinline__ bool leaves(const T* __restrict__ L, T* __restrict__ X, int n, int unit, char* smem,
                                       int* bad) {
  constexpr int PER = 64 / LEAF;   // leaves per wave at a time
  constexpr int LS = LEAF + 4;     // LDS row stride (16-byte aligned rows)
  constexpr int V = 16 / sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(V)));
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane / LEAF, j = lane % LEAF;
  T* Lt = (T*)smem + (wave * PER + half) * LEAF * LS;
  const int nl = (n + LEAF - 1) / LEAF;
  bool nf = false;
  for (int l0 = 0; l0 < nl; l0 += 4 * PER) {
    const int l = l0 + wave * PER + half;
    const int base = l * LEAF;
    const int bl = l < nl ? min(LEAF, n - base) : 0;
    // stage L^T: lane j reads L(base + i, base + j) along row i (coalesced),
    // every load issued before the first is used (addresses clamped into the
    // leaf, or into the matrix's first leaf for lanes without a leaf)
    {
      const int sb = bl > 0 ? base : 0, ilast = bl > 0 ? bl - 1 : 0;
      T v[LEAF];
#pragma unroll
      for (int i = 0; i < LEAF; ++i) {
        const int ii = min(i, ilast), jj = min(j, ii);
        v[i] = L[(sb + ii) * n + sb + jj];
      }
#pragma unroll
      for (int i = 0; i < LEAF; ++i)
        Lt[j * LS + i] = (unit && i == j) ? T(1) : ((i < bl && j <= i) ? v[i] : T(0));
    }
    __syncthreads();
    if (!unit && j < bl && Lt[j * LS + j] == T(0)) atomicMin(bad, base + j + 1);
    // x starts as -e_j, so that every lane runs the same steps: at pivot k,
    // x[k] = -x[k] / L(k, k) gives 1 / L(j, j) for k = j, X(k, j) from the
    // negated running sum for k > j and 0 above the diagonal (the + 0 turns
    // a -0 into +0).
    T x[LEAF];  // running sum of row i, then X(i, j)
#pragma unroll
    for (int i = 0; i < LEAF; ++i) x[i] = (i == j) ? T(-1) : T(0);
#pragma unroll
    for (int k = 0; k < LEAF; ++k) {
      x[k] = -x[k] / Lt[k * LS + k] + T(0);  // unit: L^T holds exact ones on its diagonal
#pragma unroll
      for (int i4 = (k + 1) / V * V; i4 < LEAF; i4 += V) {
        const vec_t lv = *(const vec_t*)(Lt + k * LS + i4);
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (i4 + e > k) x[i4 + e] += lv[e] * x[k];
      }
      __builtin_amdgcn_sched_barrier(0);  // keep each pivot's LDS reads in its step (bounded registers)
    }
    // every lane of the leaf is past its reads of L^T (lockstep within the
    // wave): X^T replaces it, column j of X as row j
#pragma unroll
    for (int i4 = 0; i4 < LEAF; i4 += V) {
      vec_t v;
#pragma unroll
      for (int e = 0; e < V; ++e) v[e] = x[i4 + e];
      *(vec_t*)(Lt + j * LS + i4) = v;
    }
    __syncthreads();
    // rows of the leaf block of X: lane j of the leaf stores X(i, j)
    for (int i = 0; i < bl; ++i) {
      if (j < bl) {
        const T v = Lt[j * LS + i];
        X[(base + i) * n + base + j] = v;
        nf |= !__builtin_isfinite(v);
      }
    }
    __syncthreads();
  }
  drain();  // the leaves' stores visible to the level products
  return nf;
}

// All levels of one matrix (see the file comment).
template <typename T, int LEAF>
__device__ __forceinline__ bool levels(const T* __restrict__ L, T* X, int n, char* ring, int tmax) {
  const int tid = threadIdx.x;
  bool nf = false;
  for (int h = LEAF; h < n; h *= 2) {
    const int span = 2 * h;
    const int nmerge = (n - h + span - 1) / span;
    const int hb_last = min(h, n - (nmerge - 1) * span - h);
    LevelTiles<T> lt{L, X, n, h, nmerge, hb_last, h < tmax ? h : tmax, 0};  // tile min(h, tmax): 32, 64 or 128
    // kind 0: T = C A^-1; kind 1: X21 = -B^-1 T (one call site per tile size)
#pragma unroll 1
    for (int kind = 0; kind < 2; ++kind) {
      lt.kind = kind;
      if (lt.TM == 128)
        nf |= run_step<T, 128>(lt, ring);
      else if (lt.TM == 64)
        nf |= run_step<T, 64>(lt, ring);
      else
        nf |= run_step<T, 32>(lt, ring);
    }
    // X12 = 0 (the merged block's upper triangle, read by the next level):
    // h rows of hb zeros per merge, the threads spread over whole rows
    for (int m = 0; m < nmerge; ++m) {
      const int o = m * span, hb = (m == nmerge - 1) ? hb_last : h;
      const int tpr = min(hb, kThreads);  // threads per row
      const int rpp = kThreads / tpr;     // rows per pass
      const int c = tid % tpr, r0 = tid / tpr;
      if (r0 < rpp)
        for (int r = r0; r < h; r += rpp)
          for (int cc = c; cc < hb; cc += tpr) X[(o + r) * n + o + h + cc] = T(0);
    }
    drain();
  }
  return nf;
}

template <typename T, int LEAF>
constexpr int batched_lds_bytes() {
  constexpr int leaf = 4 * (64 / LEAF) * LEAF * (LEAF + 4) * (int)sizeof(T);
  return leaf > Ring<T>::BYTES ? leaf : Ring<T>::BYTES;
}

// FP32: registers for two resident workgroups per CU; FP64 (twice the
// accumulator and operand registers) keeps one.
template <typename T, int LEAF>
__global__ __launch_bounds__(kThreads, sizeof(T) == 4 ? 2 : 1) void k_batched(int64_t batch, const int32_t* __restrict__ n_dev,
                                                      const int64_t* __restrict__ off_dev, const T* __restrict__ L,
                                                      T* __restrict__ X, int32_t* __restrict__ status,
                                                      const int32_t* __restrict__ order, uint32_t* queue, int unit,
                                                      int tmax) {
  // the leaves' L^T or the product ring (dynamic LDS)
  extern __shared__ __attribute__((aligned(16))) char smem[];
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
      nf |= leaves<T, LEAF>(Lm, Xm, n, unit, smem, &s_bad);
      nf |= levels<T, LEAF>(Lm, Xm, n, smem, tmax);
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

template <typename T, int LEAF>
hipError_t set_lds_attr() {
  static bool done = false;  // per instantiation
  if (done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_batched<T, LEAF>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     batched_lds_bytes<T, LEAF>());
  if (e == hipSuccess) done = true;
  return e;
}

}  // namespace

template <typename T>
hipError_t launch_batched(int64_t batch, const int32_t* n_dev, const int64_t* off_dev, const T* L, T* X,
                          int32_t* status, int32_t* order, uint32_t* queue, int unit, int grid, int leaf,
                          int tmax, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if ((leaf != 32 && leaf != 64) || (tmax != 64 && tmax != 128) || grid < 1) return hipErrorInvalidValue;
  hipError_t e = leaf == 64 ? set_lds_attr<T, 64>() : set_lds_attr<T, 32>();
  if (e != hipSuccess) return e;
  TRINV_LAUNCH(k_batched_plan, dim3(1), dim3(1024), 0, s, batch, n_dev, order, queue);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr size_t lds64 = batched_lds_bytes<T, 64>(), lds32 = batched_lds_bytes<T, 32>();
  if (leaf == 64)
    TRINV_LAUNCH((k_batched<T, 64>), dim3((unsigned)grid), dim3(kThreads), lds64, s, batch, n_dev, off_dev, L,
                       X, status, order, queue, unit, tmax);
  else
    TRINV_LAUNCH((k_batched<T, 32>), dim3((unsigned)grid), dim3(kThreads), lds32, s, batch, n_dev, off_dev, L,
                       X, status, order, queue, unit, tmax);
  return hipGetLastError();
}

template <typename T>
int batched_occupancy(int leaf, int* cus_out) {
  static int per_cu[2] = {-1, -1}, cus = 0;
  const int w = leaf == 64 ? 1 : 0;
  if (per_cu[w] < 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
    int occ = 0;
    hipError_t e = leaf == 64 ? set_lds_attr<T, 64>() : set_lds_attr<T, 32>();
    if (e == hipSuccess)
      e = leaf == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batched<T, 64>, kThreads,
                                                                    batched_lds_bytes<T, 64>())
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batched<T, 32>, kThreads,
                                                                    batched_lds_bytes<T, 32>());
    if (e != hipSuccess || occ < 1) occ = 1;
    per_cu[w] = occ;
  }
  if (cus_out) *cus_out = cus;
  return per_cu[w];
}

template <typename T>
int batched_grid(int64_t batch, int leaf, int per_cu) {
  int cus = 0;
  const int occ = batched_occupancy<T>(leaf, &cus);
  const int k = (per_cu >= 1 && per_cu <= occ) ? per_cu : occ;
  const int64_t g = (int64_t)cus * k;
  return (int)(batch < g ? batch : g);
}

template hipError_t launch_batched<float>(int64_t, const int32_t*, const int64_t*, const float*, float*, int32_t*,
                                          int32_t*, uint32_t*, int, int, int, int, hipStream_t);
template hipError_t launch_batched<double>(int64_t, const int32_t*, const int64_t*, const double*, double*, int32_t*,
                                           int32_t*, uint32_t*, int, int, int, int, hipStream_t);
template int batched_occupancy<float>(int, int*);
template int batched_occupancy<double>(int, int*);
template int batched_grid<float>(int64_t, int, int);
template int batched_grid<double>(int64_t, int, int);

}  // namespace trinv
