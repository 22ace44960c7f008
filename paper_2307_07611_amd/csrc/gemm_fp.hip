// FP64 / FP32 MFMA tile products for the off-diagonal blocks of the
// recursion, the adjoint, the factored inverse and the FP64 residual check.
//
// The recursion (Section 4.1, algorithm COMBRIT with beta = 2, transposed to
// the lower case) needs, for every merge of two inverted diagonal blocks A^-1
// (order hA) and B^-1 (order hB) with the coupling block C (hB x hA):
//     T   =  C * A^-1      full x lower   (Ptf, eq. ptfm: h^3 flops)
//     X21 = -B^-1 * T      lower x full   (Ptf again)
// Both are ordinary products whose K range per output tile is cut by the
// triangle of the triangular operand, so MFMA work on the zero triangle is
// limited to the diagonal K steps. All merges of one level run in one launch.
//
// Tiling for gfx950: a 256-thread workgroup computes a 128 x 128 tile of D
// with 16 x 16 x 4 MFMAs (FP64: v_mfma_f64_16x16x4_f64, FP32:
// v_mfma_f32_16x16x4_f32); each of the 4 waves owns a 64 x 64 sub-tile
// (4 x 4 MFMA blocks). K advances in steps of 16 through two LDS buffers, the
// next step's global loads being in flight while the current step is
// multiplied. MFMA lane layouts (measured on gfx950): lane l supplies
// A(l%16, l/16) and B(l/16, l%16); the FP64 result of register r is
// D(4r + l/16, l%16), the FP32 one D(4(l/16) + r, l%16).
//
// Every option (transposed operands, element masks, K-range rule, tile set,
// epilogue) is a template parameter, and out-of-range elements are handled by
// loading a clamped in-range address and selecting zero, so the main loop has
// no branches besides the loop itself.
#include "common.h"
#include "launch.h"

namespace trinv {

namespace {
constexpr int TM = 128, TN = 128, KT = 16;
constexpr int SA = KT + 1;  // LDS row stride of the A tile, stored [m][k]
constexpr int SB = TN + 2;  // LDS row stride of the B tile, stored [k][n]
constexpr int ABUF = TM * SA, BBUF = KT * SB;

template <typename TC>
struct Mma;
template <>
struct Mma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct Mma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Largest u with u (u + 1) / 2 <= q.
__device__ __forceinline__ int64_t tri_root(int64_t q) {
  int64_t u = (int64_t)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
  while (u * (u + 1) / 2 > q) --u;
  while ((u + 1) * (u + 2) / 2 <= q) ++u;
  return u;
}

// Logical tile t -> (product z, tile row it, tile col jt) in the stated order.
template <int TILES, int ORDER>
__device__ __forceinline__ void decode_tile(int64_t t, int64_t nz, int64_t tm, int64_t tn, int64_t& z, int64_t& it,
                                            int64_t& jt) {
  if (TILES == kAllTiles) {
    if (ORDER == kRowDesc) {  // tiles of one row (over all products) together
      const int64_t g = t / (nz * tn), r = t % (nz * tn);
      it = tm - 1 - g;
      z = r / tn;
      jt = r % tn;
    } else {  // kColAsc
      const int64_t g = t / (nz * tm), r = t % (nz * tm);
      jt = g;
      z = r / tm;
      it = r % tm;
    }
    return;
  }
  const int64_t per = tm * (tm + 1) / 2;
  z = t / per;
  const int64_t q = t % per;
  const int64_t u = tri_root(q), w = q - u * (u + 1) / 2;
  if (ORDER == kRowAsc) {
    it = u;
    jt = w;
  } else if (ORDER == kColDesc) {
    jt = tm - 1 - u;
    it = jt + w;
  } else {  // kDiagDesc
    jt = w;
    it = w + (tm - 1 - u);
  }
}

template <int MASK, bool IS_A>
__device__ __forceinline__ bool mask_ok(int64_t r, int64_t k) {
  // A(r = m, k): lower k <= m, strict lower k < m, upper k >= m.
  // B(k, r = n): lower k >= n, strict lower k > n, upper k <= n.
  if (MASK == 0) return true;
  if (IS_A) {
    if (MASK == 1) return k <= r;
    if (MASK == 2) return k < r;
    return k >= r;
  }
  if (MASK == 1) return k >= r;
  if (MASK == 2) return k > r;
  return k <= r;
}
}  // namespace

int64_t gemm_tiles(const GemmBatch& bt, int tiles) {
  const int64_t tm = (bt.M + TM - 1) / TM, tn = (bt.N + TN - 1) / TN;
  const int64_t nz = bt.nmerge * bt.nbatch;
  if (tiles == kLowerTiles) return nz * tm * (tm + 1) / 2;
  return nz * tm * tn;
}

// Epilogue flags.
enum {
  kEpStore = 1,
  kEpMirror = 2,
  kEpMirrorSkipDiag = 4,
  kEpOutLower = 8,
  kEpSubI = 16,
  kEpTileSq = 32,
  kEpLowp = 64,
  kEpRefineResid = 128,
  kEpAccum = 256  // D = alpha acc + D (read before the store)
};

// Two workgroups per CU (256 registers per lane, 2 x 68 KB of LDS): with one
// wave per SIMD, each K step's LDS reads and the store of the next step's
// operands left the matrix core idle; a second resident wave fills those gaps.
template <typename TI, typename TC, int AT, int BT, int AM, int BM, int TILES, int ORDER, int KLO, int KHI, int EP>
__global__ __launch_bounds__(256, 2) void k_gemm(GemmArgs<TI> a) {
  typedef Mma<TC> MM;
  __shared__ TC lds[2 * (ABUF + BBUF)];
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const GemmBatch bt = a.bt;
  const int64_t tm = (bt.M + TM - 1) / TM, tn = (bt.N + TN - 1) / TN;
  const int64_t nz = bt.nmerge * bt.nbatch;
  const int64_t total = (TILES == kLowerTiles) ? nz * tm * (tm + 1) / 2 : nz * tm * tn;
  const int64_t t = xcd_remap(blockIdx.x, total, 8);
  int64_t z, it, jt;
  decode_tile<TILES, ORDER>(t, nz, tm, tn, z, it, jt);
  const int64_t zb = z / bt.nmerge, zk = z % bt.nmerge;
  const bool last = (zk == bt.nmerge - 1);
  const int64_t M = last ? bt.M_last : bt.M, N = last ? bt.N_last : bt.N, K = last ? bt.K_last : bt.K;
  const int64_t m0 = it * TM, n0 = jt * TN;
  if (m0 >= M || n0 >= N) {
    if ((EP & (kEpTileSq | kEpRefineResid)) && tid == 0) a.tile_sq[t] = 0.0;
    if ((EP & kEpRefineResid) && tid == 0) a.tile_sqx[t] = 0.0;
    return;
  }

  int64_t klo = 0, khi = K;
  if (KLO == kLoN0) klo = n0;
  if (KLO == kLoM0) klo = m0;
  if (KLO == kLoMax) klo = imax64(m0, n0);
  if (KHI == kHiM1) khi = imin64(K, m0 + TM);
  if (KHI == kHiN1) khi = imin64(K, n0 + TN);
  klo = (klo / KT) * KT;

  const TI* __restrict__ Ab = a.A.base + zb * a.A.bstride2 + zk * a.A.bstride;
  const TI* __restrict__ Bb = a.B.base + zb * a.B.bstride2 + zk * a.B.bstride;
  const int64_t lda = a.A.ld, ldb = a.B.ld;

  // Staging maps (8 elements of each operand tile per thread), chosen so that
  // consecutive lanes read consecutive addresses:
  //   A 128 x 16: row-major -> 16 lanes along k; transposed -> 128 lanes along m.
  //   B 16 x 128: row-major -> 128 lanes along n; transposed -> 16 lanes along k.
  constexpr int AM_STEP = AT ? 0 : 16, AK_STEP = AT ? 2 : 0;
  constexpr int BN_STEP = BT ? 16 : 0, BK_STEP = BT ? 0 : 2;
  const int am = AT ? (tid & 127) : (tid >> 4), ak = AT ? (tid >> 7) : (tid & 15);
  const int bn = BT ? (tid >> 4) : (tid & 127), bk = BT ? (tid & 15) : (tid >> 7);

  // Each staged element has a fixed "row" index for the whole tile (m for A,
  // n for B). Rows beyond M (columns beyond N) only feed outputs that are not
  // stored, so they are clamped to the last valid row and loaded as is; only
  // the K direction needs zero fill (k >= K) and the element masks, and only
  // K steps that reach the K edge or a masked diagonal take that guarded path.
  // Each thread keeps one pointer per staged element and advances it by one
  // K step per iteration.
  const TI* pa[8];
  const TI* pb[8];
  const int64_t a_kstep = AT ? (int64_t)KT * lda : (int64_t)KT;  // pointer advance per K step
  const int64_t b_kstep = BT ? (int64_t)KT : (int64_t)KT * ldb;
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int64_t m = imin64(m0 + am + AM_STEP * p, M - 1);
    const int64_t ka = klo + ak + AK_STEP * p;
    pa[p] = AT ? Ab + ka * lda + m : Ab + m * lda + ka;
    const int64_t nn = imin64(n0 + bn + BN_STEP * p, N - 1);
    const int64_t kb = klo + bk + BK_STEP * p;
    pb[p] = BT ? Bb + nn * ldb + kb : Bb + kb * ldb + nn;
  }

  TC ra[8], rb[8];
  // Fast path: K step fully inside [0, K) and away from masked diagonals.
  auto load_fast = [&]() {
#pragma unroll
    for (int p = 0; p < 8; ++p) ra[p] = (TC)*pa[p];
#pragma unroll
    for (int p = 0; p < 8; ++p) rb[p] = (TC)*pb[p];
  };
  // Guarded path: zero fill beyond K and element masks. The address is
  // clamped back inside the operand before the load.
  auto load_guard = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int64_t k = k0 + ak + AK_STEP * p;
      const bool ok = (k < K) && mask_ok<AM, true>(m0 + am + AM_STEP * p, k);
      const int64_t back = k < K ? 0 : (k - (K - 1));  // elements of K to step back
      const TI v = *(pa[p] - (AT ? back * lda : back));
      ra[p] = ok ? (TC)v : (TC)0;
    }
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int64_t k = k0 + bk + BK_STEP * p;
      const bool ok = (k < K) && mask_ok<BM, false>(n0 + bn + BN_STEP * p, k);
      const int64_t back = k < K ? 0 : (k - (K - 1));
      const TI v = *(pb[p] - (BT ? back : back * ldb));
      rb[p] = ok ? (TC)v : (TC)0;
    }
  };
  auto needs_guard = [&](int64_t k0) -> bool {
    if (k0 + KT > K) return true;
    if (AM != 0 && k0 + KT > m0 && k0 < m0 + TM) return true;
    if (BM != 0 && k0 + KT > n0 && k0 < n0 + TN) return true;
    return false;
  };
  auto load = [&](int64_t k0) {
    if (needs_guard(k0)) load_guard(k0);
    else load_fast();
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      pa[p] += a_kstep;
      pb[p] += b_kstep;
    }
  };
  auto store = [&](int buf) {
    TC* As = lds + buf * (ABUF + BBUF);
    TC* Bs = As + ABUF;
#pragma unroll
    for (int p = 0; p < 8; ++p) As[(am + AM_STEP * p) * SA + ak + AK_STEP * p] = ra[p];
#pragma unroll
    for (int p = 0; p < 8; ++p) Bs[(bk + BK_STEP * p) * SB + bn + BN_STEP * p] = rb[p];
  };

  typename MM::acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = (TC)0;

  if (klo < khi) {
    load(klo);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = klo; k0 < khi; k0 += KT) {
      const bool more = (k0 + KT < khi);
      if (more) load(k0 + KT);
      const TC* As = lds + buf * (ABUF + BBUF);
      const TC* Bs = As + ABUF;
#pragma unroll
      for (int kk = 0; kk < KT; kk += 4) {
        TC av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = As[(wm * 64 + i * 16 + (lane & 15)) * SA + kk + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = Bs[(kk + (lane >> 4)) * SB + wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = MM::op(av[i], bv[j], acc[i][j]);
      }
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  if (EP & kEpRefineResid) {
    // R = I - L X from acc = (N_L N_X)(row, col) and the O(n^2) FP64 terms.
    double sq = 0.0, sqx = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = m0 + wm * 64 + i * 16 + MM::row(lane, r);
          const int64_t col = n0 + wn * 64 + j * 16 + (lane & 15);
          if (row < M && col < N && col <= row) {
            const double lii = a.dL[row];
            const double xij = (double)a.Xfull[row * a.ldx + col];
            double rv;
            if (row == col) rv = fma(-lii, xij, 1.0);
            else rv = -(double)acc[i][j][r] - lii * xij - (double)a.Lfull[row * a.ldl + col] * a.dX[col];
            a.R32[row * a.ldr + col] = (float)rv;
            if (a.Rt) {
              const int64_t e = col * a.ldrt + row;
              if (a.lp_is_f16) ((_Float16*)a.Rt)[e] = (_Float16)(float)rv;
              else ((__bf16*)a.Rt)[e] = (__bf16)(float)rv;
            }
            sq += rv * rv;
            sqx += xij * xij;
          } else if (row < M && col < N && a.Rt) {  // above the diagonal: zero in the transposed copy
            const int64_t e = col * a.ldrt + row;
            if (a.lp_is_f16) ((_Float16*)a.Rt)[e] = (_Float16)0.f;
            else ((__bf16*)a.Rt)[e] = (__bf16)0.f;
          }
        }
    for (int m = 32; m >= 1; m >>= 1) {
      sq += __shfl_xor(sq, m, 64);
      sqx += __shfl_xor(sqx, m, 64);
    }
    __shared__ double red2[2][4];
    if (lane == 0) {
      red2[0][wave] = sq;
      red2[1][wave] = sqx;
    }
    __syncthreads();
    if (tid == 0) {
      a.tile_sq[t] = (red2[0][0] + red2[0][1]) + (red2[0][2] + red2[0][3]);
      a.tile_sqx[t] = (red2[1][0] + red2[1][1]) + (red2[1][2] + red2[1][3]);
    }
    return;
  }

  // Epilogue: scale, identity subtraction, lower-only output, stores, norm.
  TI* __restrict__ Db = (EP & kEpStore) ? a.D.base + zb * a.D.bstride2 + zk * a.D.bstride : nullptr;
  char* __restrict__ Lb = (EP & kEpLowp) ? (char*)a.Dlp.base + 2 * (zb * a.Dlp.bstride2 + zk * a.Dlp.bstride) : nullptr;
  const double alpha = a.alpha;
  const bool full_tile = (m0 + TM <= M) && (n0 + TN <= N);
  double sq = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wm * 64 + i * 16 + MM::row(lane, r);
        const int64_t col = n0 + wn * 64 + j * 16 + (lane & 15);
        if (full_tile || (row < M && col < N)) {
          double v = alpha * (double)acc[i][j][r];
          if (EP & kEpAccum) v += (double)Db[row * a.D.ld + col];
          if ((EP & kEpSubI) && row == col) v -= 1.0;
          if ((EP & kEpOutLower) && col > row) v = 0.0;
          if (EP & kEpStore) Db[row * a.D.ld + col] = (TI)v;
          if (EP & kEpTileSq) sq += v * v;
          if (EP & kEpLowp) {
            const int64_t e = row * a.Dlp.ld + col;
            if (a.lp_is_f16) ((_Float16*)Lb)[e] = (_Float16)(float)v;
            else ((__bf16*)Lb)[e] = (__bf16)(float)v;
          }
        }
      }

  if ((EP & kEpMirror) && !((EP & kEpMirrorSkipDiag) && it == jt)) {
    TI* Zb = a.Zmirror.base + zb * a.Zmirror.bstride2 + zk * a.Zmirror.bstride;
    for (int e = tid; e < TM * TN; e += 256) {
      const int64_t mr = n0 + e / TM, mc = m0 + e % TM;
      if (mr < N && mc < M) Zb[mr * a.Zmirror.ld + mc] = (TI)0;
    }
  }

  if (EP & kEpTileSq) {
    for (int m = 32; m >= 1; m >>= 1) sq += __shfl_xor(sq, m, 64);
    if (lane == 0) red[wave] = sq;
    __syncthreads();
    if (tid == 0) a.tile_sq[t] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// Runtime options -> one of the instantiated configurations.
template <typename TI, typename TC, int AT, int BT, int AM, int BM, int TILES, int ORDER, int KLO, int KHI, int EP>
static hipError_t go(const GemmArgs<TI>& a, hipStream_t s, int64_t total) {
  TRINV_LAUNCH((k_gemm<TI, TC, AT, BT, AM, BM, TILES, ORDER, KLO, KHI, EP>), dim3((unsigned)total), dim3(256), 0,
                     s, a);
  return hipGetLastError();
}

template <typename TI>
static int epilogue_of(const GemmArgs<TI>& a) {
  int ep = 0;
  if (a.D.base) ep |= kEpStore;
  if (a.Zmirror.base) ep |= kEpMirror;
  if (a.mirror_skip_diag) ep |= kEpMirrorSkipDiag;
  if (a.out_lower) ep |= kEpOutLower;
  if (a.subtract_identity) ep |= kEpSubI;
  if (a.tile_sq) ep |= kEpTileSq;
  if (a.Dlp.base) ep |= kEpLowp;
  if (a.accumulate) ep |= kEpAccum;
  if (a.refine_resid) ep = kEpRefineResid;
  return ep;
}

template <typename TI, typename TC>
hipError_t launch_gemm(const GemmArgs<TI>& a, hipStream_t s) {
  const int64_t total = gemm_tiles(a.bt, a.tiles);
  if (total <= 0) return hipSuccess;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  if (a.tiles == kLowerTiles && a.bt.M != a.bt.N) return hipErrorInvalidValue;
  const int ep = epilogue_of(a);
  // Configurations used by the library (see the callers):
  // level product C * A^-1
  if (!a.a_trans && !a.b_trans && a.amask == 0 && a.bmask == 0 && a.tiles == kAllTiles && a.order == kColAsc &&
      a.klo == kLoN0 && a.khi == kHiK) {
    if (ep == kEpStore) return go<TI, TC, 0, 0, 0, 0, kAllTiles, kColAsc, kLoN0, kHiK, kEpStore>(a, s, total);
    if (ep == (kEpStore | kEpLowp))
      return go<TI, TC, 0, 0, 0, 0, kAllTiles, kColAsc, kLoN0, kHiK, kEpStore | kEpLowp>(a, s, total);
  }
  // level product -B^-1 * T, zeroing the mirrored block
  if (!a.a_trans && !a.b_trans && a.amask == 0 && a.bmask == 0 && a.tiles == kAllTiles && a.order == kRowDesc &&
      a.klo == kLoZero && a.khi == kHiM1) {
    if (ep == (kEpStore | kEpMirror))
      return go<TI, TC, 0, 0, 0, 0, kAllTiles, kRowDesc, kLoZero, kHiM1, kEpStore | kEpMirror>(a, s, total);
    if (ep == (kEpStore | kEpMirror | kEpLowp))
      return go<TI, TC, 0, 0, 0, 0, kAllTiles, kRowDesc, kLoZero, kHiM1, kEpStore | kEpMirror | kEpLowp>(a, s, total);
  }
  // SKUL L panel: W * U_kk^-1 (B unit upper: k <= column)
  if (!a.a_trans && !a.b_trans && a.amask == 0 && a.bmask == 0 && a.tiles == kAllTiles && a.order == kColAsc &&
      a.klo == kLoZero && a.khi == kHiN1 && ep == kEpStore)
    return go<TI, TC, 0, 0, 0, 0, kAllTiles, kColAsc, kLoZero, kHiN1, kEpStore>(a, s, total);
  // SKUL U panel: L_kk^-1 * W (A lower: k <= row), store only
  if (!a.a_trans && !a.b_trans && a.amask == 0 && a.bmask == 0 && a.tiles == kAllTiles && a.order == kRowDesc &&
      a.klo == kLoZero && a.khi == kHiM1 && ep == kEpStore)
    return go<TI, TC, 0, 0, 0, 0, kAllTiles, kRowDesc, kLoZero, kHiM1, kEpStore>(a, s, total);
  // plain accumulating product (no masks, full K): block chain sums of algorithm COMBRIT, SKUL trailing update
  if (!a.a_trans && !a.b_trans && a.amask == 0 && a.bmask == 0 && a.tiles == kAllTiles && a.order == kColAsc &&
      a.klo == kLoZero && a.khi == kHiK && ep == (kEpStore | kEpAccum))
    return go<TI, TC, 0, 0, 0, 0, kAllTiles, kColAsc, kLoZero, kHiK, kEpStore | kEpAccum>(a, s, total);
  // plain product, full K: the block products of BRSI
  if (!a.a_trans && !a.b_trans && a.amask == 0 && a.bmask == 0 && a.tiles == kAllTiles && a.order == kColAsc &&
      a.klo == kLoZero && a.khi == kHiK && ep == kEpStore)
    return go<TI, TC, 0, 0, 0, 0, kAllTiles, kColAsc, kLoZero, kHiK, kEpStore>(a, s, total);
  // projections of block Gram-Schmidt (SQR): Q_k^T V, A read transposed
  if (a.a_trans && !a.b_trans && a.amask == 0 && a.bmask == 0 && a.tiles == kAllTiles && a.order == kColAsc &&
      a.klo == kLoZero && a.khi == kHiK && ep == kEpStore)
    return go<TI, TC, 1, 0, 0, 0, kAllTiles, kColAsc, kLoZero, kHiK, kEpStore>(a, s, total);
  // SQR inverse S Q^T: A upper (k >= row), B read transposed
  if (!a.a_trans && a.b_trans && a.amask == 0 && a.bmask == 0 && a.tiles == kAllTiles && a.order == kColAsc &&
      a.klo == kLoM0 && a.khi == kHiK && ep == kEpStore)
    return go<TI, TC, 0, 1, 0, 0, kAllTiles, kColAsc, kLoM0, kHiK, kEpStore>(a, s, total);
  // residual check: tril(L) * X - I, norm only
  if (!a.a_trans && !a.b_trans && a.amask == 1 && a.bmask == 0 && a.tiles == kAllTiles && a.order == kRowDesc &&
      a.klo == kLoZero && a.khi == kHiM1 && ep == (kEpSubI | kEpTileSq))
    return go<TI, TC, 0, 0, 1, 0, kAllTiles, kRowDesc, kLoZero, kHiM1, kEpSubI | kEpTileSq>(a, s, total);
  // factored: Uinv * Linv
  if (!a.a_trans && !a.b_trans && a.amask == 3 && a.bmask == 1 && a.tiles == kAllTiles && a.order == kColAsc &&
      a.klo == kLoMax && a.khi == kHiK && ep == kEpStore)
    return go<TI, TC, 0, 0, 3, 1, kAllTiles, kColAsc, kLoMax, kHiK, kEpStore>(a, s, total);
  // adjoint: M = tril(X^T tril(G))
  if (a.a_trans && !a.b_trans && a.amask == 3 && a.bmask == 1 && a.tiles == kLowerTiles && a.order == kRowAsc &&
      a.klo == kLoM0 && a.khi == kHiK && ep == (kEpStore | kEpOutLower))
    return go<TI, TC, 1, 0, 3, 1, kLowerTiles, kRowAsc, kLoM0, kHiK, kEpStore | kEpOutLower>(a, s, total);
  // adjoint: grad = -tril(M X^T), zeroing the strict upper tiles
  if (!a.a_trans && a.b_trans && a.amask == 1 && a.bmask == 3 && a.tiles == kLowerTiles && a.order == kColDesc &&
      a.klo == kLoZero && a.khi == kHiN1 && ep == (kEpStore | kEpOutLower | kEpMirror | kEpMirrorSkipDiag))
    return go<TI, TC, 0, 1, 1, 3, kLowerTiles, kColDesc, kLoZero, kHiN1,
              kEpStore | kEpOutLower | kEpMirror | kEpMirrorSkipDiag>(a, s, total);
  // refinement residual on FP64 MFMA: N_L N_X (both strictly lower), lower tiles
  if (!a.a_trans && !a.b_trans && a.amask == 2 && a.bmask == 2 && a.tiles == kLowerTiles && a.order == kDiagDesc &&
      a.klo == kLoN0 && a.khi == kHiM1 && ep == kEpRefineResid)
    return go<TI, TC, 0, 0, 2, 2, kLowerTiles, kDiagDesc, kLoN0, kHiM1, kEpRefineResid>(a, s, total);
  return hipErrorInvalidValue;
}

template hipError_t launch_gemm<double, double>(const GemmArgs<double>&, hipStream_t);
template hipError_t launch_gemm<float, float>(const GemmArgs<float>&, hipStream_t);
template hipError_t launch_gemm<float, double>(const GemmArgs<float>&, hipStream_t);

}  // namespace trinv
