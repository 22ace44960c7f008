// FP64 / FP32 MFMA tile products for the off-diagonal blocks of the
// recursion and for the FP64 residual check.
//
// The recursion (Section 4.1, algorithm COMBRIT with beta = 2, transposed to
// the lower case) needs, for every merge of two inverted diagonal blocks A^-1
// (order hA) and B^-1 (order hB) with the coupling block C (hB x hA):
//     T   =  C * A^-1      full x lower   (Ptf, eq. ptfm: h^3 flops)
//     X21 = -B^-1 * T      lower x full   (Ptf again)
// Both are ordinary products whose K range per output tile is cut by the
// triangle of the triangular operand, so MFMA work on the zero triangle is
// limited to the diagonal K step. All merges of one level run in one launch.
//
// Tiling for gfx950: a 256-thread workgroup computes a 128 x 128 tile of D
// with 16 x 16 x 4 MFMAs (FP64: v_mfma_f64_16x16x4_f64, FP32:
// v_mfma_f32_16x16x4_f32); each of the 4 waves owns a 64 x 64 sub-tile
// (4 x 4 MFMA blocks). K advances in steps of 16 through two LDS buffers, the
// next step's global loads being in flight while the current step is
// multiplied. MFMA lane layouts (measured on gfx950): lane l supplies
// A(l%16, l/16) and B(l/16, l%16); the FP64 result of register r is
// D(4r + l/16, l%16), the FP32 one D(4(l/16) + r, l%16).
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
__device__ __forceinline__ void decode_tile(int64_t t, int tiles, int order, int64_t nz, int64_t tm,
                                            int64_t tn, int64_t& z, int64_t& it, int64_t& jt) {
  if (tiles == kAllTiles) {
    if (order == kRowDesc) {  // tiles of one row (over all products) together
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
  if (order == kRowAsc) {
    it = u;
    jt = w;
  } else if (order == kColDesc) {
    jt = tm - 1 - u;
    it = jt + w;
  } else {  // kDiagDesc
    jt = w;
    it = w + (tm - 1 - u);
  }
}
}  // namespace

int64_t gemm_tiles(const GemmBatch& bt, int tiles) {
  const int64_t tm = (bt.M + TM - 1) / TM, tn = (bt.N + TN - 1) / TN;
  const int64_t nz = bt.nmerge * bt.nbatch;
  if (tiles == kLowerTiles) return nz * tm * (tm + 1) / 2;
  return nz * tm * tn;
}

template <typename TI, typename TC>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs<TI> a) {
  typedef Mma<TC> MM;
  __shared__ TC lds[2 * (ABUF + BBUF)];
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const GemmBatch& bt = a.bt;
  const int64_t tm = (bt.M + TM - 1) / TM, tn = (bt.N + TN - 1) / TN;
  const int64_t nz = bt.nmerge * bt.nbatch;
  const int64_t total = (a.tiles == kLowerTiles) ? nz * tm * (tm + 1) / 2 : nz * tm * tn;
  const int64_t t = xcd_remap(blockIdx.x, total, 8);
  int64_t z, it, jt;
  decode_tile(t, a.tiles, a.order, nz, tm, tn, z, it, jt);
  const int64_t zb = z / bt.nmerge, zk = z % bt.nmerge;
  const bool last = (zk == bt.nmerge - 1);
  const int64_t M = last ? bt.M_last : bt.M, N = last ? bt.N_last : bt.N, K = last ? bt.K_last : bt.K;
  const int64_t m0 = it * TM, n0 = jt * TN;
  if (m0 >= M || n0 >= N) {
    if (a.tile_sq && tid == 0) a.tile_sq[t] = 0.0;
    return;
  }

  int64_t klo = 0, khi = K;
  if (a.klo == kLoN0) klo = n0;
  else if (a.klo == kLoM0) klo = m0;
  else if (a.klo == kLoMax) klo = imax64(m0, n0);
  if (a.khi == kHiM1) khi = imin64(K, m0 + TM);
  else if (a.khi == kHiN1) khi = imin64(K, n0 + TN);
  klo = (klo / KT) * KT;

  const TI* __restrict__ Ab = a.A.base + zb * a.A.bstride2 + zk * a.A.bstride;
  const TI* __restrict__ Bb = a.B.base + zb * a.B.bstride2 + zk * a.B.bstride;
  const int64_t a_sm = a.a_trans ? 1 : a.A.ld, a_sk = a.a_trans ? a.A.ld : 1;
  const int64_t b_sk = a.b_trans ? 1 : a.B.ld, b_sn = a.b_trans ? a.B.ld : 1;

  // Staging maps (8 elements of each operand tile per thread), chosen so that
  // consecutive lanes read consecutive addresses:
  //   A 128 x 16: row-major -> 16 lanes along k; transposed -> 128 lanes along m.
  //   B 16 x 128: row-major -> 128 lanes along n; transposed -> 16 lanes along k.
  const int am = a.a_trans ? (tid & 127) : (tid >> 4), ak = a.a_trans ? (tid >> 7) : (tid & 15);
  const int am_step = a.a_trans ? 0 : 16, ak_step = a.a_trans ? 2 : 0;
  const int bn = a.b_trans ? (tid >> 4) : (tid & 127), bk = a.b_trans ? (tid & 15) : (tid >> 7);
  const int bn_step = a.b_trans ? 16 : 0, bk_step = a.b_trans ? 0 : 2;
  TC ra[8], rb[8];

  auto load = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int64_t m = m0 + am + am_step * p, k = k0 + ak + ak_step * p;
      bool ok = (m < M) && (k < K);
      if (a.amask == 1) ok = ok && (k <= m);
      else if (a.amask == 2) ok = ok && (k < m);
      else if (a.amask == 3) ok = ok && (k >= m);
      ra[p] = ok ? (TC)Ab[m * a_sm + k * a_sk] : (TC)0;
    }
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int64_t k = k0 + bk + bk_step * p, nn = n0 + bn + bn_step * p;
      bool ok = (k < K) && (nn < N);
      if (a.bmask == 1) ok = ok && (k >= nn);
      else if (a.bmask == 2) ok = ok && (k > nn);
      else if (a.bmask == 3) ok = ok && (k <= nn);
      rb[p] = ok ? (TC)Bb[k * b_sk + nn * b_sn] : (TC)0;
    }
  };
  auto store = [&](int buf) {
    TC* As = lds + buf * (ABUF + BBUF);
    TC* Bs = As + ABUF;
#pragma unroll
    for (int p = 0; p < 8; ++p) As[(am + am_step * p) * SA + ak + ak_step * p] = ra[p];
#pragma unroll
    for (int p = 0; p < 8; ++p) Bs[(bk + bk_step * p) * SB + bn + bn_step * p] = rb[p];
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

  // Epilogue: scale, identity subtraction, lower-only output, stores, norm.
  TI* __restrict__ Db = a.D.base ? a.D.base + zb * a.D.bstride2 + zk * a.D.bstride : nullptr;
  char* __restrict__ Lb =
      a.Dlp.base ? (char*)a.Dlp.base + 2 * (zb * a.Dlp.bstride2 + zk * a.Dlp.bstride) : nullptr;
  double sq = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wm * 64 + i * 16 + MM::row(lane, r);
        const int64_t col = n0 + wn * 64 + j * 16 + (lane & 15);
        if (row < M && col < N) {
          double v = a.alpha * (double)acc[i][j][r];
          if (a.subtract_identity && row == col) v -= 1.0;
          if (a.out_lower && col > row) v = 0.0;
          if (Db) Db[row * a.D.ld + col] = (TI)v;
          sq += v * v;
          if (Lb) {
            const int64_t e = row * a.Dlp.ld + col;
            if (a.lp_is_f16) ((_Float16*)Lb)[e] = (_Float16)(float)v;
            else ((__bf16*)Lb)[e] = (__bf16)(float)v;
          }
        }
      }

  if (a.Zmirror.base && !(a.mirror_skip_diag && it == jt)) {
    TI* Zb = a.Zmirror.base + zb * a.Zmirror.bstride2 + zk * a.Zmirror.bstride;
    for (int e = tid; e < TM * TN; e += 256) {
      const int64_t mr = n0 + e / TM, mc = m0 + e % TM;
      if (mr < N && mc < M) Zb[mr * a.Zmirror.ld + mc] = (TI)0;
    }
  }

  if (a.tile_sq) {
    for (int m = 32; m >= 1; m >>= 1) sq += __shfl_xor(sq, m, 64);
    if (lane == 0) red[wave] = sq;
    __syncthreads();
    if (tid == 0) a.tile_sq[t] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

template <typename TI, typename TC>
hipError_t launch_gemm(const GemmArgs<TI>& a, hipStream_t s) {
  const int64_t total = gemm_tiles(a.bt, a.tiles);
  if (total <= 0) return hipSuccess;
  if (total > 0x7fffffff) return hipErrorInvalidValue;
  if (a.tiles == kLowerTiles && a.bt.M != a.bt.N) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_gemm<TI, TC>), dim3((unsigned)total), dim3(256), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_gemm<double, double>(const GemmArgs<double>&, hipStream_t);
template hipError_t launch_gemm<float, float>(const GemmArgs<float>&, hipStream_t);
template hipError_t launch_gemm<float, double>(const GemmArgs<float>&, hipStream_t);

}  // namespace trinv
