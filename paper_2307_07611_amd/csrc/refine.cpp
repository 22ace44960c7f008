// Mixed-precision path: the recursion of Section 4.1 (algorithm COMBRIT,
// beta = 2) with its off-diagonal products on BF16 (or FP16) MFMA with FP32
// accumulation, FP64 leaves (column recurrence CRIT, Section 4.2), and then
// Newton-Schulz refinement (not in the paper):
//     R = I - L X,   X <- X + X R   (R_{k+1} = R_k^2 in exact arithmetic;
//                                    X stays lower triangular)
// until ||R||_F / (||L||_F ||X||_F) <= tol.
//
// Residual, assembled and stored in FP64: with L = D_L + N_L and X = D_X + N_X
// (diagonal + strictly lower parts),
//     R = (I - D_L D_X) - D_L N_X - N_L D_X - N_L N_X,
// where the O(n^2) terms are formed exactly in FP64 in the epilogue and the
// O(n^3) product N_L N_X runs on MFMA with both factors split into hi + lo
// slices (three products). Correction: X R = D_X R + N_X R, the first term in
// FP64, the second on MFMA (N_X is small next to D_X for diagonally dominant
// inverses, so its low-precision error is scaled down accordingly).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "api_internal.h"
#include "lowp.h"
#include "profile.h"

namespace trinv {

namespace {

constexpr int64_t kPart = 4096;
constexpr int64_t kBand = 256;  // >= product tile (256) - split tile (64)

int64_t lp_ld(int64_t n) { return (n + 8 + 63) / 64 * 64; }
int64_t t_ld(int64_t hA) { return (hA + 8 + 63) / 64 * 64; }

int64_t lp_t_elems(int64_t n, int64_t leaf) {
  int64_t m = 0;
  for (const Level& l : levels_of(n, leaf)) m = std::max(m, l.nmerge * l.hA * t_ld(l.hA));
  return m;
}

struct WsRefine {
  uint64_t* status;
  // row-major planes of the forward recursion: hi(L), hi(X), hi(X)^T, T^T
  unsigned short *Lhi, *Xb, *Xbt, *Tt;
  // panel-blocked planes of the refinement products: A roles hi/lo(N_L) and
  // hi(N_X); B roles hi/lo(N_X)^T and R^T
  unsigned short *PLhi, *PLlo, *PX, *PXthi, *PXtlo, *PRt;
  float* R32;
  double *dL, *dX, *dX2, *tile_sq, *tile_sqx, *partial, *scal, *split_sq, *split_dsq;
  int64_t ldp, kb;
};

WsRefine carve_refine(Carve& c, int64_t n, int64_t leaf) {
  WsRefine w;
  w.ldp = lp_ld(n);
  w.kb = pb_kblocks(n);
  const size_t pl = (size_t)n * w.ldp + 512;  // one row-major plane (+ slack for over-reads)
  const size_t pp = pb_elems(n);              // one panel-blocked plane
  w.status = c.take<uint64_t>(1);
  w.Lhi = c.take<unsigned short>(pl);
  w.Xb = c.take<unsigned short>(pl);
  w.Xbt = c.take<unsigned short>(pl);
  w.Tt = c.take<unsigned short>((size_t)lp_t_elems(n, leaf) + 512);
  w.PLhi = c.take<unsigned short>(pp);
  w.PLlo = c.take<unsigned short>(pp);
  w.PX = c.take<unsigned short>(pp);
  w.PXthi = c.take<unsigned short>(pp);
  w.PXtlo = c.take<unsigned short>(pp);
  w.PRt = c.take<unsigned short>(pp);
  w.R32 = c.take<float>((size_t)n * n);
  w.dL = c.take<double>((size_t)n);
  w.dX = c.take<double>((size_t)n);
  w.dX2 = c.take<double>((size_t)n);
  GemmBatch bt{1, 1, n, n, n, n, n, n};
  const int64_t nt = std::max<int64_t>({1, gemm_lp_tiles(bt, kLowerTiles), gemm_tiles(bt, kLowerTiles)});
  w.tile_sq = c.take<double>((size_t)nt);
  w.tile_sqx = c.take<double>((size_t)nt);
  w.partial = c.take<double>(kPart);
  w.split_sq = c.take<double>((size_t)split_tiles(n));
  w.split_dsq = c.take<double>((size_t)split_tiles(n));
  w.scal = c.take<double>(8);
  return w;
}

// Level products of the forward recursion on low-precision MFMA.
// sL, sX: power-of-two scales of the L and X planes (1 for BF16); T is stored
// with the scale of X. X above the leaf blocks is zeroed by the leaf launch.
hipError_t lp_levels(int64_t n, double* X, int64_t ldx, int64_t leaf, int f16, const WsRefine& w, double sL,
                     double sX, int x_round, hipStream_t s) {
  const int64_t ldp = w.ldp;
  for (const Level& lv : levels_of(n, leaf)) {
    const int64_t hA = lv.hA, span = lv.span, ldt = t_ld(hA);
    const int64_t stp = span * (ldp + 1), stx = span * (ldx + 1);
    const double fh = (double)hA, hB = (double)lv.hB_last, full = (double)(lv.nmerge - 1);
    // T = C * A^-1 (stored transposed)
    LpGemmArgs g1{};
    g1.A_hi = w.Lhi + hA * ldp;  // C
    g1.lda = ldp;
    g1.a_bstride = stp;
    g1.Bt_hi = w.Xbt;  // (A^-1)^T rows = A^-1 columns
    g1.ldb = ldp;
    g1.b_bstride = stp;
    g1.bt = {lv.nmerge, 1, hA, hA, hA, lv.hB_last, hA, hA};
    g1.alpha = 1.0 / sL;  // acc = (sL C)(sX A^-1); T is kept scaled by sX
    g1.lp_scale = 1.0;
    g1.Ot = w.Tt;
    g1.ldot = ldt;
    g1.ot_bstride = hA * ldt;
    LpConfig c1{f16, 1, 0, 1, kAllTiles, kColAsc, kLoN0, kHiK, kLpEpT};
    hipError_t e;
    {
      ProfLaunch pl(f16 ? "f16_level_T" : "bf16_level_T", full * fh * fh * (fh + 1) + hB * fh * (fh + 1),
                    2.0 * (full * 2.5 * fh * fh + (2 * hB * fh + fh * fh / 2)), s);
      e = launch_gemm_lp(g1, c1, s);
    }
    if (e != hipSuccess) return e;
    // X21 = -B^-1 * T
    LpGemmArgs g2{};
    g2.A_hi = w.Xb + hA * ldp + hA;  // B^-1 row-major
    g2.lda = ldp;
    g2.a_bstride = stp;
    g2.Bt_hi = w.Tt;
    g2.ldb = ldt;
    g2.b_bstride = hA * ldt;
    g2.bt = {lv.nmerge, 1, hA, hA, hA, lv.hB_last, hA, lv.hB_last};
    g2.alpha = -1.0 / (sX * sX);  // acc = (sX B^-1)(sX T)
    g2.lp_scale = sX;
    g2.X = X + hA * ldx;
    g2.ldx = ldx;
    g2.x_bstride = stx;
    g2.Xlp = w.Xb + hA * ldp;
    g2.ldxlp = ldp;
    g2.xlp_bstride = stp;
    g2.Xlpt = w.Xbt + hA;
    g2.ldxlpt = ldp;
    g2.xlpt_bstride = stp;
    g2.x_round = x_round;
    LpConfig c2{f16, 1, 1, 0, kAllTiles, kRowDesc, kLoZero, kHiM1, kLpEpX21};
    {
      ProfLaunch pl(f16 ? "f16_level_X21" : "bf16_level_X21", full * fh * fh * (fh + 1) + fh * hB * (hB + 1),
                    full * (2 * (fh * fh / 2 + fh * fh) + 12 * fh * fh) + (2 * (hB * hB / 2 + hB * fh) + 12 * hB * fh),
                    s);
      e = launch_gemm_lp(g2, c2, s);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

double tri_flops(double n) { return n * (n - 1) * (n - 2) / 3.0; }  // strictly-lower x strictly-lower

// Power of two s with m * s < 2^e (1 for m = 0 or non-finite m).
double pow2_scale(double m, int e) {
  if (!(m > 0.0) || !std::isfinite(m)) return 1.0;
  int x = 0;
  std::frexp(m, &x);  // m < 2^x
  return std::ldexp(1.0, e - x);
}

// Host copy of one reduction result.
hipError_t read_scalar(const double* d, double* h, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(h, d, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

// Frobenius norms of L and X (lower triangles), of their strictly lower
// parts N_L, N_X and of their diagonals.
struct Norms {
  double L, X, nl, nx, dl, dx;
};

Norms norms_from(const double* h6) {  // h6[2..5]: ||L||^2, ||diag L||^2, ||X||^2, ||diag X||^2
  Norms q;
  q.L = std::sqrt(h6[2]);
  q.dl = std::sqrt(h6[3]);
  q.X = std::sqrt(h6[4]);
  q.dx = std::sqrt(h6[5]);
  q.nl = std::sqrt(std::max(0.0, h6[2] - h6[3]));
  q.nx = std::sqrt(std::max(0.0, h6[4] - h6[5]));
  return q;
}

// Estimated error of rho. Split product: random-walk model, the rounding
// errors of the ~n terms of an entry adding like independent random signs,
// so that ||dR||_F is about c ||N_L||_F ||N_X||_F / sqrt(n): slices
// c = 0.5 u^2 (0.25 u^2 measured for BF16 at n = 16384) plus the FP32
// accumulation and FP16 subnormal slices, c = 2^-24 sqrt(n) / 8 (FP16 at
// n = 1000..16384 measured up to 2^-24 sqrt(n) / 12 beyond the slice term).
// FP64 product: 2^-53 per entry relative to |N_L||N_X|.
double resid_est(int f16, bool fp64, double n, const Norms& q) {
  if (fp64) return std::ldexp(1.0, -53) * q.nl * q.nx / (q.L * q.X);
  const double u = f16 ? std::ldexp(1.0, -11) : std::ldexp(1.0, -8);
  const double c = 0.5 * u * u + std::ldexp(1.0, -24) * std::sqrt(n) / 8.0;
  return c * q.nl * q.nx / (std::sqrt(n) * q.L * q.X);
}

// Worst-case bound of the same error: every rounding at its largest and in
// the same direction. Entrywise |dR| <= (slices + gamma_m (1 + 4u)) |N_L||N_X|
// + FP64 assembly, with || |N_L||N_X| ||_F <= ||N_L||_F ||N_X||_F; FP16 adds
// the absolute rounding of subnormal slice values (spacing 2^-24 of the
// scaled value). FP32 accumulation with unit roundoff 2^-23 (covers a
// truncating add). The FP64 product: gamma_n with 2^-53.
double resid_bound(int f16, int nsp, bool fp64, double n, const Norms& q, double sL, double sX, double rho) {
  const double u64 = std::ldexp(1.0, -53);
  double dr = 3.0 * u64 * (q.nl * q.nx + q.dl * q.nx + q.nl * q.dx) + u64 * std::sqrt(n);  // assembly
  if (fp64) {
    const double g = n * u64 / (1.0 - n * u64);
    dr += g * q.nl * q.nx;
  } else {
    const double u = f16 ? std::ldexp(1.0, -11) : std::ldexp(1.0, -8);
    const double slices = nsp == 2 ? u * u : 3.0 * u * u + 3.0 * u * u * u;
    const double m = nsp * n, uf = std::ldexp(1.0, -23);
    const double g = (m * uf < 1.0) ? m * uf / (1.0 - m * uf) : INFINITY;
    dr += (slices + g * (1.0 + 4.0 * u)) * q.nl * q.nx;
    if (f16) dr += std::ldexp(1.0, -24) * (1.0 + u) * n * (q.nx / sL + q.nl / sX) * (nsp == 2 ? 1.0 : 2.0);
  }
  return dr / (q.L * q.X) + 2.0 * n * n * u64 * rho;  // + the norms' own summation
}

// R = I - L X with the split product: A roles hi / lo(N_L) (w.PLhi, w.PLlo),
// B roles hi(N_X)^T (w.PXthi) and, for nsp = 3, lo(N_X)^T (w.PXtlo); FP32 R
// into R (ldr), R^T in low precision into w.PRt if write_rt, per-tile sums
// into w.tile_sq / w.tile_sqx, reduced into w.scal[0], w.scal[1].
hipError_t split_residual(int f16, int nsp, int64_t n, const double* L, int64_t ldl, const double* X, int64_t ldx,
                          const double* dx, const WsRefine& w, double sL, double sX, float* R, int64_t ldr,
                          bool write_rt, hipStream_t s) {
  const double dn = (double)n;
  GemmBatch bt{1, 1, n, n, n, n, n, n};
  LpGemmArgs gr{};
  gr.A_hi = w.PLhi;
  gr.A_lo = w.PLlo;
  gr.lda = w.kb;
  gr.Bt_hi = w.PXthi;
  gr.Bt_lo = nsp == 3 ? w.PXtlo : nullptr;
  gr.ldb = w.kb;
  gr.bt = bt;
  gr.alpha = 1.0 / (sL * sX);  // acc = (sL N_L)(sX N_X)
  gr.lp_scale = 1.0;
  gr.X = (double*)X;
  gr.ldx = ldx;
  gr.L = L;
  gr.ldl = ldl;
  gr.dL = w.dL;
  gr.dX = dx;
  gr.R32 = R;
  gr.ldr = ldr;
  gr.Rt = write_rt ? w.PRt : nullptr;
  gr.ldrt = w.kb;
  gr.tile_sq = w.tile_sq;
  gr.tile_sqx = w.tile_sqx;
  LpConfig cr{f16, nsp, 0, 0, kLowerTiles, kDiagDesc, kLoN0Pb, kHiM1, kLpEpResid};
  hipError_t e;
  {
    ProfLaunch pl(nsp == 2 ? (f16 ? "f16_residual2" : "bf16_residual2") : (f16 ? "f16_residual" : "bf16_residual"),
                  nsp * tri_flops(dn), dn * dn / 2 * ((nsp + 1) * 2 + 8 + 8 + 4 + 2), s);
    e = launch_gemm_lp(gr, cr, s);
  }
  if (e != hipSuccess) return e;
  const int64_t ntl = gemm_lp_tiles(bt, kLowerTiles);
  if ((e = launch_reduce_sum(w.tile_sq, ntl, w.scal + 0, s)) != hipSuccess) return e;
  return launch_reduce_sum(w.tile_sqx, ntl, w.scal + 1, s);
}

// Zero bands of the six panel-blocked planes (see launch_zero_band_pb): the
// residual and correction products read each 256-row panel up to the end of
// its diagonal 256 x 256 block, up to kBand columns past the 64 x 64 tiles
// the splits and epilogues write.
hipError_t zero_bands(const WsRefine& w, int64_t n, hipStream_t s) {
  void* planes[6] = {w.PLhi, w.PLlo, w.PX, w.PXthi, w.PXtlo, w.PRt};
  const int right[6] = {1, 1, 1, 0, 0, 0};
  return launch_zero_band_pb(planes, right, 6, w.kb, n, kBand, s);
}

}  // namespace

size_t refine_workspace_bytes(int mode, int64_t n, const trinv_opts& o, int64_t leaf) {
  (void)mode;
  if (n <= 0 || !refine_order_ok(n)) return 0;
  Carve c(nullptr, 0);
  carve_refine(c, n, leaf);
  if (o.upper) c.take<double>((size_t)n * n);  // the transposed input
  return c.used;
}

bool refine_order_ok(int64_t n) { return n <= kMaxRefineOrder; }

int refine_inverse(int mode, int64_t n, const double* L, int64_t ldl, double* X, int64_t ldx, const trinv_opts& o,
                   int64_t leaf, void* ws, size_t ws_bytes, hipStream_t s, trinv_info* info) {
  if (!refine_order_ok(n)) return TRINV_ERR_UNSUPPORTED;
  if (leaf < 32) return TRINV_ERR_ARG;
  if (o.resid < TRINV_RESID_AUTO || o.resid > TRINV_RESID_FP64) return TRINV_ERR_ARG;
  const int f16 = mode == TRINV_F16_REFINE;
  Carve c(ws, ws_bytes);
  WsRefine w = carve_refine(c, n, leaf);
  double* Ut = o.upper ? c.take<double>((size_t)n * n) : nullptr;
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  const int64_t ldp = w.ldp;
  const double dn = (double)n;

  // An upper input is inverted through its transpose (Section 2: the two
  // cases are transposes of each other): L = U^T (lower), X = L^-1, and the
  // result X^T = U^-1 is transposed in place at the end.
  if (o.upper) {
    HIP_TRY(launch_transpose<double>(L, ldl, Ut, n, n, s));
    L = Ut;
    ldl = n;
  }
  auto finish = [&](int st) -> int {
    if (o.upper && (st == TRINV_OK || st == TRINV_ERR_NOT_CONVERGED))
      if (launch_transpose_inplace<double>(X, ldx, n, s) != hipSuccess) return TRINV_ERR_HIP;
    return st;
  };

  HIP_TRY(launch_fill_u64(w.status, ~0ull, 1, s));
  HIP_TRY(zero_bands(w, n, s));
  // FP16 planes carry one power-of-two scale each (exact, undone through the
  // epilogues' alpha) so that the values sit in FP16's normal range; BF16 has
  // the exponent range of FP32 and uses 1. L: from max |L|; X during the
  // forward: from 1 / min |L_ii| (the diagonal of X) with 2^5 of headroom;
  // X during refinement: from max |X|; R: from ||R||_F (>= max |R_ij|).
  double sL = 1.0, sXf = 1.0;
  if (f16) {
    double mx = 0.0;
    HIP_TRY(launch_maxabs<double>(L, n, ldl, 1, o.unit_diag, w.partial, kPart, w.scal + 6, s));
    HIP_TRY(read_scalar(w.scal + 6, &mx, s));
    sL = pow2_scale(mx, 14);
  }
  {  // staging: L -> hi / lo slices (row-major) and diag(L)
    ProfLaunch pl("split", 0.0, dn * dn / 2 * (8 + 4), s);
    // strictly lower part: the diagonal enters the residual in FP64 only
    SplitOut so{};
    so.hi = w.Lhi;  // row-major hi(L) for the forward products
    so.ldo = ldp;
    so.hi_b = w.PLhi;  // panel-blocked hi / lo for the residual
    so.lo_b = w.PLlo;
    so.kb = w.kb;
    so.sq = w.split_sq;  // ||tril(L)||^2 and the diagonal's part, per tile
    so.dsq = w.split_dsq;
    HIP_TRY(launch_split(L, ldl, n, f16, so, w.dL, o.unit_diag, 1, sL, s));
  }
  // ||tril(L)||^2 and sum of diag(L)^2 (L is read once, by the split)
  HIP_TRY(launch_reduce_sum(w.split_sq, split_tiles(n), w.scal + 2, s));
  HIP_TRY(launch_reduce_sum(w.split_dsq, split_tiles(n), w.scal + 3, s));
  if (f16) {
    std::vector<double> d((size_t)n);
    HIP_TRY(hipMemcpyAsync(d.data(), w.dL, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double mn = INFINITY;
    for (double v : d) mn = std::min(mn, std::fabs(v));
    if (mn > 0.0) sXf = pow2_scale(1.0 / mn, 11);
  }
  // The first iterate X0 keeps its FP64 diagonal and takes its low-precision
  // copies' values (divided by their scale) everywhere below it, so its hi
  // slice under the same scale holds it exactly and the first residual needs
  // two products, (hi(N_L) + lo(N_L)) hi(N_X).
  const int x0_exact = 1;
  {  // leaves in FP64, with row-major and transposed low-precision copies
    const double nl = (double)((n + leaf - 1) / leaf), b = (double)leaf;
    ProfLaunch pl("leaf_f64", nl * b * b * b / 3.0, nl * b * b * (8 + 8 + 4) + dn * dn / 2 * 8, s);
    HIP_TRY(launch_leaf<double>(n, L, ldl, X, ldx, 0, 1, (int)leaf, o.unit_diag, w.Xb, w.Xbt, f16, ldp, sXf,
                                w.status, 0, s, x0_exact, 1));
  }
  HIP_TRY(lp_levels(n, X, ldx, leaf, f16, w, sL, sXf, x0_exact, s));

  GemmBatch bt{1, 1, n, n, n, n, n, n};
  int iter = 0;
  double rho = 0.0;
  // Precision of the residual's O(n^3) product (opts.resid): the split
  // product's error is estimated by resid_est; AUTO uses it only while that
  // estimate is at most half the tolerance (decided once, from the first
  // iterate's norms), otherwise FP64 MFMA.
  int resid_fp64 = o.resid == TRINV_RESID_FP64 ? 1 : -1;
  Norms q{};
  bool have_norms = false;
  // diag(X) in use and the spare buffer a fused correction writes the next
  // one into (it reads the current one).
  double *dx = w.dX, *dx_next = w.dX2;
  bool x_sliced = false;  // B-role slices and diagonal of the current X written by the correction
  bool px_stale = false;  // the A-role slice (read by the correction only) lags behind X
  for (;;) {
    // residual of the current X
    // the forward's X0 is exact in its hi slice under the forward's scale:
    // no lo slice, two products
    const bool x_hi_exact = x0_exact && iter == 0;
    double sX = x_hi_exact ? sXf : 1.0;
    if (f16 && !x_hi_exact) {
      double mx = 0.0;
      HIP_TRY(launch_maxabs<double>(X, n, ldx, 1, 0, w.partial, kPart, w.scal + 6, s));
      HIP_TRY(read_scalar(w.scal + 6, &mx, s));
      sX = pow2_scale(mx, 14);
    }
    if (!x_sliced) {
      ProfLaunch pl("split", 0.0, dn * dn / 2 * (x_hi_exact ? 2 + 4 : 8 + 6), s);
      SplitOut so{};
      so.hi_b = w.PX;  // A role of the correction
      so.hi_tb = w.PXthi;  // B role of the residual
      so.lo_tb = x_hi_exact ? nullptr : w.PXtlo;
      so.kb = w.kb;
      if (!have_norms) {  // the norms of X for the precision decision, from the split's read
        so.sq = w.split_sq;
        so.dsq = w.split_dsq;
      }
      if (x_hi_exact)  // X0's strictly lower values are its low-precision copy over sX, exactly
        HIP_TRY(launch_split_lp_source(X, ldx, w.Xb, ldp, n, f16, so, dx, sX, s));
      else
        HIP_TRY(launch_split(X, ldx, n, f16, so, dx, 0, 1, sX, s));
      px_stale = false;
    }
    // The norms of X (first iterate): AUTO needs them to choose the
    // residual's precision before launching it (one wait); with the
    // precision fixed by the options they are read in the same wait as the
    // residual's sums.
    bool norms_pending = false;
    if (!have_norms) {
      HIP_TRY(launch_reduce_sum(w.split_sq, split_tiles(n), w.scal + 4, s));
      HIP_TRY(launch_reduce_sum(w.split_dsq, split_tiles(n), w.scal + 5, s));
      if (o.resid == TRINV_RESID_SPLIT) resid_fp64 = 0;
      if (resid_fp64 < 0) {
        double h6[6];
        HIP_TRY(hipMemcpyAsync(h6, w.scal, sizeof(h6), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        q = norms_from(h6);
        have_norms = true;
        resid_fp64 = resid_est(f16, false, dn, q) <= 0.5 * o.tol ? 0 : 1;
      } else {
        norms_pending = true;
      }
    }
    const int nsp = x_hi_exact ? 2 : 3;
    auto residual = [&](bool fp64) -> hipError_t {
      if (fp64) {
        GemmArgs<double> gf{};
        gf.A = {L, ldl, 0, 0};
        gf.amask = 2;
        gf.B = {X, ldx, 0, 0};
        gf.bmask = 2;
        gf.alpha = 1.0;
        gf.tiles = kLowerTiles;
        gf.order = kDiagDesc;
        gf.klo = kLoN0;
        gf.khi = kHiM1;
        gf.bt = bt;
        gf.refine_resid = 1;
        gf.Lfull = L;
        gf.ldl = ldl;
        gf.Xfull = X;
        gf.ldx = ldx;
        gf.dL = w.dL;
        gf.dX = dx;
        gf.R32 = w.R32;
        gf.ldr = n;
        gf.Rt = nullptr;  // R^T for the correction is cast from R32 below
        gf.ldrt = 0;
        gf.lp_is_f16 = f16;
        gf.tile_sq = w.tile_sq;
        gf.tile_sqx = w.tile_sqx;
        {
          ProfLaunch pl("f64_residual", tri_flops(dn), dn * dn / 2 * (8 * 2 + 8 + 8 + 4 + 2), s);
          hipError_t e = launch_gemm<double, double>(gf, s);
          if (e != hipSuccess) return e;
        }
        const int64_t ntf = gemm_tiles(bt, kLowerTiles);
        hipError_t e = launch_reduce_sum(w.tile_sq, ntf, w.scal + 0, s);
        if (e != hipSuccess) return e;
        return launch_reduce_sum(w.tile_sqx, ntf, w.scal + 1, s);
      }
      // BF16: R^T leaves in the epilogue; FP16: written below, once ||R|| is known
      return split_residual(f16, nsp, n, L, ldl, X, ldx, dx, w, sL, sX, w.R32, n, !f16, s);
    };
    HIP_TRY(residual(resid_fp64 == 1));
    // the norms, and after the forward the leaves' zero-pivot index, in one
    // wait for the stream
    double h[6];
    uint64_t bad = ~0ull;
    HIP_TRY(hipMemcpyAsync(h, w.scal, (norms_pending ? 6 : 3) * sizeof(double), hipMemcpyDeviceToHost, s));
    if (iter == 0) HIP_TRY(hipMemcpyAsync(&bad, w.status, sizeof(bad), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (iter == 0) {
      if (bad != ~0ull && bad <= (uint64_t)n) {
        if (info) info->first_bad_index = (int64_t)bad;
        return TRINV_ERR_SINGULAR;
      }
    }
    if (norms_pending) {
      q = norms_from(h);
      have_norms = true;
    }
    rho = std::sqrt(h[0]) / (std::sqrt(h[2]) * std::sqrt(h[1]));
    const double est = resid_est(f16, resid_fp64 != 0, dn, q);
    if (info) {
      info->rel_residual = rho;
      info->iterations = iter;
      info->resid_error_est = est;
      info->resid_error_bound = resid_bound(f16, nsp, resid_fp64 != 0, dn, q, sL, sX, rho);
    }
    if (!std::isfinite(rho)) return TRINV_ERR_NONFINITE;
    if (rho + est <= o.tol) return finish(TRINV_OK);
    if (iter >= o.max_iter) return finish(TRINV_ERR_NOT_CONVERGED);
    double sR = 1.0;
    if (f16 || resid_fp64) {  // R^T for the correction's B operand (FP16: scaled by ||R||_F)
      if (f16) sR = pow2_scale(std::sqrt(h[0]), 14);
      SplitOut so{};
      so.hi_tb = w.PRt;
      so.kb = w.kb;
      ProfLaunch pl("split", 0.0, dn * dn / 2 * (4 + 2), s);
      HIP_TRY(launch_split_f32(w.R32, n, n, f16, so, sR, s));
    }
    if (px_stale) {  // a second correction after a fused one: the A-role slice of X
      ProfLaunch pl("split", 0.0, dn * dn / 2 * (8 + 2), s);
      SplitOut so{};
      so.hi_b = w.PX;
      so.kb = w.kb;
      HIP_TRY(launch_split(X, ldx, n, f16, so, nullptr, 0, 1, sX, s));
      px_stale = false;
    }
    // correction: X <- X + D_X R + N_X R
    LpGemmArgs gc{};
    gc.A_hi = w.PX;
    gc.lda = w.kb;
    gc.Bt_hi = w.PRt;
    gc.ldb = w.kb;
    gc.bt = bt;
    gc.alpha = 1.0 / (sX * sR);  // acc = (sX N_X)(sR R)
    gc.lp_scale = 1.0;
    gc.X = X;
    gc.ldx = ldx;
    gc.dX = dx;
    gc.R32 = w.R32;
    gc.ldr = n;
    // BF16 with interior tiles only: the correction also writes the slices of
    // the new X for the next residual (the split would re-read all of X)
    const bool fuse = !f16 && !resid_fp64 && n % 256 == 0;
    if (fuse) {
      gc.Xn_tb_hi = w.PXthi;  // read by the residual only, not by the correction
      gc.Xn_tb_lo = w.PXtlo;
      gc.dXn = dx_next;
      gc.kbx = w.kb;
    }
    LpConfig cc{f16, 1, 0, 0, kLowerTiles, kDiagDesc, kLoN0Pb, kHiM1, kLpEpCorr};
    {
      ProfLaunch pl(f16 ? "f16_correction" : "bf16_correction", tri_flops(dn) + dn * dn,
                    dn * dn / 2 * (2 + 2 + 4 + 16 + (fuse ? 4 : 0)), s);
      HIP_TRY(launch_gemm_lp(gc, cc, s));
    }
    if (fuse) std::swap(dx, dx_next);
    x_sliced = fuse;
    px_stale = fuse;
    ++iter;
  }
}

}  // namespace trinv

// ---------------------------------------------------------------- residual helper
using namespace trinv;

extern "C" size_t trinv_refine_residual_workspace_bytes(int mode, int64_t n) {
  (void)mode;
  if (n <= 0 || !refine_order_ok(n)) return 0;
  Carve c(nullptr, 0);
  carve_refine(c, n, 64);
  return c.used;
}

extern "C" int trinv_refine_residual(int mode, int64_t n, const void* Lv, int64_t ldl, const void* Xv, int64_t ldx,
                                     int32_t nsplit, float* R, int64_t ldr, void* ws, size_t ws_bytes,
                                     trinv_stream_t stream, double* out_host) {
  if (n < 0 || ldl < n || ldx < n || ldr < n || !out_host) return TRINV_ERR_ARG;
  for (int i = 0; i < 5; ++i) out_host[i] = 0.0;
  if (n == 0) return TRINV_OK;
  if (!Lv || !Xv || !R) return TRINV_ERR_ARG;
  if (mode != TRINV_BF16_REFINE && mode != TRINV_F16_REFINE) return TRINV_ERR_UNSUPPORTED;
  if (nsplit != 2 && nsplit != 3) return TRINV_ERR_ARG;
  if (!refine_order_ok(n)) return TRINV_ERR_UNSUPPORTED;
  const double* L = (const double*)Lv;
  const double* X = (const double*)Xv;
  if (overlaps(R, span_bytes(n, n, ldr, 4), L, span_bytes(n, n, ldl, 8)) ||
      overlaps(R, span_bytes(n, n, ldr, 4), X, span_bytes(n, n, ldx, 8)))
    return TRINV_ERR_ARG;
  const int f16 = mode == TRINV_F16_REFINE;
  Carve c(ws, ws_bytes);
  WsRefine w = carve_refine(c, n, 64);
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(zero_bands(w, n, s));
  double sL = 1.0, sX = 1.0;
  if (f16) {  // as the refinement loop scales them: from max |L| and max |X|
    double mx = 0.0;
    HIP_TRY(launch_maxabs<double>(L, n, ldl, 1, 0, w.partial, kPart, w.scal + 6, s));
    HIP_TRY(read_scalar(w.scal + 6, &mx, s));
    sL = pow2_scale(mx, 14);
    HIP_TRY(launch_maxabs<double>(X, n, ldx, 1, 0, w.partial, kPart, w.scal + 6, s));
    HIP_TRY(read_scalar(w.scal + 6, &mx, s));
    sX = pow2_scale(mx, 14);
  }
  SplitOut sl{};
  sl.hi_b = w.PLhi;
  sl.lo_b = w.PLlo;
  sl.kb = w.kb;
  sl.sq = w.split_sq;
  sl.dsq = w.split_dsq;
  HIP_TRY(launch_split(L, ldl, n, f16, sl, w.dL, 0, 1, sL, s));
  HIP_TRY(launch_reduce_sum(w.split_sq, split_tiles(n), w.scal + 2, s));
  HIP_TRY(launch_reduce_sum(w.split_dsq, split_tiles(n), w.scal + 3, s));
  SplitOut sx{};
  sx.hi_tb = w.PXthi;
  sx.lo_tb = nsplit == 3 ? w.PXtlo : nullptr;
  sx.kb = w.kb;
  sx.sq = w.split_sq;
  sx.dsq = w.split_dsq;
  HIP_TRY(launch_split(X, ldx, n, f16, sx, w.dX, 0, 1, sX, s));
  HIP_TRY(launch_reduce_sum(w.split_sq, split_tiles(n), w.scal + 4, s));
  HIP_TRY(launch_reduce_sum(w.split_dsq, split_tiles(n), w.scal + 5, s));
  HIP_TRY(split_residual(f16, nsplit, n, L, ldl, X, ldx, w.dX, w, sL, sX, R, ldr, !f16, s));
  double h6[6];
  HIP_TRY(hipMemcpyAsync(h6, w.scal, sizeof(h6), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const Norms q = norms_from(h6);
  out_host[0] = std::sqrt(h6[0]);
  out_host[1] = std::sqrt(h6[2]);
  out_host[2] = std::sqrt(h6[1]);
  const double rho = out_host[0] / (out_host[1] * out_host[2]);
  out_host[3] = resid_est(f16, false, (double)n, q);
  out_host[4] = resid_bound(f16, nsplit, false, (double)n, q, sL, sX, rho);
  return TRINV_OK;
}
