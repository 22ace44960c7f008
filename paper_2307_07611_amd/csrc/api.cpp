// C ABI of libtrinv and the recursion scheduler.
//
// The scheduler runs the paper's 2x2 block recursion (Section 4.1, algorithm
// COMBRIT with beta = 2) bottom-up: first every leaf (order `leaf`) is
// inverted by the column recurrence (one launch), then level d = 0, 1, ...
// merges pairs of neighbouring inverted blocks of order hA = leaf * 2^d into
// blocks of order 2 hA with two tile-product launches per level:
//     T   =  C * A^-1       (all merges of the level in one launch)
//     X21 = -B^-1 * T       (ditto; also zeroes the block above the diagonal)
// For n that is not leaf * 2^k the last leaf and the last block of each level
// are shorter; every such split gives the same inverse in exact arithmetic.
#include "api_internal.h"
#include "profile.h"

#include <algorithm>
#include <cmath>
#include <cstring>

using namespace trinv;

namespace trinv {

trinv_opts resolve_opts(const trinv_opts* o) {
  trinv_opts r;
  trinv_default_opts(&r);
  if (o) r = *o;
  if (r.max_iter < 0) r.max_iter = 0;
  if (!(r.tol > 0)) r.tol = 1e-12;
  return r;
}

// beta > 2 selects the COMBRIT top level (0 and 2: binary recursion).
bool combrit_beta(const trinv_opts& o) { return o.beta > 2; }

int default_leaf(int mode, int64_t n) {
  if (mode == TRINV_BF16_REFINE || mode == TRINV_F16_REFINE) return n >= 4096 ? 128 : 64;
  if (mode == TRINV_F32) return n <= 512 ? 32 : 64;
  if (n <= 1024) return 32;
  if (n <= 8192) return 64;
  return 128;
}

bool valid_leaf(int64_t b) { return b == 16 || b == 32 || b == 64 || b == 128; }

std::vector<Level> levels_of(int64_t n, int64_t leaf) {
  std::vector<Level> v;
  for (int64_t hA = leaf; hA < n; hA *= 2) {
    Level l;
    l.hA = hA;
    l.span = 2 * hA;
    l.nmerge = (n - hA + l.span - 1) / l.span;
    const int64_t o_last = (l.nmerge - 1) * l.span;
    l.hB_last = std::min(hA, n - o_last - hA);
    v.push_back(l);
  }
  return v;
}

int64_t t_elems(int64_t n, int64_t leaf) {
  int64_t m = 0;
  for (const Level& l : levels_of(n, leaf)) m = std::max(m, l.nmerge * l.hA * l.hA);
  return m;
}

template <typename T, typename TC>
hipError_t run_levels(int64_t n, const T* L, int64_t ldl, T* X, int64_t ldx, int64_t stride, int64_t batch,
                      int64_t leaf, T* Tws, hipStream_t s) {
  const int64_t tbatch = t_elems(n, leaf);
  for (const Level& lv : levels_of(n, leaf)) {
    const int64_t hA = lv.hA, st_l = lv.span * (ldl + 1), st_x = lv.span * (ldx + 1);
    GemmArgs<T> g1{};
    g1.A = {L + hA * ldl, ldl, st_l, stride};  // C = L21 of each merge
    g1.B = {X, ldx, st_x, stride};             // A^-1
    g1.D = {Tws, hA, hA * hA, tbatch};
    g1.alpha = 1.0;  // A^-1 has exact zeros above its diagonal: no mask needed
    g1.tiles = kAllTiles;
    g1.order = kColAsc;
    g1.klo = kLoN0;
    g1.khi = kHiK;
    g1.bt = {lv.nmerge, batch, hA, hA, hA, lv.hB_last, hA, hA};
    // Algorithmic work of a level: per merge hB*hA*(hA+1) flops for C*A^-1 and
    // hA*hB*(hB+1) for B^-1*T; bytes: read C, A^-1, B^-1 (triangles), write X21.
    const double es = sizeof(T);
    const int64_t full = (lv.nmerge - 1) * batch;
    const double hB = (double)lv.hB_last, fh = (double)hA;
    const double fl1 = ((double)full * fh * fh * (fh + 1) + (double)batch * hB * fh * (fh + 1));
    const double fl2 = ((double)full * fh * fh * (fh + 1) + (double)batch * fh * hB * (hB + 1));
    const double by1 = es * ((double)full * (fh * fh + fh * fh / 2 + fh * fh) + (double)batch * (hB * fh + fh * fh / 2 + hB * fh));
    const double by2 = es * ((double)full * (fh * fh / 2 + fh * fh + 2 * fh * fh) + (double)batch * (hB * hB / 2 + hB * fh + 2 * hB * fh));
    // one profile class per kernel instantiation
    const char* cls1 = sizeof(T) == 8 ? "f64_level_T" : "f32_level_T";
    const char* cls2 = sizeof(T) == 8 ? "f64_level_X21" : "f32_level_X21";
    hipError_t e;
    {
      ProfLaunch pl(cls1, fl1, by1, s);
      e = launch_gemm<T, TC>(g1, s);
    }
    if (e != hipSuccess) return e;
    GemmArgs<T> g2{};
    g2.A = {X + hA * ldx + hA, ldx, st_x, stride};  // B^-1
    g2.B = {Tws, hA, hA * hA, tbatch};
    g2.D = {X + hA * ldx, ldx, st_x, stride};       // X21
    g2.Zmirror = {X + hA, ldx, st_x, stride};       // X12 = 0
    g2.alpha = -1.0;  // B^-1 has exact zeros above its diagonal: no mask needed
    g2.tiles = kAllTiles;
    g2.order = kRowDesc;
    g2.klo = kLoZero;
    g2.khi = kHiM1;
    g2.bt = {lv.nmerge, batch, hA, hA, hA, lv.hB_last, hA, lv.hB_last};
    {
      ProfLaunch pl(cls2, fl2, by2, s);
      e = launch_gemm<T, TC>(g2, s);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t run_levels<double, double>(int64_t, const double*, int64_t, double*, int64_t, int64_t, int64_t,
                                               int64_t, double*, hipStream_t);
template hipError_t run_levels<float, float>(int64_t, const float*, int64_t, float*, int64_t, int64_t, int64_t,
                                             int64_t, float*, hipStream_t);

int wait_status(hipStream_t s, const uint64_t* status_dev, int64_t n, int64_t* first_bad) {
  if (hipStreamSynchronize(s) != hipSuccess) return TRINV_ERR_HIP;
  uint64_t bad = ~0ull;
  if (hipMemcpy(&bad, status_dev, sizeof(bad), hipMemcpyDeviceToHost) != hipSuccess) return TRINV_ERR_HIP;
  const int64_t idx = (bad == ~0ull || bad > (uint64_t)n) ? 0 : (int64_t)bad;
  if (first_bad) *first_bad = idx;
  return idx ? TRINV_ERR_SINGULAR : TRINV_OK;
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const char* a0 = (const char*)a;
  const char* b0 = (const char*)b;
  return a0 < b0 + bbytes && b0 < a0 + abytes;
}

size_t span_bytes(int64_t rows, int64_t cols, int64_t ld, size_t es) {
  if (rows <= 0 || cols <= 0) return 0;
  return (size_t)((rows - 1) * ld + cols) * es;
}

}  // namespace trinv

namespace {

constexpr int64_t kPartials = 4096;

struct WsPlain {
  uint64_t* status;
  unsigned* nonfinite;  // blocking calls: set if X holds a NaN or an infinity
  void* T;
  void* Ut;  // transposed input (upper mode)
  void* Xt;  // transposed output (upper mode)
};

WsPlain carve_plain(Carve& c, int mode, int64_t n, int64_t leaf, bool upper) {
  WsPlain w;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  w.status = c.take<uint64_t>(1);
  w.nonfinite = c.take<unsigned>(1);
  w.T = c.take<char>(es * (size_t)t_elems(n, leaf));
  w.Ut = upper ? (void*)c.take<char>(es * (size_t)n * n) : nullptr;
  w.Xt = upper ? (void*)c.take<char>(es * (size_t)n * n) : nullptr;
  return w;
}

template <typename T>
hipError_t plain_inverse(int64_t n, const T* L, int64_t ldl, T* X, int64_t ldx, const trinv_opts& o, int64_t leaf,
                         const WsPlain& w, hipStream_t s) {
  const T* Lin = L;
  int64_t ldin = ldl;
  T* Xout = X;
  int64_t ldout = ldx;
  hipError_t e;
  if (o.upper) {
    if ((e = launch_transpose<T>(L, ldl, (T*)w.Ut, n, n, s)) != hipSuccess) return e;
    Lin = (const T*)w.Ut;
    ldin = n;
    Xout = (T*)w.Xt;
    ldout = n;
  }
  {
    const double nl = (double)((n + leaf - 1) / leaf), b = (double)leaf;
    ProfLaunch pl(sizeof(T) == 8 ? "leaf_f64" : "leaf_f32", nl * b * b * b / 3.0, nl * b * b * sizeof(T), s);
    e = launch_leaf<T>(n, Lin, ldin, Xout, ldout, 0, 1, (int)leaf, o.unit_diag, nullptr, nullptr, 0, 0, 1.0, w.status, 0, s);
  }
  if (e != hipSuccess) return e;
  if ((e = run_levels<T, T>(n, Lin, ldin, Xout, ldout, 0, 1, leaf, (T*)w.T, s)) != hipSuccess) return e;
  if (o.upper) return launch_transpose<T>(Xout, n, X, ldx, n, s);
  return hipSuccess;
}

struct WsResid {
  double* tile_sq;
  double* partial;
  double* scalars;
};

WsResid carve_resid(Carve& c, int64_t n) {
  WsResid w;
  GemmBatch bt{1, 1, n, n, n, n, n, n};
  w.tile_sq = c.take<double>((size_t)std::max<int64_t>(1, gemm_tiles(bt, kAllTiles)));
  w.partial = c.take<double>(kPartials);
  w.scalars = c.take<double>(4);
  return w;
}

template <typename T>
int residual_t(int64_t n, const T* L, int64_t ldl, const T* X, int64_t ldx, const WsResid& w, hipStream_t s,
               double* out3) {
  GemmArgs<T> g{};
  g.A = {L, ldl, 0, 0};
  g.B = {X, ldx, 0, 0};
  g.D = {nullptr, 0, 0, 0};
  g.alpha = 1.0;
  g.amask = 1;  // tril(L): the strict upper part of the input is not part of L
  g.tiles = kAllTiles;
  g.order = kRowDesc;
  g.klo = kLoZero;
  g.khi = kHiM1;
  g.subtract_identity = 1;
  g.tile_sq = w.tile_sq;
  g.bt = {1, 1, n, n, n, n, n, n};
  HIP_TRY(launch_gemm<T, double>(g, s));
  HIP_TRY(launch_reduce_sum(w.tile_sq, gemm_tiles(g.bt, kAllTiles), w.scalars + 0, s));
  HIP_TRY(launch_sumsq<T>(L, n, ldl, 1, 0, w.partial, kPartials, w.scalars + 1, s));
  HIP_TRY(launch_sumsq<T>(X, n, ldx, 0, 0, w.partial, kPartials, w.scalars + 2, s));
  double h[3];
  HIP_TRY(hipMemcpyAsync(h, w.scalars, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < 3; ++i) out3[i] = std::sqrt(h[i]);
  return TRINV_OK;
}

}  // namespace

// ---------------------------------------------------------------- C ABI
extern "C" {

void trinv_default_opts(trinv_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_iter = 4;
  o->tol = 1e-12;
}

const char* trinv_status_string(int s) {
  switch (s) {
    case TRINV_OK: return "ok";
    case TRINV_ERR_ARG: return "invalid argument";
    case TRINV_ERR_SINGULAR: return "singular: exact zero diagonal entry";
    case TRINV_ERR_NONFINITE: return "non-finite value in the result";
    case TRINV_ERR_NOT_CONVERGED: return "refinement did not reach the tolerance";
    case TRINV_ERR_HIP: return "HIP runtime error";
    case TRINV_ERR_UNSUPPORTED: return "unsupported mode or size";
    case TRINV_ERR_WORKSPACE: return "workspace too small";
    default: return "unknown status";
  }
}

size_t trinv_residual_workspace_bytes(int mode, int64_t n) {
  (void)mode;
  if (n <= 0) return 0;
  Carve c(nullptr, 0);
  carve_resid(c, n);
  return c.used;
}

int trinv_residual(int mode, int64_t n, const void* L, int64_t ldl, const void* X, int64_t ldx, void* ws,
                   size_t ws_bytes, trinv_stream_t stream, double* out_host) {
  if (n < 0 || ldl < n || ldx < n || !out_host) return TRINV_ERR_ARG;
  if (n == 0) {
    out_host[0] = out_host[1] = out_host[2] = 0.0;
    return TRINV_OK;
  }
  if (!L || !X) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32) return TRINV_ERR_UNSUPPORTED;
  Carve c(ws, ws_bytes);
  WsResid w = carve_resid(c, n);
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (mode == TRINV_F64) return residual_t<double>(n, (const double*)L, ldl, (const double*)X, ldx, w, s, out_host);
  return residual_t<float>(n, (const float*)L, ldl, (const float*)X, ldx, w, s, out_host);
}

size_t trinv_workspace_bytes(int mode, int64_t n, const trinv_opts* opts) {
  if (n <= 0) return 0;
  const trinv_opts o = resolve_opts(opts);
  const int64_t leaf = o.leaf ? o.leaf : default_leaf(mode, n);
  if (mode == TRINV_BF16_REFINE || mode == TRINV_F16_REFINE) return refine_workspace_bytes(mode, n, o, leaf);
  Carve c(nullptr, 0);
  if (combrit_beta(o) && n % o.beta == 0) {
    c.take<uint64_t>(1);
    c.take<unsigned>(1);
    c.take<char>(combrit_workspace_bytes(mode, n, o.beta, leaf));
  } else {
    carve_plain(c, mode, n, leaf, o.upper != 0);
  }
  if (o.check) carve_resid(c, n);
  return c.used;
}

int trinv_tril_inverse(int mode, int64_t n, const void* L, int64_t ldl, void* X, int64_t ldx, const trinv_opts* opts,
                       void* ws, size_t ws_bytes, trinv_stream_t stream, trinv_info* info) {
  info_reset(info);
  if (n < 0 || ldl < n || ldx < n) return TRINV_ERR_ARG;
  if (n == 0) return TRINV_OK;
  if (!L || !X) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32 && mode != TRINV_BF16_REFINE && mode != TRINV_F16_REFINE)
    return TRINV_ERR_UNSUPPORTED;
  const trinv_opts o = resolve_opts(opts);
  const int64_t leaf = o.leaf ? o.leaf : default_leaf(mode, n);
  if (!valid_leaf(leaf)) return TRINV_ERR_ARG;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  if (overlaps(L, span_bytes(n, n, ldl, es), X, span_bytes(n, n, ldx, es))) return TRINV_ERR_ARG;
  if (o.beta < 0 || o.beta == 1 || o.beta > 16) return TRINV_ERR_ARG;
  if (o.resid < TRINV_RESID_AUTO || o.resid > TRINV_RESID_FP64) return TRINV_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  if ((mode == TRINV_BF16_REFINE || mode == TRINV_F16_REFINE) && combrit_beta(o)) return TRINV_ERR_UNSUPPORTED;
  if (mode == TRINV_BF16_REFINE || mode == TRINV_F16_REFINE)
    return refine_inverse(mode, n, (const double*)L, ldl, (double*)X, ldx, o, leaf, ws, ws_bytes, s, info);

  Carve c(ws, ws_bytes);
  WsPlain w{};
  void* cw = nullptr;
  size_t cw_bytes = 0;
  if (combrit_beta(o)) {
    if (n % o.beta != 0 || ldl != ldx) return TRINV_ERR_ARG;
    if (o.upper) return TRINV_ERR_UNSUPPORTED;
    w.status = c.take<uint64_t>(1);
    w.nonfinite = c.take<unsigned>(1);
    cw_bytes = combrit_workspace_bytes(mode, n, o.beta, leaf);
    cw = c.take<char>(cw_bytes);
  } else {
    w = carve_plain(c, mode, n, leaf, o.upper != 0);
  }
  WsResid wr{};
  if (o.check) wr = carve_resid(c, n);
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  HIP_TRY(launch_fill_u64(w.status, ~0ull, 1, s));
  if (cw && mode == TRINV_F64)
    HIP_TRY(combrit_t<double>(n, (const double*)L, ldl, (double*)X, o.unit_diag, o.beta, leaf, cw, cw_bytes,
                              w.status, s));
  else if (cw)
    HIP_TRY(combrit_t<float>(n, (const float*)L, ldl, (float*)X, o.unit_diag, o.beta, leaf, cw, cw_bytes, w.status,
                             s));
  else if (mode == TRINV_F64)
    HIP_TRY(plain_inverse<double>(n, (const double*)L, ldl, (double*)X, ldx, o, leaf, w, s));
  else
    HIP_TRY(plain_inverse<float>(n, (const float*)L, ldl, (float*)X, ldx, o, leaf, w, s));
  if (!o.blocking) return TRINV_OK;
  // a NaN or an infinity in L (or an overflow) shows in X
  HIP_TRY(launch_zero(w.nonfinite, sizeof(unsigned), s));
  if (mode == TRINV_F64)
    HIP_TRY(launch_nonfinite<double>((const double*)X, n, ldx, w.nonfinite, s));
  else
    HIP_TRY(launch_nonfinite<float>((const float*)X, n, ldx, w.nonfinite, s));
  int64_t bad = 0;
  int st = wait_status(s, w.status, n, &bad);
  if (info) info->first_bad_index = bad;
  if (st != TRINV_OK) return st;
  unsigned nf = 0;
  HIP_TRY(hipMemcpy(&nf, w.nonfinite, sizeof(nf), hipMemcpyDeviceToHost));
  if (nf) return TRINV_ERR_NONFINITE;
  if (o.check && !o.upper && !o.unit_diag) {
    double r3[3];
    st = (mode == TRINV_F64) ? residual_t<double>(n, (const double*)L, ldl, (const double*)X, ldx, wr, s, r3)
                             : residual_t<float>(n, (const float*)L, ldl, (const float*)X, ldx, wr, s, r3);
    if (st != TRINV_OK) return st;
    const double rel = r3[0] / (r3[1] * r3[2]);
    if (info) info->rel_residual = rel;
    if (!std::isfinite(rel)) return TRINV_ERR_NONFINITE;
  }
  return TRINV_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- factored inverse
// A = L U given as its triangular factors (Section 5, algorithm SKUL, whose
// output statement is S K = A^-1 with S = U^-1 and K = L^-1): Linv and Uinv
// come from the same recursion (U through its transpose), and the optional
// Ainv = Uinv * Linv is an upper x lower product whose K range for output
// (i, j) starts at max(i, j) (the Pul product of the paper's cost notation).
namespace {

// L and U^T are inverted together, as a strided batch of two lower
// triangles: every level launch then has twice the tiles.
struct WsFactored {
  uint64_t* status;
  unsigned* nonfinite;
  void* T;    // level workspace for the batch of two
  void* In;   // [L, U^T], n x n each
  void* Out;  // [L^-1, (U^-1)^T]
};

WsFactored carve_factored(Carve& c, int mode, int64_t n, int64_t leaf) {
  WsFactored w;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  w.status = c.take<uint64_t>(1);
  w.nonfinite = c.take<unsigned>(1);
  w.T = c.take<char>(es * 2 * (size_t)t_elems(n, leaf));
  w.In = c.take<char>(es * 2 * (size_t)n * n);
  w.Out = c.take<char>(es * 2 * (size_t)n * n);
  return w;
}

// Linv = L^-1, Uinv = U^-1 through the batch of two (unit diagonals are
// written as exact ones in the copies, so the batch runs without the flag and
// forms the same values: X_ii = 1/1, X_ij = -s/1).
template <typename T>
hipError_t factored_pair(int64_t n, const T* L, int64_t ldl, int l_unit, const T* U, int64_t ldu, int u_unit,
                         T* Linv, int64_t ldli, T* Uinv, int64_t ldui, int64_t leaf, const WsFactored& w,
                         hipStream_t s) {
  const int64_t nn = n * n;
  T* in = (T*)w.In;
  T* out = (T*)w.Out;
  hipError_t e;
  if ((e = launch_block_copy<T>(L, ldl, 0, in, n, 0, n, 1, T(1), s)) != hipSuccess) return e;
  if ((e = launch_transpose<T>(U, ldu, in + nn, n, n, s)) != hipSuccess) return e;
  if (l_unit && (e = launch_set_diag<T>(in, n, n, T(1), s)) != hipSuccess) return e;
  if (u_unit && (e = launch_set_diag<T>(in + nn, n, n, T(1), s)) != hipSuccess) return e;
  {
    const double nl = 2.0 * (double)((n + leaf - 1) / leaf), b = (double)leaf;
    ProfLaunch pl(sizeof(T) == 8 ? "leaf_f64" : "leaf_f32", nl * b * b * b / 3.0, nl * b * b * sizeof(T), s);
    e = launch_leaf<T>(n, in, n, out, n, nn, 2, (int)leaf, 0, nullptr, nullptr, 0, 0, 1.0, w.status, 0, s);
  }
  if (e != hipSuccess) return e;
  if ((e = run_levels<T, T>(n, in, n, out, n, nn, 2, leaf, (T*)w.T, s)) != hipSuccess) return e;
  if ((e = launch_block_copy<T>(out, n, 0, Linv, ldli, 0, n, 1, T(1), s)) != hipSuccess) return e;
  return launch_transpose<T>(out + nn, n, Uinv, ldui, n, s);
}

template <typename T>
hipError_t upper_times_lower(int64_t n, const T* Uinv, int64_t ldui, const T* Linv, int64_t ldli, T* Ainv,
                             int64_t ldai, hipStream_t s) {
  GemmArgs<T> g{};
  g.A = {Uinv, ldui, 0, 0};
  g.B = {Linv, ldli, 0, 0};
  g.D = {Ainv, ldai, 0, 0};
  g.alpha = 1.0;
  g.amask = 3;  // upper: k >= m
  g.bmask = 1;  // lower: k >= n
  g.tiles = kAllTiles;
  g.order = kColAsc;
  g.klo = kLoMax;
  g.khi = kHiK;
  g.bt = {1, 1, n, n, n, n, n, n};
  return launch_gemm<T, T>(g, s);
}

}  // namespace

extern "C" size_t trinv_factored_workspace_bytes(int mode, int64_t n, const trinv_opts* opts) {
  if (n <= 0) return 0;
  const trinv_opts o = resolve_opts(opts);
  const int64_t leaf = o.leaf ? o.leaf : default_leaf(mode, n);
  Carve c(nullptr, 0);
  carve_factored(c, mode, n, leaf);
  return c.used;
}

extern "C" int trinv_factored_inverse(int mode, int64_t n, const void* L, int64_t ldl, int32_t l_unit,
                                      const void* U, int64_t ldu, int32_t u_unit, void* Linv, int64_t ldli,
                                      void* Uinv, int64_t ldui, void* Ainv, int64_t ldai, const trinv_opts* opts,
                                      void* ws, size_t ws_bytes, trinv_stream_t stream, trinv_info* info) {
  info_reset(info);
  if (n < 0 || ldl < n || ldu < n || ldli < n || ldui < n || (Ainv && ldai < n)) return TRINV_ERR_ARG;
  if (n == 0) return TRINV_OK;
  if (!L || !U || !Linv || !Uinv) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32) return TRINV_ERR_UNSUPPORTED;
  trinv_opts o = resolve_opts(opts);
  const int64_t leaf = o.leaf ? o.leaf : default_leaf(mode, n);
  if (!valid_leaf(leaf)) return TRINV_ERR_ARG;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  const size_t bl = span_bytes(n, n, ldl, es), bu = span_bytes(n, n, ldu, es);
  const void* outs[3] = {Linv, Uinv, Ainv};
  const size_t ob[3] = {span_bytes(n, n, ldli, es), span_bytes(n, n, ldui, es), span_bytes(n, n, ldai, es)};
  for (int i = 0; i < 3; ++i) {
    if (!outs[i]) continue;
    if (overlaps(outs[i], ob[i], L, bl) || overlaps(outs[i], ob[i], U, bu)) return TRINV_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (outs[j] && overlaps(outs[i], ob[i], outs[j], ob[j])) return TRINV_ERR_ARG;
  }
  Carve c(ws, ws_bytes);
  WsFactored w = carve_factored(c, mode, n, leaf);
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_fill_u64(w.status, ~0ull, 1, s));
  if (mode == TRINV_F64) {
    HIP_TRY(factored_pair<double>(n, (const double*)L, ldl, l_unit, (const double*)U, ldu, u_unit, (double*)Linv,
                                  ldli, (double*)Uinv, ldui, leaf, w, s));
    if (Ainv)
      HIP_TRY(upper_times_lower<double>(n, (const double*)Uinv, ldui, (const double*)Linv, ldli, (double*)Ainv,
                                        ldai, s));
  } else {
    HIP_TRY(factored_pair<float>(n, (const float*)L, ldl, l_unit, (const float*)U, ldu, u_unit, (float*)Linv, ldli,
                                 (float*)Uinv, ldui, leaf, w, s));
    if (Ainv)
      HIP_TRY(upper_times_lower<float>(n, (const float*)Uinv, ldui, (const float*)Linv, ldli, (float*)Ainv, ldai,
                                       s));
  }
  if (!o.blocking) return TRINV_OK;
  HIP_TRY(launch_zero(w.nonfinite, sizeof(unsigned), s));
  for (int i = 0; i < 3; ++i) {
    if (!outs[i]) continue;
    const int64_t ld = i == 0 ? ldli : (i == 1 ? ldui : ldai);
    if (mode == TRINV_F64)
      HIP_TRY(launch_nonfinite<double>((const double*)outs[i], n, ld, w.nonfinite, s));
    else
      HIP_TRY(launch_nonfinite<float>((const float*)outs[i], n, ld, w.nonfinite, s));
  }
  int64_t bad = 0;
  const int st = wait_status(s, w.status, n, &bad);
  if (info) info->first_bad_index = bad;
  if (st != TRINV_OK) return st;
  unsigned nf = 0;
  HIP_TRY(hipMemcpy(&nf, w.nonfinite, sizeof(nf), hipMemcpyDeviceToHost));
  return nf ? TRINV_ERR_NONFINITE : TRINV_OK;
}

// ---------------------------------------------------------------- adjoint
// gradL = -tril(X^T G X^T) for a strided batch (not part of the paper; from
// dX = -X dL X). Two tri-structured products, n^3/3 flops each:
//   M     = tril(X^T G):  M(i,k) = sum_{l >= max(i,k)} X(l,i) G(l,k), k <= i
//   gradL = -tril(M X^T): grad(i,j) = -sum_{k <= j} M(i,k) X(j,k),   j <= i
// Only lower output tiles are formed; the strict upper tiles of gradL are
// zeroed by the mirror stores of the second product.
extern "C" size_t trinv_backward_workspace_bytes(int mode, int64_t batch, int64_t n) {
  if (n <= 0 || batch <= 0) return 0;
  Carve c(nullptr, 0);
  c.take<char>((mode == TRINV_F32 ? 4 : 8) * (size_t)batch * n * n);
  return c.used;
}

namespace {
template <typename T>
hipError_t backward_t(int64_t batch, int64_t n, const T* X, const T* G, T* grad, int64_t stride, T* Mws,
                      hipStream_t s) {
  GemmArgs<T> g1{};
  g1.A = {X, n, 0, stride};
  g1.a_trans = 1;
  g1.amask = 3;  // (X^T)(i,l) = X(l,i) is non-zero for l >= i
  g1.B = {G, n, 0, stride};
  g1.bmask = 1;  // only tril(G) contributes
  g1.D = {Mws, n, 0, n * n};
  g1.alpha = 1.0;
  g1.tiles = kLowerTiles;
  g1.order = kRowAsc;
  g1.klo = kLoM0;
  g1.khi = kHiK;
  g1.out_lower = 1;
  g1.bt = {1, batch, n, n, n, n, n, n};
  hipError_t e = launch_gemm<T, T>(g1, s);
  if (e != hipSuccess) return e;
  GemmArgs<T> g2{};
  g2.A = {Mws, n, 0, n * n};
  g2.amask = 1;
  g2.B = {X, n, 0, stride};
  g2.b_trans = 1;
  g2.bmask = 3;  // (X^T)(k,j) = X(j,k) is non-zero for k <= j
  g2.D = {grad, n, 0, stride};
  g2.Zmirror = {grad, n, 0, stride};
  g2.mirror_skip_diag = 1;
  g2.alpha = -1.0;
  g2.tiles = kLowerTiles;
  g2.order = kColDesc;
  g2.klo = kLoZero;
  g2.khi = kHiN1;
  g2.out_lower = 1;
  g2.bt = {1, batch, n, n, n, n, n, n};
  return launch_gemm<T, T>(g2, s);
}
}  // namespace

extern "C" int trinv_tril_inverse_backward(int mode, int64_t batch, int64_t n, const void* X, const void* G,
                                           void* gradL, int64_t stride, void* ws, size_t ws_bytes,
                                           trinv_stream_t stream) {
  if (n < 0 || batch < 0 || stride < n * n) return TRINV_ERR_ARG;
  if (n == 0 || batch == 0) return TRINV_OK;
  if (!X || !G || !gradL) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32) return TRINV_ERR_UNSUPPORTED;
  const size_t es = mode == TRINV_F32 ? 4 : 8, nb = span_bytes(batch, n * n, stride, es);
  if (overlaps(gradL, nb, X, nb) || overlaps(gradL, nb, G, nb)) return TRINV_ERR_ARG;
  Carve c(ws, ws_bytes);
  void* Mws = c.take<char>(es * (size_t)batch * n * n);
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (mode == TRINV_F64)
    HIP_TRY(backward_t<double>(batch, n, (const double*)X, (const double*)G, (double*)gradL, stride, (double*)Mws, s));
  else
    HIP_TRY(backward_t<float>(batch, n, (const float*)X, (const float*)G, (float*)gradL, stride, (float*)Mws, s));
  return TRINV_OK;
}
