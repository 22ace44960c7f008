// Algorithm SQR (Section 5): modified Gram-Schmidt A = Q R together with
// S = R^-1, so that S Q^T = A^-1.
//
// Blocked, right-looking, on a working copy V of A, with panels of 16 (8 for
// n > 1024) columns inside outer blocks of 128:
//   1. a panel is orthogonalized column by column in one workgroup (its
//      columns of Q and its diagonal block of R);
//   2. the later columns of the outer block lose the panel's components:
//      R_pJ = Q_p^T V_J (split over row chunks, partial products summed in a
//      fixed order), V_J -= Q_p R_pJ (FP64 / FP32 MFMA products);
//   3. once the outer block is done, the same two products with its 128
//      columns update every later column.
// Inside a panel the projections are applied one column at a time, as
// modified Gram-Schmidt does; between panels one product applies all the
// columns of a panel at once (block Gram-Schmidt), which is the same
// arithmetic up to rounding when the columns of the panel are orthonormal.
// S = R^-1 is formed once R is complete, by the recursive triangular engine
// (upper mode), where the algorithm grows S one column at a time beside R;
// A^-1 = S Q^T is one more product.
#include <algorithm>

#include "api_internal.h"
#include "profile.h"

using namespace trinv;

namespace {

constexpr int64_t kOuter = 128;
constexpr int64_t kMaxN = 4096;  // the panel holds a column in one workgroup's registers
constexpr int64_t kChunk = 256;  // rows per partial product of a projection (split K)

int64_t chunks(int64_t n) { return (n + kChunk - 1) / kChunk; }

trinv_opts upper_opts(const trinv_opts& o) {
  trinv_opts u = o;
  u.upper = 1;
  u.unit_diag = 0;
  u.blocking = 0;
  u.check = 0;
  u.beta = 0;
  return u;
}

struct WsSqr {
  uint64_t* status;
  void *V, *part, *tws;
  size_t tws_bytes;
};

WsSqr carve_sqr(Carve& c, int mode, int64_t n, const trinv_opts& o) {
  WsSqr w;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  w.status = c.take<uint64_t>(1);
  w.V = c.take<char>(es * (size_t)n * n);
  w.part = c.take<char>(es * (size_t)chunks(n) * kOuter * n);
  const trinv_opts u = upper_opts(o);
  w.tws_bytes = trinv_workspace_bytes(mode, n, &u);
  w.tws = c.take<char>(w.tws_bytes);
  return w;
}

// R[r0 : r0 + m, c0 : c0 + nc] = Q[:, r0 : r0 + m]^T V[:, c0 : c0 + nc], then
// V[:, c0 : c0 + nc] -= Q[:, r0 : r0 + m] R[r0 : r0 + m, c0 : c0 + nc].
// The first product has a short output and a long K (the n rows): it runs
// as one launch of partial products over row chunks of kChunk (the merges of
// the launch), summed in chunk order by a second kernel.
template <typename T>
hipError_t project(int64_t n, const T* Q, T* R, T* V, int64_t r0, int64_t m, int64_t c0, int64_t nc, T* part,
                   const char* pre, hipStream_t s) {
  char cls[32];
  const double fm = (double)m, fn = (double)n, fc = (double)nc;
  const int64_t nch = chunks(n);
  hipError_t e;
  {
    GemmArgs<T> g{};
    g.A = {Q + r0, n, kChunk * n, 0};  // read transposed: A(i, k) = Q[(k + z kChunk) n + r0 + i]
    g.a_trans = 1;
    g.B = {V + c0, n, kChunk * n, 0};
    g.D = {part, nc, m * nc, 0};
    g.alpha = 1.0;
    g.tiles = kAllTiles;
    g.order = kColAsc;
    g.klo = kLoZero;
    g.khi = kHiK;
    g.bt = {nch, 1, m, nc, kChunk, m, nc, n - (nch - 1) * kChunk};
    snprintf(cls, sizeof(cls), "%s_sqr_proj", pre);
    ProfLaunch pl(cls, 2.0 * fm * fc * fn, sizeof(T) * (fm * fn + fn * fc + nch * fm * fc), s);
    if ((e = launch_gemm<T, T>(g, s)) != hipSuccess) return e;
  }
  if ((e = launch_sum_blocks<T>(part, nc, m * nc, nch, m, nc, R + r0 * n + c0, n, s)) != hipSuccess) return e;
  GemmArgs<T> g{};
  g.A = {Q + r0, n, 0, 0};
  g.B = {R + r0 * n + c0, n, 0, 0};
  g.D = {V + c0, n, 0, 0};
  g.alpha = -1.0;
  g.accumulate = 1;
  g.tiles = kAllTiles;
  g.order = kColAsc;
  g.klo = kLoZero;
  g.khi = kHiK;
  g.bt = {1, 1, n, nc, m, n, nc, m};
  snprintf(cls, sizeof(cls), "%s_sqr_update", pre);
  ProfLaunch pl(cls, 2.0 * fm * fc * fn, sizeof(T) * (fm * fn + fm * fc + 2.0 * fn * fc), s);
  return launch_gemm<T, T>(g, s);
}

template <typename T>
hipError_t sqr_qr(int64_t n, const T* A, T* Q, T* R, const WsSqr& w, hipStream_t s) {
  T* V = (T*)w.V;
  hipError_t e;
  if ((e = launch_block_copy<T>(A, n, 0, V, n, 0, n, 1, T(1), s)) != hipSuccess) return e;
  if ((e = launch_zero(R, sizeof(T) * (size_t)n * n, s)) != hipSuccess) return e;
  const char* pre = sizeof(T) == 8 ? "f64" : "f32";
  char cls[32];
  snprintf(cls, sizeof(cls), "%s_sqr_panel", pre);
  const int64_t pw = mgs_panel_width(n);
  for (int64_t ob0 = 0; ob0 < n; ob0 += kOuter) {
    const int64_t ob1 = std::min(ob0 + kOuter, n);
    for (int64_t p0 = ob0; p0 < ob1; p0 += pw) {
      const int64_t wd = std::min(pw, ob1 - p0), p1 = p0 + wd;
      {
        ProfLaunch pl(cls, 2.0 * n * wd * wd, sizeof(T) * 2.0 * n * wd, s);
        if ((e = launch_mgs_panel<T>(V, Q, R, n, n, p0, (int)wd, w.status, s)) != hipSuccess) return e;
      }
      if (p1 < ob1 && (e = project<T>(n, Q, R, V, p0, wd, p1, ob1 - p1, (T*)w.part, pre, s)) != hipSuccess)
        return e;
    }
    if (ob1 < n && (e = project<T>(n, Q, R, V, ob0, ob1 - ob0, ob1, n - ob1, (T*)w.part, pre, s)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

// Ainv = S Q^T (S upper: k >= row; Q read transposed).
template <typename T>
hipError_t s_times_qt(int64_t n, const T* S, const T* Q, T* Ainv, hipStream_t s) {
  GemmArgs<T> g{};
  g.A = {S, n, 0, 0};
  g.B = {Q, n, 0, 0};
  g.b_trans = 1;
  g.D = {Ainv, n, 0, 0};
  g.alpha = 1.0;
  g.tiles = kAllTiles;
  g.order = kColAsc;
  g.klo = kLoM0;
  g.khi = kHiK;
  g.bt = {1, 1, n, n, n, n, n, n};
  const double fn = (double)n;
  ProfLaunch pl(sizeof(T) == 8 ? "f64_sqr_ainv" : "f32_sqr_ainv", fn * fn * (fn + 1), sizeof(T) * 2.5 * fn * fn, s);
  return launch_gemm<T, T>(g, s);
}

}  // namespace

extern "C" size_t trinv_sqr_workspace_bytes(int mode, int64_t n, const trinv_opts* opts) {
  if (n <= 0) return 0;
  const trinv_opts o = resolve_opts(opts);
  Carve c(nullptr, 0);
  carve_sqr(c, mode, n, o);
  return c.used;
}

extern "C" int trinv_sqr(int mode, int64_t n, const void* A, void* Q, void* R, void* S, void* Ainv,
                         const trinv_opts* opts, void* ws, size_t ws_bytes, trinv_stream_t stream, trinv_info* info) {
  info_reset(info);
  if (n < 0) return TRINV_ERR_ARG;
  if (n == 0) return TRINV_OK;
  if (!A || !Q || !R || !S) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32) return TRINV_ERR_UNSUPPORTED;
  const trinv_opts o = resolve_opts(opts);
  if (o.upper || o.unit_diag || o.beta > 2 || n > kMaxN) return TRINV_ERR_UNSUPPORTED;
  const int64_t leaf = o.leaf ? o.leaf : default_leaf(mode, n);
  if (!valid_leaf(leaf)) return TRINV_ERR_ARG;
  const size_t es = mode == TRINV_F32 ? 4 : 8, nb = (size_t)n * n * es;
  const void* outs[4] = {Q, R, S, Ainv};
  for (int i = 0; i < 4; ++i) {
    if (!outs[i]) continue;
    if (overlaps(outs[i], nb, A, nb)) return TRINV_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (outs[j] && overlaps(outs[i], nb, outs[j], nb)) return TRINV_ERR_ARG;
  }
  Carve c(ws, ws_bytes);
  const WsSqr w = carve_sqr(c, mode, n, o);
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_fill_u64(w.status, ~0ull, 1, s));
  if (mode == TRINV_F64)
    HIP_TRY(sqr_qr<double>(n, (const double*)A, (double*)Q, (double*)R, w, s));
  else
    HIP_TRY(sqr_qr<float>(n, (const float*)A, (float*)Q, (float*)R, w, s));
  const trinv_opts u = upper_opts(o);
  const int st = trinv_tril_inverse(mode, n, R, n, S, n, &u, w.tws, w.tws_bytes, stream, nullptr);
  if (st != TRINV_OK) return st;
  if (Ainv) {
    if (mode == TRINV_F64)
      HIP_TRY(s_times_qt<double>(n, (const double*)S, (const double*)Q, (double*)Ainv, s));
    else
      HIP_TRY(s_times_qt<float>(n, (const float*)S, (const float*)Q, (float*)Ainv, s));
  }
  if (!o.blocking) return TRINV_OK;
  int64_t bad = 0;
  const int st2 = wait_status(s, w.status, n, &bad);
  if (info) info->first_bad_index = bad;
  return st2;
}
