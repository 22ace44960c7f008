// Algorithm SKUL (Section 5): A = L U (Crout: L lower, U unit upper, no
// pivoting) together with S = U^-1 and K = L^-1, so that S K = A^-1.
//
// Blocked, right-looking, on a working copy W of A, in steps of nb = 128:
//   1. the diagonal block W_kk is factored in one workgroup, which grows its
//      inverses K_kk = L_kk^-1 and S_kk = U_kk^-1 in the same pass over the
//      pivots (the fused recurrences of SKUL);
//   2. the panels follow from them on MFMA: L_ik = W_ik S_kk (i > k) and
//      U_kj = K_kk W_kj (j > k);
//   3. the trailing block is updated: W_ij -= L_ik U_kj.
// The paper grows K and S over the whole matrix beside the Crout loop; here
// only the diagonal-block inverses are grown that way (they feed the panels),
// and the full K, S (and optionally A^-1 = S K) are formed by the recursive
// engine once L and U are complete (trinv_factored_inverse).
#include <algorithm>

#include "api_internal.h"
#include "profile.h"

using namespace trinv;

namespace {

constexpr int64_t kNb = 128;

struct WsSkul {
  uint64_t* status;
  void *W, *Kb, *Sb, *fws;
  size_t fws_bytes;
};

WsSkul carve_skul(Carve& c, int mode, int64_t n, const trinv_opts& o) {
  WsSkul w;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  w.status = c.take<uint64_t>(1);
  w.W = c.take<char>(es * (size_t)n * n);
  for (void** p : {&w.Kb, &w.Sb}) *p = c.take<char>(es * (size_t)kNb * kNb);
  w.fws_bytes = trinv_factored_workspace_bytes(mode, n, &o);
  w.fws = c.take<char>(w.fws_bytes);
  return w;
}

template <typename T>
hipError_t skul_lu(int64_t n, const T* A, T* L, T* U, const WsSkul& w, hipStream_t s) {
  T* W = (T*)w.W;
  T *Kb = (T*)w.Kb, *Sb = (T*)w.Sb;
  hipError_t e;
  if ((e = launch_block_copy<T>(A, n, 0, W, n, 0, n, 1, T(1), s)) != hipSuccess) return e;
  if ((e = launch_zero(L, sizeof(T) * (size_t)n * n, s)) != hipSuccess) return e;
  if ((e = launch_zero(U, sizeof(T) * (size_t)n * n, s)) != hipSuccess) return e;
  const char* pre = sizeof(T) == 8 ? "f64" : "f32";
  char cls[32];
  for (int64_t k0 = 0; k0 < n; k0 += kNb) {
    const int64_t b = std::min(kNb, n - k0), r1 = k0 + b, rest = n - r1;
    {
      snprintf(cls, sizeof(cls), "%s_skul_diag", pre);
      ProfLaunch pl(cls, 4.0 * b * b * b / 3.0, sizeof(T) * 5.0 * b * b, s);
      if ((e = launch_crout_diag<T>(W + k0 * n + k0, n, 0, (int)b, L + k0 * n + k0, U + k0 * n + k0, n, 0, Kb, Sb, kNb,
                                    0, 1, k0, w.status, s)) != hipSuccess)
        return e;
    }
    if (rest == 0) break;
    const double fb = (double)b, fr = (double)rest;
    {  // L panel: L[r1:, k0:r1] = W[r1:, k0:r1] S_kk
      GemmArgs<T> g{};
      g.A = {W + r1 * n + k0, n, 0, 0};
      g.B = {Sb, kNb, 0, 0};
      g.D = {L + r1 * n + k0, n, 0, 0};
      g.alpha = 1.0;
      g.tiles = kAllTiles;
      g.order = kColAsc;
      g.klo = kLoZero;
      g.khi = kHiN1;  // S_kk(k, col) = 0 for k > col
      g.bt = {1, 1, rest, b, b, rest, b, b};
      snprintf(cls, sizeof(cls), "%s_skul_panel", pre);
      ProfLaunch pl(cls, fr * fb * (fb + 1), sizeof(T) * 2.0 * fr * fb, s);
      if ((e = launch_gemm<T, T>(g, s)) != hipSuccess) return e;
    }
    {  // U panel: U[k0:r1, r1:] = K_kk W[k0:r1, r1:]
      GemmArgs<T> g{};
      g.A = {Kb, kNb, 0, 0};
      g.B = {W + k0 * n + r1, n, 0, 0};
      g.D = {U + k0 * n + r1, n, 0, 0};
      g.alpha = 1.0;
      g.tiles = kAllTiles;
      g.order = kRowDesc;
      g.klo = kLoZero;
      g.khi = kHiM1;  // K_kk(row, k) = 0 for k > row
      g.bt = {1, 1, b, rest, b, b, rest, b};
      snprintf(cls, sizeof(cls), "%s_skul_upanel", pre);
      ProfLaunch pl(cls, fb * (fb + 1) * fr, sizeof(T) * 2.0 * fr * fb, s);
      if ((e = launch_gemm<T, T>(g, s)) != hipSuccess) return e;
    }
    {  // trailing: W[r1:, r1:] -= L[r1:, k0:r1] U[k0:r1, r1:]
      GemmArgs<T> g{};
      g.A = {L + r1 * n + k0, n, 0, 0};
      g.B = {U + k0 * n + r1, n, 0, 0};
      g.D = {W + r1 * n + r1, n, 0, 0};
      g.alpha = -1.0;
      g.accumulate = 1;
      g.tiles = kAllTiles;
      g.order = kColAsc;
      g.klo = kLoZero;
      g.khi = kHiK;
      g.bt = {1, 1, rest, rest, b, rest, rest, b};
      snprintf(cls, sizeof(cls), "%s_skul_update", pre);
      ProfLaunch pl(cls, 2.0 * fr * fr * fb, sizeof(T) * 2.0 * fr * fr, s);
      if ((e = launch_gemm<T, T>(g, s)) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace

extern "C" size_t trinv_skul_workspace_bytes(int mode, int64_t n, const trinv_opts* opts) {
  if (n <= 0) return 0;
  const trinv_opts o = resolve_opts(opts);
  Carve c(nullptr, 0);
  carve_skul(c, mode, n, o);
  return c.used;
}

extern "C" int trinv_skul(int mode, int64_t n, const void* A, void* L, void* U, void* S, void* K, void* Ainv,
                          const trinv_opts* opts, void* ws, size_t ws_bytes, trinv_stream_t stream,
                          trinv_info* info) {
  info_reset(info);
  if (n < 0) return TRINV_ERR_ARG;
  if (n == 0) return TRINV_OK;
  if (!A || !L || !U || !S || !K) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32) return TRINV_ERR_UNSUPPORTED;
  trinv_opts o = resolve_opts(opts);
  if (o.upper || o.unit_diag || o.beta > 2) return TRINV_ERR_UNSUPPORTED;
  const int64_t leaf = o.leaf ? o.leaf : default_leaf(mode, n);
  if (!valid_leaf(leaf)) return TRINV_ERR_ARG;
  const size_t es = mode == TRINV_F32 ? 4 : 8, nb = (size_t)n * n * es;
  const void* outs[5] = {L, U, S, K, Ainv};
  for (int i = 0; i < 5; ++i) {
    if (!outs[i]) continue;
    if (overlaps(outs[i], nb, A, nb)) return TRINV_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (outs[j] && overlaps(outs[i], nb, outs[j], nb)) return TRINV_ERR_ARG;
  }
  Carve c(ws, ws_bytes);
  WsSkul w = carve_skul(c, mode, n, o);
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_fill_u64(w.status, ~0ull, 1, s));
  if (mode == TRINV_F64)
    HIP_TRY(skul_lu<double>(n, (const double*)A, (double*)L, (double*)U, w, s));
  else
    HIP_TRY(skul_lu<float>(n, (const float*)A, (float*)L, (float*)U, w, s));
  trinv_opts of = o;
  of.blocking = 0;
  const int st = trinv_factored_inverse(mode, n, L, n, 0, U, n, 1, K, n, S, n, Ainv, n, &of, w.fws, w.fws_bytes,
                                        stream, nullptr);
  if (st != TRINV_OK) return st;
  if (!o.blocking) return TRINV_OK;
  int64_t bad = 0;
  const int st2 = wait_status(s, w.status, n, &bad);
  if (info) info->first_bad_index = bad;
  return st2;
}
