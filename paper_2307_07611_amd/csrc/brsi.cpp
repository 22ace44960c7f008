// General inverse by BRSI with gamma = 2 (Section 5, Steps of BRSI and the
// gamma = 2 derivation). For A with diagonal blocks A11, A22 of order h:
//   S11 = A11^-1, S22 = A22^-1           (this recursion, both in one batch)
//   S12 = -S11 A12 S22                    (U0^-1 = [[S11, S12], [0, S22]])
//   W   = (I + S12 A21)^-1                (this recursion)
//   A^-1 = [[W S11, W S12], [-S22 A21 W S11, S22 - S22 A21 W S12]].
// The recursion runs breadth-wise over a batch: every node of one depth takes
// its two diagonal blocks to the next depth together, so the number of
// sequential bottom-level steps is the number of blocks of one diagonal (not
// 3^depth), and every product of a depth is one strided batched launch on the
// FP64 / FP32 MFMA tile products. Orders at the bottom (<= 128) are inverted
// by the fused Crout step of SKUL (L U, K = L^-1, S = U^-1 in one workgroup)
// and A^-1 = S K. The order is padded to b 2^depth (b <= 128) with an
// identity tail, [[A, 0], [0, I]]^-1 = [[A^-1, 0], [0, I]], so that every
// split is even. No pivoting: the diagonal blocks met on the way must be
// invertible (as for the positive definite matrices of the derivation, or
// diagonally dominant ones).
#include <algorithm>

#include "api_internal.h"
#include "profile.h"

using namespace trinv;

namespace {

constexpr int64_t kBase = 128;

struct BrsiPlan {
  int64_t n, np;  // order, padded order np = b 2^depth
  int depth;
};

BrsiPlan brsi_plan(int64_t n) {
  BrsiPlan p{n, n, 0};
  while (((n + ((int64_t)1 << p.depth) - 1) >> p.depth) > kBase) ++p.depth;
  const int64_t b = (n + ((int64_t)1 << p.depth) - 1) >> p.depth;
  p.np = b << p.depth;
  return p;
}

struct BrsiWs {
  uint64_t* status;
  void *Apad, *Xpad;                     // padded input / output (np != n)
  void *bL, *bU, *bK, *bS;               // bottom level: batch of kBase^2 blocks
  std::vector<void*> C, CI, Tb, S12, P, Wb;  // per depth < depth
};

BrsiWs carve_brsi(Carve& c, const BrsiPlan& p, size_t es) {
  BrsiWs w;
  w.status = c.take<uint64_t>(1);
  const bool pad = p.np != p.n;
  w.Apad = c.take<char>(pad ? es * (size_t)p.np * p.np : 0);
  w.Xpad = c.take<char>(pad ? es * (size_t)p.np * p.np : 0);
  const size_t nbase = (size_t)1 << p.depth;
  for (void** q : {&w.bL, &w.bU, &w.bK, &w.bS}) *q = c.take<char>(es * nbase * kBase * kBase);
  for (int d = 0; d < p.depth; ++d) {
    const size_t B = (size_t)1 << d, h = (size_t)(p.np >> (d + 1));
    w.C.push_back(c.take<char>(es * 2 * B * h * h));
    w.CI.push_back(c.take<char>(es * 2 * B * h * h));
    w.Tb.push_back(c.take<char>(es * B * h * h));
    w.S12.push_back(c.take<char>(es * B * h * h));
    w.P.push_back(c.take<char>(es * B * h * h));
    w.Wb.push_back(c.take<char>(es * B * h * h));
  }
  return w;
}

// D_b = alpha A_b B_b (+ D_b if acc) for b < B, all operands m x m.
template <typename T>
hipError_t bprod(int64_t m, int64_t B, const T* A, int64_t lda, int64_t sa, const T* Bm, int64_t ldb, int64_t sb,
                 T* D, int64_t ldd, int64_t sd, double alpha, int acc, const char* cls, hipStream_t s) {
  GemmArgs<T> g{};
  g.A = {A, lda, 0, sa};
  g.B = {Bm, ldb, 0, sb};
  g.D = {D, ldd, 0, sd};
  g.alpha = alpha;
  g.accumulate = acc;
  g.tiles = kAllTiles;
  g.order = kColAsc;
  g.klo = kLoZero;
  g.khi = kHiK;
  g.bt = {1, B, m, m, m, m, m, m};
  const double fm = (double)m;
  ProfLaunch pl(cls, 2.0 * B * fm * fm * fm, sizeof(T) * (3.0 + acc) * B * fm * fm, s);
  return launch_gemm<T, T>(g, s);
}

// Inverses of a strided batch of B matrices of order m (depth d of the plan):
// In_b at In + b si (leading dimension ldi), Out_b at Out + b so (ldo).
template <typename T>
hipError_t brsi_rec(int d, int64_t m, int64_t B, const T* In, int64_t ldi, int64_t si, T* Out, int64_t ldo, int64_t so,
                    const BrsiPlan& p, const BrsiWs& w, hipStream_t s) {
  hipError_t e;
  const char* pre = sizeof(T) == 8 ? "f64" : "f32";
  char cls[32];
  if (d == p.depth) {  // bottom: Crout with the inverse factors, then S K
    T *L = (T*)w.bL, *U = (T*)w.bU, *K = (T*)w.bK, *S = (T*)w.bS;
    const int64_t bb = kBase * kBase;
    {
      snprintf(cls, sizeof(cls), "%s_brsi_base", pre);
      const double fm = (double)m;
      ProfLaunch pl(cls, B * 4.0 * fm * fm * fm / 3.0, sizeof(T) * B * 5.0 * fm * fm, s);
      if ((e = launch_crout_diag<T>(In, ldi, si, (int)m, L, U, kBase, bb, K, S, kBase, bb, B, 0, w.status, s)) !=
          hipSuccess)
        return e;
    }
    GemmArgs<T> g{};
    g.A = {S, kBase, 0, bb};
    g.B = {K, kBase, 0, bb};
    g.D = {Out, ldo, 0, so};
    g.alpha = 1.0;
    g.amask = 3;  // S upper
    g.bmask = 1;  // K lower
    g.tiles = kAllTiles;
    g.order = kColAsc;
    g.klo = kLoMax;
    g.khi = kHiK;
    g.bt = {1, B, m, m, m, m, m, m};
    snprintf(cls, sizeof(cls), "%s_brsi_base_sk", pre);
    const double fm = (double)m;
    ProfLaunch pl(cls, B * 2.0 * fm * fm * fm / 3.0, sizeof(T) * B * 3.0 * fm * fm, s);
    return launch_gemm<T, T>(g, s);
  }
  const int64_t h = m / 2, hh = h * h;
  T *C = (T*)w.C[d], *CI = (T*)w.CI[d], *Tb = (T*)w.Tb[d], *S12 = (T*)w.S12[d], *P = (T*)w.P[d], *Wb = (T*)w.Wb[d];
  const T* A12 = In + h;
  const T* A21 = In + h * ldi;
  T *X11 = Out, *X12 = Out + h, *X21 = Out + h * ldo, *X22 = Out + h * ldo + h;
  snprintf(cls, sizeof(cls), "%s_brsi_prod", pre);
  // diagonal blocks of every matrix, A11 of matrix b at C[2b], A22 at C[2b + 1]
  if ((e = launch_block_copy<T>(In, ldi, si, C, h, 2 * hh, h, B, T(1), s)) != hipSuccess) return e;
  if ((e = launch_block_copy<T>(In + h * ldi + h, ldi, si, C + hh, h, 2 * hh, h, B, T(1), s)) != hipSuccess) return e;
  if ((e = brsi_rec<T>(d + 1, h, 2 * B, C, h, hh, CI, h, hh, p, w, s)) != hipSuccess) return e;
  const T* S11 = CI;
  const T* S22 = CI + hh;  // both at stride 2 hh
  // S12 = -(S11 A12) S22
  if ((e = bprod<T>(h, B, S11, h, 2 * hh, A12, ldi, si, Tb, h, hh, 1.0, 0, cls, s)) != hipSuccess) return e;
  if ((e = bprod<T>(h, B, Tb, h, hh, S22, h, 2 * hh, S12, h, hh, -1.0, 0, cls, s)) != hipSuccess) return e;
  // W = (I + S12 A21)^-1
  if ((e = launch_embed<T>(nullptr, 0, 0, 0, P, h, hh, h, B, s)) != hipSuccess) return e;
  if ((e = bprod<T>(h, B, S12, h, hh, A21, ldi, si, P, h, hh, 1.0, 1, cls, s)) != hipSuccess) return e;
  if ((e = brsi_rec<T>(d + 1, h, B, P, h, hh, Wb, h, hh, p, w, s)) != hipSuccess) return e;
  // top block row: X11 = W S11, X12 = W S12
  if ((e = bprod<T>(h, B, Wb, h, hh, S11, h, 2 * hh, X11, ldo, so, 1.0, 0, cls, s)) != hipSuccess) return e;
  if ((e = bprod<T>(h, B, Wb, h, hh, S12, h, hh, X12, ldo, so, 1.0, 0, cls, s)) != hipSuccess) return e;
  // bottom block row with T = S22 A21: X21 = -T X11, X22 = S22 - T X12
  if ((e = bprod<T>(h, B, S22, h, 2 * hh, A21, ldi, si, Tb, h, hh, 1.0, 0, cls, s)) != hipSuccess) return e;
  if ((e = launch_block_copy<T>(S22, h, 2 * hh, X22, ldo, so, h, B, T(1), s)) != hipSuccess) return e;
  if ((e = bprod<T>(h, B, Tb, h, hh, X12, ldo, so, X22, ldo, so, -1.0, 1, cls, s)) != hipSuccess) return e;
  return bprod<T>(h, B, Tb, h, hh, X11, ldo, so, X21, ldo, so, -1.0, 0, cls, s);
}

}  // namespace

extern "C" size_t trinv_brsi_workspace_bytes(int mode, int64_t n, const trinv_opts* opts) {
  (void)opts;
  if (n <= 0) return 0;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  Carve c(nullptr, 0);
  carve_brsi(c, brsi_plan(n), es);
  return c.used;
}

extern "C" int trinv_brsi(int mode, int64_t n, const void* A, int64_t lda, void* Ainv, int64_t ldx,
                          const trinv_opts* opts, void* ws, size_t ws_bytes, trinv_stream_t stream, trinv_info* info) {
  info_reset(info);
  if (n < 0) return TRINV_ERR_ARG;
  if (n == 0) return TRINV_OK;
  if (!A || !Ainv || lda < n || ldx < n) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32) return TRINV_ERR_UNSUPPORTED;
  const trinv_opts o = resolve_opts(opts);
  if (o.upper || o.unit_diag || o.beta > 2) return TRINV_ERR_UNSUPPORTED;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  if (overlaps(A, span_bytes(n, n, lda, es), Ainv, span_bytes(n, n, ldx, es))) return TRINV_ERR_ARG;
  const BrsiPlan p = brsi_plan(n);
  Carve c(ws, ws_bytes);
  const BrsiWs w = carve_brsi(c, p, es);
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_fill_u64(w.status, ~0ull, 1, s));
  const bool pad = p.np != n;
  if (mode == TRINV_F64) {
    const double* In = (const double*)A;
    double* Out = (double*)Ainv;
    int64_t ldi = lda, ldo = ldx;
    if (pad) {
      HIP_TRY(launch_embed<double>(In, lda, 0, n, (double*)w.Apad, p.np, 0, p.np, 1, s));
      In = (const double*)w.Apad;
      Out = (double*)w.Xpad;
      ldi = ldo = p.np;
    }
    HIP_TRY(brsi_rec<double>(0, p.np, 1, In, ldi, 0, Out, ldo, 0, p, w, s));
    if (pad) HIP_TRY(launch_block_copy<double>(Out, p.np, 0, (double*)Ainv, ldx, 0, n, 1, 1.0, s));
  } else {
    const float* In = (const float*)A;
    float* Out = (float*)Ainv;
    int64_t ldi = lda, ldo = ldx;
    if (pad) {
      HIP_TRY(launch_embed<float>(In, lda, 0, n, (float*)w.Apad, p.np, 0, p.np, 1, s));
      In = (const float*)w.Apad;
      Out = (float*)w.Xpad;
      ldi = ldo = p.np;
    }
    HIP_TRY(brsi_rec<float>(0, p.np, 1, In, ldi, 0, Out, ldo, 0, p, w, s));
    if (pad) HIP_TRY(launch_block_copy<float>(Out, p.np, 0, (float*)Ainv, ldx, 0, n, 1, 1.0f, s));
  }
  if (!o.blocking) return TRINV_OK;
  int64_t bad = 0;
  const int st = wait_status(s, w.status, n, &bad);
  if (info) info->first_bad_index = bad;
  return st;
}
