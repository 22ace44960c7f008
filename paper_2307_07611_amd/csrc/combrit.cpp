// Top level of algorithm COMBRIT (Section 4.1) with a beta x beta block grid,
// in the lower-triangular form: for L with diagonal blocks L_jj (order
// m = n / beta),
//   1. iD_jj = L_jj^-1 for every diagonal block (all blocks in one batched
//      run of the binary recursion, i.e. COMBRIT with beta = 2; Remark
//      rmkCOMBRIT leaves the method for the diagonal blocks open);
//   2. B_ij = L_ij iD_jj (i > j): L = B D with D = diag(L_jj), B unit lower
//      block-triangular (the transpose of the paper's row scaling);
//   3. iB = B^-1 by the block form of Theorem Combinatorix: (iB)_ij is the
//      signed sum over the chains j = c_0 < ... < c_k = i of the block
//      products B_{c_k c_{k-1}} ... B_{c_1 c_0}. Grouping the chains by their
//      last step gives (iB)_ij = -sum_{k=j}^{i-1} B_ik (iB)_kj with
//      (iB)_jj = I, i.e. (iB)_{j+d, j} = -B_{j+d, j} - B[j+d, j+1 : j+d]
//      (iB)[j+1 : j+d, j]: a copy and one product per block band d = i - j
//      over the stacked blocks;
//   4. X_ij = iD_ii (iB)_ij (i > j), X_ii = iD_ii, X_ij = 0 above.
// Every step runs on the FP64 / FP32 MFMA tile products; the blocks of one
// band are independent and share one launch (block (j + d, j) lies at a fixed
// stride from block (j - 1 + d, j - 1)).
#include "api_internal.h"
#include "profile.h"

namespace trinv {

size_t combrit_workspace_bytes(int mode, int64_t n, int beta, int64_t leaf) {
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  const int64_t m = n / beta;
  Carve c(nullptr, 0);
  c.take<uint64_t>((size_t)beta);                       // per-block pivot status
  c.take<char>(es * (size_t)beta * t_elems(m, leaf));  // level workspace of the diagonal blocks
  c.take<char>(es * (size_t)n * n);                     // B
  c.take<char>(es * (size_t)n * n);                     // iB
  return c.used;
}

template <typename T>
hipError_t combrit_t(int64_t n, const T* L, int64_t ld, T* X, int unit, int beta, int64_t leaf, void* ws,
                     size_t ws_bytes, uint64_t* status, hipStream_t s) {
  const int64_t m = n / beta;
  Carve c(ws, ws_bytes);
  uint64_t* words = c.take<uint64_t>((size_t)beta);
  T* Tws = (T*)c.take<char>(sizeof(T) * (size_t)beta * t_elems(m, leaf));
  T* WB = (T*)c.take<char>(sizeof(T) * (size_t)n * n);
  T* WiB = (T*)c.take<char>(sizeof(T) * (size_t)n * n);
  if (!c.ok()) return hipErrorInvalidValue;
  const char* pre = sizeof(T) == 8 ? "f64" : "f32";
  const int64_t dL = m * (ld + 1), dW = m * (n + 1);  // diagonal-block strides
  hipError_t e;
  // 1. diagonal blocks
  if ((e = launch_fill_u64(words, ~0ull, beta, s)) != hipSuccess) return e;
  {
    const double nl = (double)((m + leaf - 1) / leaf) * beta, b = (double)leaf;
    ProfLaunch pl(sizeof(T) == 8 ? "leaf_f64" : "leaf_f32", nl * b * b * b / 3.0, nl * b * b * sizeof(T), s);
    e = launch_leaf<T>(m, L, ld, X, ld, dL, beta, (int)leaf, unit, nullptr, nullptr, 0, 0, 1.0, words, 1, s);
  }
  if (e != hipSuccess) return e;
  if ((e = run_levels<T, T>(m, L, ld, X, ld, dL, beta, leaf, Tws, s)) != hipSuccess) return e;
  if ((e = launch_fold_status(words, beta, m, status, s)) != hipSuccess) return e;
  const double fm = (double)m;
  // 2. B_ij = L_ij iD_jj, one launch per band d (blocks j = 0 .. beta - 1 - d)
  for (int d = 1; d < beta; ++d) {
    GemmArgs<T> g{};
    g.A = {L + d * m * ld, ld, dL, 0};
    g.B = {X, ld, dL, 0};
    g.D = {WB + d * m * n, n, dW, 0};
    g.alpha = 1.0;
    g.tiles = kAllTiles;
    g.order = kColAsc;
    g.klo = kLoN0;  // iD_jj(k, col) = 0 for k < col
    g.khi = kHiK;
    g.bt = {beta - d, 1, m, m, m, m, m, m};
    char cls[32];
    snprintf(cls, sizeof(cls), "%s_combrit_scale", pre);
    ProfLaunch pl(cls, (beta - d) * fm * fm * (fm + 1), sizeof(T) * (beta - d) * 2.5 * fm * fm, s);
    if ((e = launch_gemm<T, T>(g, s)) != hipSuccess) return e;
  }
  // 3. iB by bands in order: (iB)_{j+d, j} = -B_{j+d, j} - B[j+d, j+1 : j+d] (iB)[j+1 : j+d, j]
  //    (the chains through the identity block (iB)_jj are the copy of -B)
  for (int d = 1; d < beta; ++d) {
    if ((e = launch_block_copy<T>(WB + d * m * n, n, dW, WiB + d * m * n, n, dW, m, beta - d, T(-1), s)) !=
        hipSuccess)
      return e;
    if (d == 1) continue;
    GemmArgs<T> g{};
    g.A = {WB + d * m * n + m, n, dW, 0};  // row block j + d, columns j + 1 .. j + d - 1
    g.B = {WiB + m * n, n, dW, 0};         // rows j + 1 .. j + d - 1 of column block j
    g.D = {WiB + d * m * n, n, dW, 0};
    g.alpha = -1.0;
    g.accumulate = 1;
    g.tiles = kAllTiles;
    g.order = kColAsc;
    g.klo = kLoZero;
    g.khi = kHiK;
    g.bt = {beta - d, 1, m, m, (d - 1) * m, m, m, (d - 1) * m};
    char cls[32];
    snprintf(cls, sizeof(cls), "%s_combrit_chain", pre);
    ProfLaunch pl(cls, (beta - d) * 2.0 * fm * fm * (d - 1) * fm, sizeof(T) * (beta - d) * (2.0 * d + 1) * fm * fm,
                  s);
    if ((e = launch_gemm<T, T>(g, s)) != hipSuccess) return e;
  }
  // 4. X_ij = iD_ii iB_ij, zeroing the mirrored upper block X_ji
  for (int d = 1; d < beta; ++d) {
    GemmArgs<T> g{};
    g.A = {X + d * m * (ld + 1), ld, dL, 0};  // iD_{j+d}
    g.B = {WiB + d * m * n, n, dW, 0};
    g.D = {X + d * m * ld, ld, dL, 0};
    g.Zmirror = {X + d * m, ld, dL, 0};
    g.alpha = 1.0;
    g.tiles = kAllTiles;
    g.order = kRowDesc;
    g.klo = kLoZero;
    g.khi = kHiM1;  // iD(row, k) = 0 for k > row
    g.bt = {beta - d, 1, m, m, m, m, m, m};
    char cls[32];
    snprintf(cls, sizeof(cls), "%s_combrit_out", pre);
    ProfLaunch pl(cls, (beta - d) * fm * fm * (fm + 1), sizeof(T) * (beta - d) * 3.5 * fm * fm, s);
    if ((e = launch_gemm<T, T>(g, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t combrit_t<double>(int64_t, const double*, int64_t, double*, int, int, int64_t, void*, size_t,
                                      uint64_t*, hipStream_t);
template hipError_t combrit_t<float>(int64_t, const float*, int64_t, float*, int, int, int64_t, void*, size_t,
                                     uint64_t*, hipStream_t);

}  // namespace trinv
