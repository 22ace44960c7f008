// Batched inversion of many independent lower-triangular matrices of order
// 1..1024: a one-workgroup plan kernel sorts the matrices by order, then one
// persistent launch (persistent.hip) inverts them, each workgroup taking whole
// matrices from a device-side queue. A uniform batch with fewer matrices than
// compute units instead runs the level recursion with the batch as an extra
// launch dimension (every level product spread over the whole chip).
#include <algorithm>
#include <vector>

#include "api_internal.h"
#include "profile.h"

using namespace trinv;

namespace {

struct WsPersistent {
  int32_t* order;
  uint32_t* queue;
};

WsPersistent carve_persistent(Carve& c, int64_t batch) {
  WsPersistent w;
  w.order = c.take<int32_t>((size_t)batch);
  w.queue = c.take<uint32_t>(1);
  return w;
}

// Few equal orders packed densely: the level path fills the chip better.
constexpr int64_t kLevelPathMaxBatch = 256;

bool level_path(int64_t batch, const int32_t* n_host, const int64_t* off_host) {
  if (batch > kLevelPathMaxBatch || n_host[0] < 128) return false;
  for (int64_t i = 0; i < batch; ++i)
    if (n_host[i] != n_host[0] || off_host[i] != i * (int64_t)n_host[0] * n_host[0]) return false;
  return true;
}

struct WsLevels {
  uint64_t* first_bad;
  void* T;
};

WsLevels carve_levels(Carve& c, int mode, int64_t batch, int64_t n, int64_t leaf) {
  WsLevels w;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  w.first_bad = c.take<uint64_t>((size_t)batch);
  w.T = c.take<char>(es * (size_t)batch * (size_t)t_elems(n, leaf));
  return w;
}

int64_t level_leaf(int mode, int64_t n, int32_t opt_leaf) { return opt_leaf ? opt_leaf : default_leaf(mode, n); }

}  // namespace

extern "C" size_t trinv_batched_workspace_bytes(int mode, int64_t batch, const int32_t* n_host,
                                                const trinv_opts* opts) {
  if (batch <= 0) return 0;
  Carve c(nullptr, 0);
  carve_persistent(c, batch);
  if (n_host && batch <= kLevelPathMaxBatch) {
    bool same = n_host[0] >= 128 && n_host[0] <= 1024;
    for (int64_t i = 1; i < batch && same; ++i) same = n_host[i] == n_host[0];
    const trinv_opts o = resolve_opts(opts);
    if (same && (o.leaf == 0 || o.leaf == 16))
      carve_levels(c, mode, batch, n_host[0], level_leaf(mode, n_host[0], o.leaf));
  }
  return c.used;
}

extern "C" int trinv_tril_inverse_batched(int mode, int64_t batch, const int32_t* n_host, const int32_t* n_dev,
                                          const int64_t* off_host, const int64_t* off_dev, const void* L_packed,
                                          void* X_packed, int32_t* status_dev, const trinv_opts* opts, void* ws,
                                          size_t ws_bytes, trinv_stream_t stream) {
  if (batch < 0 || batch > INT32_MAX) return TRINV_ERR_ARG;
  if (batch == 0) return TRINV_OK;
  if (!n_host || !off_host || !n_dev || !off_dev || !L_packed || !X_packed || !status_dev) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32) return TRINV_ERR_UNSUPPORTED;
  const trinv_opts o = resolve_opts(opts);
  if (o.upper) return TRINV_ERR_UNSUPPORTED;
  if (o.leaf != 0 && o.leaf != 16) return TRINV_ERR_ARG;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  int64_t extent = 0;
  double flops = 0.0, bytes = 0.0;
  for (int64_t i = 0; i < batch; ++i) {
    const int64_t n = n_host[i];
    if (n < 1 || n > 1024 || off_host[i] < 0) return TRINV_ERR_ARG;
    extent = std::max<int64_t>(extent, off_host[i] + n * n);
    flops += (double)n * n * n / 3.0;
    bytes += es * ((double)n * (n + 1) / 2 + (double)n * n);  // lower triangle in, full X out
  }
  if (overlaps(L_packed, (size_t)extent * es, X_packed, (size_t)extent * es)) return TRINV_ERR_ARG;
  Carve c(ws, ws_bytes);
  WsPersistent w = carve_persistent(c, batch);
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (level_path(batch, n_host, off_host)) {
    const int64_t n = n_host[0], leaf = level_leaf(mode, n, o.leaf);
    WsLevels wl = carve_levels(c, mode, batch, n, leaf);
    if (!c.ok()) return TRINV_ERR_WORKSPACE;
    HIP_TRY(launch_fill_u64(wl.first_bad, ~0ull, batch, s));
    if (mode == TRINV_F64) {
      HIP_TRY(launch_leaf<double>(n, (const double*)L_packed, n, (double*)X_packed, n, n * n, batch, (int)leaf,
                                  o.unit_diag, nullptr, nullptr, 0, 0, 1.0, wl.first_bad, 1, s));
      HIP_TRY(run_levels<double, double>(n, (const double*)L_packed, n, (double*)X_packed, n, n * n, batch, leaf,
                                         (double*)wl.T, s));
    } else {
      HIP_TRY(launch_leaf<float>(n, (const float*)L_packed, n, (float*)X_packed, n, n * n, batch, (int)leaf,
                                 o.unit_diag, nullptr, nullptr, 0, 0, 1.0, wl.first_bad, 1, s));
      HIP_TRY(run_levels<float, float>(n, (const float*)L_packed, n, (float*)X_packed, n, n * n, batch, leaf,
                                       (float*)wl.T, s));
    }
    HIP_TRY(launch_status_to_i32(wl.first_bad, status_dev, batch, s));
  } else {
    ProfLaunch pl(mode == TRINV_F32 ? "f32_batched" : "f64_batched", flops, bytes, s);
    if (mode == TRINV_F32)
      HIP_TRY(launch_batched<float>(batch, n_dev, off_dev, (const float*)L_packed, (float*)X_packed, status_dev,
                                    w.order, w.queue, o.unit_diag, batched_grid<float>(batch), s));
    else
      HIP_TRY(launch_batched<double>(batch, n_dev, off_dev, (const double*)L_packed, (double*)X_packed, status_dev,
                                     w.order, w.queue, o.unit_diag, batched_grid<double>(batch), s));
  }
  if (!o.blocking) return TRINV_OK;
  std::vector<int32_t> st((size_t)batch);
  HIP_TRY(hipMemcpyAsync(st.data(), status_dev, (size_t)batch * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int32_t v : st)
    if (v < 0) return TRINV_ERR_ARG;  // n_dev disagreed with n_host
  for (int32_t v : st)
    if (v > 0) return TRINV_ERR_SINGULAR;
  return TRINV_OK;
}
