// Batched inversion of many independent lower-triangular matrices of order
// 1..1024: a one-workgroup plan kernel sorts the matrices by order, then one
// persistent launch (persistent.hip) inverts them, each workgroup taking whole
// matrices from a device-side queue. Uniform and uneven batches take the same
// path.
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

}  // namespace

extern "C" size_t trinv_batched_workspace_bytes(int mode, int64_t batch, const int32_t* n_host,
                                                const trinv_opts* opts) {
  (void)mode;
  (void)n_host;
  (void)opts;
  if (batch <= 0) return 0;
  Carve c(nullptr, 0);
  carve_persistent(c, batch);
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
  {
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
