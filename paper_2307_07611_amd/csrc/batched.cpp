// Batched inversion of many independent lower-triangular matrices.
//
// Uniform orders run the same level recursion as the single-matrix path with
// the batch as an extra launch dimension (every launch covers all matrices).
#include <algorithm>

#include "api_internal.h"

using namespace trinv;

namespace {

bool uniform_sizes(int64_t batch, const int32_t* n_host, const int64_t* off_host) {
  for (int64_t i = 0; i < batch; ++i) {
    if (n_host[i] != n_host[0]) return false;
    if (off_host[i] != i * (int64_t)n_host[0] * n_host[0]) return false;
  }
  return true;
}

struct WsUniform {
  uint64_t* first_bad;
  void* T;
};

WsUniform carve_uniform(Carve& c, int mode, int64_t batch, int64_t n, int64_t leaf) {
  WsUniform w;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  w.first_bad = c.take<uint64_t>((size_t)batch);
  w.T = c.take<char>(es * (size_t)batch * (size_t)t_elems(n, leaf));
  return w;
}

}  // namespace

extern "C" size_t trinv_batched_workspace_bytes(int mode, int64_t batch, const int32_t* n_host,
                                                const trinv_opts* opts) {
  if (batch <= 0 || !n_host) return 0;
  const trinv_opts o = resolve_opts(opts);
  const int64_t n = n_host[0];
  const int64_t leaf = o.leaf ? o.leaf : default_leaf(mode, n);
  Carve c(nullptr, 0);
  carve_uniform(c, mode, batch, n, leaf);
  return c.used;
}

extern "C" int trinv_tril_inverse_batched(int mode, int64_t batch, const int32_t* n_host, const int32_t* n_dev,
                                          const int64_t* off_host, const int64_t* off_dev, const void* L_packed,
                                          void* X_packed, int32_t* status_dev, const trinv_opts* opts, void* ws,
                                          size_t ws_bytes, trinv_stream_t stream) {
  (void)n_dev;
  (void)off_dev;
  if (batch < 0) return TRINV_ERR_ARG;
  if (batch == 0) return TRINV_OK;
  if (!n_host || !off_host || !L_packed || !X_packed || !status_dev) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32) return TRINV_ERR_UNSUPPORTED;
  for (int64_t i = 0; i < batch; ++i)
    if (n_host[i] < 1 || n_host[i] > 1024 || off_host[i] < 0) return TRINV_ERR_ARG;
  if (!uniform_sizes(batch, n_host, off_host)) return TRINV_ERR_UNSUPPORTED;
  const trinv_opts o = resolve_opts(opts);
  const int64_t n = n_host[0];
  const int64_t leaf = o.leaf ? o.leaf : default_leaf(mode, n);
  if (!valid_leaf(leaf)) return TRINV_ERR_ARG;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  const size_t nb = (size_t)batch * n * n * es;
  if (overlaps(L_packed, nb, X_packed, nb)) return TRINV_ERR_ARG;
  Carve c(ws, ws_bytes);
  WsUniform w = carve_uniform(c, mode, batch, n, leaf);
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_fill_u64(w.first_bad, ~0ull, batch, s));
  if (mode == TRINV_F64) {
    HIP_TRY(launch_leaf<double>(n, (const double*)L_packed, n, (double*)X_packed, n, n * n, batch, (int)leaf,
                                o.unit_diag, nullptr, nullptr, 0, 0, w.first_bad, 1, s));
    HIP_TRY(run_levels<double, double>(n, (const double*)L_packed, n, (double*)X_packed, n, n * n, batch, leaf,
                                       (double*)w.T, s));
  } else {
    HIP_TRY(launch_leaf<float>(n, (const float*)L_packed, n, (float*)X_packed, n, n * n, batch, (int)leaf,
                               o.unit_diag, nullptr, nullptr, 0, 0, w.first_bad, 1, s));
    HIP_TRY(run_levels<float, float>(n, (const float*)L_packed, n, (float*)X_packed, n, n * n, batch, leaf,
                                     (float*)w.T, s));
  }
  HIP_TRY(launch_status_to_i32(w.first_bad, status_dev, batch, s));
  if (!o.blocking) return TRINV_OK;
  HIP_TRY(hipStreamSynchronize(s));
  return TRINV_OK;
}
