// Batched inversion of many independent lower-triangular matrices of order
// 1..1024: a one-workgroup plan kernel sorts the matrices by order, then one
// persistent launch (persistent.hip) inverts them, each workgroup taking whole
// matrices from a device-side queue. A uniform batch with fewer matrices than
// compute units instead runs the level recursion with the batch as an extra
// launch dimension (every level product spread over the whole chip).
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
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

// Tunable parameters of the persistent launch: the leaf order (the
// recursion's cut-off: 32 or 64; 0 = the mode's default) and the resident
// workgroups per CU (0: the occupancy limit).
struct PersistentConfig {
  int leaf = 0;
  int per_cu = 0;
};

// Default leaf order: 64 for FP32; 32 for FP64 (a 64-leaf stage of FP64 L^T
// takes 136 KB of LDS, one workgroup per CU).
int default_batched_leaf(int mode) { return mode == TRINV_F32 ? 64 : 32; }

// The kernel's work depends on the orders only: a batch is keyed by its mode,
// count, sum of orders, sum of squared orders and largest order.
typedef std::tuple<int, int64_t, int64_t, int64_t, int> BatchKey;

std::mutex g_tuned_mu;
std::map<BatchKey, PersistentConfig> g_tuned;  // autotuner results, per process

PersistentConfig tuned_config(const BatchKey& k) {
  std::lock_guard<std::mutex> lock(g_tuned_mu);
  auto it = g_tuned.find(k);
  return it == g_tuned.end() ? PersistentConfig{} : it->second;
}

// Validates the batch (as trinv_tril_inverse_batched documents) and fills
// its key and algorithmic work; TRINV_OK or the error status.
int check_batch(int mode, int64_t batch, const int32_t* n_host, const int32_t* n_dev, const int64_t* off_host,
                const int64_t* off_dev, const void* L_packed, void* X_packed, int32_t* status_dev,
                const trinv_opts& o, BatchKey* key, double* flops, double* bytes) {
  if (batch < 0 || batch > INT32_MAX) return TRINV_ERR_ARG;
  if (!n_host || !off_host || !n_dev || !off_dev || !L_packed || !X_packed || !status_dev) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32) return TRINV_ERR_UNSUPPORTED;
  if (o.upper) return TRINV_ERR_UNSUPPORTED;
  if (o.leaf != 0 && o.leaf != 32 && o.leaf != 64) return TRINV_ERR_ARG;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  int64_t extent = 0, s1 = 0, s2 = 0;
  int nmax = 0;
  *flops = 0.0;
  *bytes = 0.0;
  for (int64_t i = 0; i < batch; ++i) {
    const int64_t n = n_host[i];
    if (n < 1 || n > 1024 || off_host[i] < 0) return TRINV_ERR_ARG;
    extent = std::max<int64_t>(extent, off_host[i] + n * n);
    *flops += (double)n * n * n / 3.0;
    *bytes += es * ((double)n * (n + 1) / 2 + (double)n * n);  // lower triangle in, full X out
    s1 += n;
    s2 += n * n;
    nmax = std::max<int>(nmax, (int)n);
  }
  if (overlaps(L_packed, (size_t)extent * es, X_packed, (size_t)extent * es)) return TRINV_ERR_ARG;
  *key = BatchKey(mode, batch, s1, s2, nmax);
  return TRINV_OK;
}

// The persistent launch pair with configuration c (opts.leaf, when set,
// overrides the configuration's leaf).
hipError_t launch_persistent(int mode, int64_t batch, const int32_t* n_dev, const int64_t* off_dev,
                             const void* L_packed, void* X_packed, int32_t* status_dev, const WsPersistent& w,
                             const trinv_opts& o, const PersistentConfig& c, hipStream_t s) {
  const int leaf = o.leaf ? o.leaf : (c.leaf ? c.leaf : default_batched_leaf(mode));
  if (mode == TRINV_F32)
    return launch_batched<float>(batch, n_dev, off_dev, (const float*)L_packed, (float*)X_packed, status_dev,
                                 w.order, w.queue, o.unit_diag, batched_grid<float>(batch, leaf, c.per_cu), leaf, s);
  return launch_batched<double>(batch, n_dev, off_dev, (const double*)L_packed, (double*)X_packed, status_dev,
                                w.order, w.queue, o.unit_diag, batched_grid<double>(batch, leaf, c.per_cu), leaf, s);
}

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
    if (same && (o.leaf == 0 || o.leaf == 32 || o.leaf == 64))
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
  const trinv_opts o = resolve_opts(opts);
  BatchKey key;
  double flops = 0.0, bytes = 0.0;
  const int chk = check_batch(mode, batch, n_host, n_dev, off_host, off_dev, L_packed, X_packed, status_dev, o, &key,
                              &flops, &bytes);
  if (chk != TRINV_OK) return chk;
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
    if (mode == TRINV_F64)
      HIP_TRY(launch_nonfinite_status<double>((const double*)X_packed, n, n * n, batch, status_dev, s));
    else
      HIP_TRY(launch_nonfinite_status<float>((const float*)X_packed, n, n * n, batch, status_dev, s));
  } else {
    ProfLaunch pl(mode == TRINV_F32 ? "f32_batched" : "f64_batched", flops, bytes, s);
    HIP_TRY(launch_persistent(mode, batch, n_dev, off_dev, L_packed, X_packed, status_dev, w, o, tuned_config(key),
                              s));
  }
  if (!o.blocking) return TRINV_OK;
  std::vector<int32_t> st((size_t)batch);
  HIP_TRY(hipMemcpyAsync(st.data(), status_dev, (size_t)batch * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int32_t v : st)
    if (v == -1) return TRINV_ERR_ARG;  // n_dev disagreed with n_host
  for (int32_t v : st)
    if (v > 0) return TRINV_ERR_SINGULAR;
  for (int32_t v : st)
    if (v == -2) return TRINV_ERR_NONFINITE;
  return TRINV_OK;
}

extern "C" int trinv_batched_autotune(int mode, int64_t batch, const int32_t* n_host, const int32_t* n_dev,
                                      const int64_t* off_host, const int64_t* off_dev, const void* L_packed,
                                      void* X_packed, int32_t* status_dev, const trinv_opts* opts, void* ws,
                                      size_t ws_bytes, trinv_stream_t stream, trinv_batched_config* out) {
  if (out) *out = trinv_batched_config{0, 0, -1.0f};
  if (batch < 0 || batch > INT32_MAX) return TRINV_ERR_ARG;
  if (batch == 0) return TRINV_OK;
  const trinv_opts o = resolve_opts(opts);
  BatchKey key;
  double flops = 0.0, bytes = 0.0;
  const int chk = check_batch(mode, batch, n_host, n_dev, off_host, off_dev, L_packed, X_packed, status_dev, o, &key,
                              &flops, &bytes);
  if (chk != TRINV_OK) return chk;
  Carve c(ws, ws_bytes);
  WsPersistent w = carve_persistent(c, batch);
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  if (level_path(batch, n_host, off_host)) return TRINV_OK;  // the level path has nothing to tune
  hipStream_t s = (hipStream_t)stream;
  std::vector<PersistentConfig> cands;
  for (int leaf : {32, 64}) {
    if (o.leaf && leaf != o.leaf) continue;
    const int occ = mode == TRINV_F32 ? batched_occupancy<float>(leaf, nullptr) : batched_occupancy<double>(leaf, nullptr);
    for (int k = 1; k <= occ; k *= 2) cands.push_back(PersistentConfig{leaf, k});
    if ((occ & (occ - 1)) != 0) cands.push_back(PersistentConfig{leaf, occ});
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return TRINV_ERR_HIP;
  }
  PersistentConfig best;
  float best_ms = -1.0f;
  hipError_t err = hipSuccess;
  for (const PersistentConfig& cfg : cands) {
    // one untimed launch, then the fastest of three
    err = launch_persistent(mode, batch, n_dev, off_dev, L_packed, X_packed, status_dev, w, o, cfg, s);
    float ms = -1.0f;
    for (int r = 0; r < 3 && err == hipSuccess; ++r) {
      if ((err = hipEventRecord(e0, s)) != hipSuccess) break;
      if ((err = launch_persistent(mode, batch, n_dev, off_dev, L_packed, X_packed, status_dev, w, o, cfg, s)) !=
          hipSuccess)
        break;
      if ((err = hipEventRecord(e1, s)) != hipSuccess) break;
      if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
      float t = 0.0f;
      if ((err = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) break;
      if (ms < 0.0f || t < ms) ms = t;
    }
    if (err != hipSuccess) break;
    if (best_ms < 0.0f || ms < best_ms) {
      best_ms = ms;
      best = cfg;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return TRINV_ERR_HIP;
  {
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    g_tuned[key] = best;
  }
  // leave X and status from the chosen configuration
  HIP_TRY(launch_persistent(mode, batch, n_dev, off_dev, L_packed, X_packed, status_dev, w, o, best, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (out) *out = trinv_batched_config{best.leaf, best.per_cu, best_ms};
  return TRINV_OK;
}

extern "C" int trinv_batched_set_config(int mode, int64_t batch, const int32_t* n_host,
                                        const trinv_batched_config* cfg) {
  if (batch <= 0 || batch > INT32_MAX || !n_host || !cfg) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32) return TRINV_ERR_UNSUPPORTED;
  if ((cfg->leaf != 32 && cfg->leaf != 64) || cfg->wgs_per_cu < 0) return TRINV_ERR_ARG;
  int64_t s1 = 0, s2 = 0;
  int nmax = 0;
  for (int64_t i = 0; i < batch; ++i) {
    const int64_t n = n_host[i];
    if (n < 1 || n > 1024) return TRINV_ERR_ARG;
    s1 += n;
    s2 += n * n;
    nmax = std::max<int>(nmax, (int)n);
  }
  std::lock_guard<std::mutex> lock(g_tuned_mu);
  g_tuned[BatchKey(mode, batch, s1, s2, nmax)] = PersistentConfig{cfg->leaf, cfg->wgs_per_cu};
  return TRINV_OK;
}

// Allocation-free variant for callers that cannot allocate device memory
// (graph capture, serving loops): the persistent launch with its plan and
// queue in the library's per-device scratch instead of a workspace.
extern "C" int trinv_tril_inverse_batched_noalloc(int mode, int64_t batch, const int32_t* n_host,
                                                  const int32_t* n_dev, const int64_t* off_host,
                                                  const int64_t* off_dev, const void* L_packed, void* X_packed,
                                                  int32_t* status_dev, const trinv_opts* opts,
                                                  trinv_stream_t stream) {
  if (batch < 0 || batch > kNoAllocMaxBatch) return TRINV_ERR_ARG;
  if (batch == 0) return TRINV_OK;
  const trinv_opts o = resolve_opts(opts);
  BatchKey key;
  double flops = 0.0, bytes = 0.0;
  const int chk = check_batch(mode, batch, n_host, n_dev, off_host, off_dev, L_packed, X_packed, status_dev, o, &key,
                              &flops, &bytes);
  if (chk != TRINV_OK) return chk;
  WsPersistent w{};
  HIP_TRY(batched_scratch(&w.order, &w.queue));
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_persistent(mode, batch, n_dev, off_dev, L_packed, X_packed, status_dev, w, o, tuned_config(key), s));
  if (!o.blocking) return TRINV_OK;
  // statuses in fixed-size pieces (no host allocation either)
  int32_t st[1024];
  int worst = TRINV_OK;
  for (int64_t i0 = 0; i0 < batch; i0 += 1024) {
    const int64_t cnt = std::min<int64_t>(1024, batch - i0);
    HIP_TRY(hipMemcpyAsync(st, status_dev + i0, (size_t)cnt * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t i = 0; i < cnt; ++i) {
      if (st[i] == -1) return TRINV_ERR_ARG;  // n_dev disagreed with n_host
      if (st[i] > 0) worst = TRINV_ERR_SINGULAR;
      if (st[i] == -2 && worst == TRINV_OK) worst = TRINV_ERR_NONFINITE;
    }
  }
  return worst;
}
