// Batched inversion of many independent lower-triangular matrices of order
// 1..1024: a one-workgroup plan kernel sorts the matrices by order, then one
// persistent launch (persistent.hip) inverts them, each workgroup taking whole
// matrices from a device-side queue. A uniform batch with fewer matrices than
// compute units instead runs the level recursion with the batch as an extra
// launch dimension (every level product spread over the whole chip).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
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

// Upper input (opts.upper): the transposes U_i^T staged densely packed (Ut,
// at the dense offsets doff), inverted as lower into Xt at the same offsets,
// and Xt_i^T written to X_i. The persistent and level launches take one
// offset array for L and X, hence the dense staging of both.
struct WsUpper {
  int64_t* doff = nullptr;
  void* Ut = nullptr;
  void* Xt = nullptr;
  int64_t elems = 0;  // sum of n_i^2
};

WsUpper carve_upper(Carve& c, int mode, int64_t batch, const int32_t* n_host) {
  WsUpper w;
  const size_t es = mode == TRINV_F32 ? 4 : 8;
  for (int64_t i = 0; i < batch; ++i) w.elems += (int64_t)n_host[i] * n_host[i];
  w.doff = c.take<int64_t>((size_t)batch);
  w.Ut = c.take<char>(es * (size_t)w.elems);
  w.Xt = c.take<char>(es * (size_t)w.elems);
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
// recursion's cut-off: 32 or 64; 0 = the mode's default), the resident
// workgroups per CU (0: the occupancy limit) and the largest tile of the
// level products (64 or 128; 0 = 128).
struct PersistentConfig {
  int leaf = 0;
  int per_cu = 0;
  int tile = 0;
};

// Default leaf order: 64 for FP32; 32 for FP64 (a 64-leaf stage of FP64 L^T
// takes 136 KB of LDS, one workgroup per CU).
int default_batched_leaf(int mode) { return mode == TRINV_F32 ? 64 : 32; }

// The kernel's work depends on the orders only: a batch is keyed by its mode,
// count, sum of orders, sum of squared orders and largest order.
typedef std::tuple<int, int64_t, int64_t, int64_t, int> BatchKey;

std::mutex g_tuned_mu;
std::map<BatchKey, PersistentConfig> g_tuned;  // autotuner results, per process

// On-disk tuning cache (opt-in): the environment variable TRINV_TUNE_CACHE
// names a text file of lines "device mode count sum sum_sq largest leaf
// wgs_per_cu tile ms", device = the GPU's architecture name and CU count. The
// lines of the current device are loaded at the first lookup of the process
// (later lines win); every autotuner result is appended.
bool g_disk_loaded = false;

std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return std::string();
  std::string arch(p.gcnArchName);
  for (char& ch : arch)
    if (ch == ' ' || ch == '\t' || ch == '\n') ch = '_';
  return arch + "/" + std::to_string(p.multiProcessorCount);
}

void load_disk_cache_locked() {
  if (g_disk_loaded) return;
  g_disk_loaded = true;
  const char* path = std::getenv("TRINV_TUNE_CACHE");
  if (!path || !*path) return;
  const std::string tag = device_tag();
  if (tag.empty()) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char t[160];
  int mode = 0, nmax = 0, leaf = 0, per_cu = 0, tile = 0;
  long long batch = 0, s1 = 0, s2 = 0;
  float ms = 0.0f;
  while (std::fscanf(f, "%159s %d %lld %lld %lld %d %d %d %d %f", t, &mode, &batch, &s1, &s2, &nmax, &leaf, &per_cu,
                     &tile, &ms) == 10)
    if (tag == t && (leaf == 32 || leaf == 64) && per_cu >= 0 && (tile == 0 || tile == 64 || tile == 128))
      g_tuned[BatchKey(mode, batch, s1, s2, nmax)] = PersistentConfig{leaf, per_cu, tile};
  std::fclose(f);
}

void append_disk_cache_locked(const BatchKey& k, const PersistentConfig& c, float ms) {
  const char* path = std::getenv("TRINV_TUNE_CACHE");
  if (!path || !*path) return;
  const std::string tag = device_tag();
  if (tag.empty()) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %lld %lld %lld %d %d %d %d %.4f\n", tag.c_str(), std::get<0>(k), (long long)std::get<1>(k),
               (long long)std::get<2>(k), (long long)std::get<3>(k), std::get<4>(k), c.leaf, c.per_cu, c.tile, ms);
  std::fclose(f);
}

PersistentConfig tuned_config(const BatchKey& k) {
  std::lock_guard<std::mutex> lock(g_tuned_mu);
  load_disk_cache_locked();
  auto it = g_tuned.find(k);
  return it == g_tuned.end() ? PersistentConfig{} : it->second;
}

// Order signature of a batch (as check_batch keys it); false if an order is
// outside 1..1024.
bool batch_key(int mode, int64_t batch, const int32_t* n_host, BatchKey* key) {
  int64_t s1 = 0, s2 = 0;
  int nmax = 0;
  for (int64_t i = 0; i < batch; ++i) {
    const int64_t n = n_host[i];
    if (n < 1 || n > 1024) return false;
    s1 += n;
    s2 += n * n;
    nmax = std::max<int>(nmax, (int)n);
  }
  *key = BatchKey(mode, batch, s1, s2, nmax);
  return true;
}

// Validates the batch (as trinv_tril_inverse_batched documents) and fills
// its key and algorithmic work; TRINV_OK or the error status.
int check_batch(int mode, int64_t batch, const int32_t* n_host, const int32_t* n_dev, const int64_t* off_host,
                const int64_t* off_dev, const void* L_packed, void* X_packed, int32_t* status_dev,
                const trinv_opts& o, BatchKey* key, double* flops, double* bytes) {
  if (batch < 0 || batch > INT32_MAX) return TRINV_ERR_ARG;
  if (!n_host || !off_host || !n_dev || !off_dev || !L_packed || !X_packed || !status_dev) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32) return TRINV_ERR_UNSUPPORTED;
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
  const int tile = c.tile ? c.tile : 128;
  if (mode == TRINV_F32)
    return launch_batched<float>(batch, n_dev, off_dev, (const float*)L_packed, (float*)X_packed, status_dev,
                                 w.order, w.queue, o.unit_diag, batched_grid<float>(batch, leaf, c.per_cu), leaf, tile,
                                 s);
  return launch_batched<double>(batch, n_dev, off_dev, (const double*)L_packed, (double*)X_packed, status_dev,
                                w.order, w.queue, o.unit_diag, batched_grid<double>(batch, leaf, c.per_cu), leaf, tile,
                                s);
}

}  // namespace

extern "C" size_t trinv_batched_workspace_bytes(int mode, int64_t batch, const int32_t* n_host,
                                                const trinv_opts* opts) {
  if (batch <= 0) return 0;
  Carve c(nullptr, 0);
  carve_persistent(c, batch);
  const trinv_opts o = resolve_opts(opts);
  if (o.upper && n_host) {
    for (int64_t i = 0; i < batch; ++i)
      if (n_host[i] < 1 || n_host[i] > 1024) return 0;
    carve_upper(c, mode, batch, n_host);
  }
  if (n_host && batch <= kLevelPathMaxBatch) {
    bool same = n_host[0] >= 128 && n_host[0] <= 1024;
    for (int64_t i = 1; i < batch && same; ++i) same = n_host[i] == n_host[0];
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
  WsUpper wu;
  if (o.upper) wu = carve_upper(c, mode, batch, n_host);
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  // the lower inversion's operands: the caller's, or the dense transposes
  const void* Lk = L_packed;
  void* Xk = X_packed;
  const int64_t* offk_dev = off_dev;
  const int64_t* offk_host = off_host;
  std::vector<int64_t> dense;
  if (o.upper) {
    dense.resize((size_t)batch);
    int64_t acc = 0;
    for (int64_t i = 0; i < batch; ++i) {
      dense[(size_t)i] = acc;
      acc += (int64_t)n_host[i] * n_host[i];
    }
    HIP_TRY(launch_dense_offsets(n_dev, batch, wu.doff, s));
    if (mode == TRINV_F64)
      HIP_TRY(launch_transpose_packed<double>(batch, n_dev, off_dev, (const double*)L_packed, wu.doff,
                                              (double*)wu.Ut, wu.elems, s));
    else
      HIP_TRY(launch_transpose_packed<float>(batch, n_dev, off_dev, (const float*)L_packed, wu.doff,
                                             (float*)wu.Ut, wu.elems, s));
    Lk = wu.Ut;
    Xk = wu.Xt;
    offk_dev = wu.doff;
    offk_host = dense.data();
  }
  if (level_path(batch, n_host, offk_host)) {
    const int64_t n = n_host[0], leaf = level_leaf(mode, n, o.leaf);
    WsLevels wl = carve_levels(c, mode, batch, n, leaf);
    if (!c.ok()) return TRINV_ERR_WORKSPACE;
    HIP_TRY(launch_fill_u64(wl.first_bad, ~0ull, batch, s));
    if (mode == TRINV_F64) {
      HIP_TRY(launch_leaf<double>(n, (const double*)Lk, n, (double*)Xk, n, n * n, batch, (int)leaf,
                                  o.unit_diag, nullptr, nullptr, 0, 0, 1.0, wl.first_bad, 1, s));
      HIP_TRY(run_levels<double, double>(n, (const double*)Lk, n, (double*)Xk, n, n * n, batch, leaf,
                                         (double*)wl.T, s));
    } else {
      HIP_TRY(launch_leaf<float>(n, (const float*)Lk, n, (float*)Xk, n, n * n, batch, (int)leaf,
                                 o.unit_diag, nullptr, nullptr, 0, 0, 1.0, wl.first_bad, 1, s));
      HIP_TRY(run_levels<float, float>(n, (const float*)Lk, n, (float*)Xk, n, n * n, batch, leaf,
                                       (float*)wl.T, s));
    }
    HIP_TRY(launch_status_to_i32(wl.first_bad, status_dev, batch, s));
    if (mode == TRINV_F64)
      HIP_TRY(launch_nonfinite_status<double>((const double*)Xk, n, n * n, batch, status_dev, s));
    else
      HIP_TRY(launch_nonfinite_status<float>((const float*)Xk, n, n * n, batch, status_dev, s));
  } else {
    ProfLaunch pl(mode == TRINV_F32 ? "f32_batched" : "f64_batched", flops, bytes, s);
    HIP_TRY(launch_persistent(mode, batch, n_dev, offk_dev, Lk, Xk, status_dev, w, o, tuned_config(key), s));
  }
  if (o.upper) {  // X_i = (Xt_i)^T, the upper inverse (zeros below its diagonal)
    if (mode == TRINV_F64)
      HIP_TRY(launch_transpose_packed<double>(batch, n_dev, wu.doff, (const double*)wu.Xt, off_dev,
                                              (double*)X_packed, INT64_MAX, s));
    else
      HIP_TRY(launch_transpose_packed<float>(batch, n_dev, wu.doff, (const float*)wu.Xt, off_dev,
                                             (float*)X_packed, INT64_MAX, s));
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
  if (out) *out = trinv_batched_config{0, 0, -1.0f, 0};
  if (batch < 0 || batch > INT32_MAX) return TRINV_ERR_ARG;
  if (batch == 0) return TRINV_OK;
  const trinv_opts o = resolve_opts(opts);
  BatchKey key;
  double flops = 0.0, bytes = 0.0;
  const int chk = check_batch(mode, batch, n_host, n_dev, off_host, off_dev, L_packed, X_packed, status_dev, o, &key,
                              &flops, &bytes);
  if (chk != TRINV_OK) return chk;
  if (o.upper) return TRINV_ERR_UNSUPPORTED;  // tune the lower form: the configuration serves both
  Carve c(ws, ws_bytes);
  WsPersistent w = carve_persistent(c, batch);
  if (!ws || !c.ok()) return TRINV_ERR_WORKSPACE;
  if (level_path(batch, n_host, off_host)) return TRINV_OK;  // the level path has nothing to tune
  hipStream_t s = (hipStream_t)stream;
  std::vector<PersistentConfig> cands;
  for (int leaf : {32, 64}) {
    if (o.leaf && leaf != o.leaf) continue;
    const int occ = mode == TRINV_F32 ? batched_occupancy<float>(leaf, nullptr) : batched_occupancy<double>(leaf, nullptr);
    for (int tile : {64, 128}) {
      for (int k = 1; k <= occ; k *= 2) cands.push_back(PersistentConfig{leaf, k, tile});
      if ((occ & (occ - 1)) != 0) cands.push_back(PersistentConfig{leaf, occ, tile});
    }
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
    load_disk_cache_locked();
    g_tuned[key] = best;
    append_disk_cache_locked(key, best, best_ms);
  }
  // leave X and status from the chosen configuration
  HIP_TRY(launch_persistent(mode, batch, n_dev, off_dev, L_packed, X_packed, status_dev, w, o, best, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (out) *out = trinv_batched_config{best.leaf, best.per_cu, best_ms, best.tile};
  return TRINV_OK;
}

extern "C" int trinv_batched_set_config(int mode, int64_t batch, const int32_t* n_host,
                                        const trinv_batched_config* cfg) {
  if (batch <= 0 || batch > INT32_MAX || !n_host || !cfg) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32) return TRINV_ERR_UNSUPPORTED;
  if ((cfg->leaf != 32 && cfg->leaf != 64) || cfg->wgs_per_cu < 0 ||
      (cfg->tile != 0 && cfg->tile != 64 && cfg->tile != 128))
    return TRINV_ERR_ARG;
  BatchKey key;
  if (!batch_key(mode, batch, n_host, &key)) return TRINV_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_tuned_mu);
  load_disk_cache_locked();
  g_tuned[key] = PersistentConfig{cfg->leaf, cfg->wgs_per_cu, cfg->tile};
  return TRINV_OK;
}

extern "C" int trinv_batched_get_config(int mode, int64_t batch, const int32_t* n_host, trinv_batched_config* cfg) {
  if (batch <= 0 || batch > INT32_MAX || !n_host || !cfg) return TRINV_ERR_ARG;
  if (mode != TRINV_F64 && mode != TRINV_F32) return TRINV_ERR_UNSUPPORTED;
  BatchKey key;
  if (!batch_key(mode, batch, n_host, &key)) return TRINV_ERR_ARG;
  const PersistentConfig c = tuned_config(key);
  *cfg = trinv_batched_config{c.leaf ? c.leaf : default_batched_leaf(mode), c.per_cu, -1.0f, c.tile ? c.tile : 128};
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
  if (o.upper) return TRINV_ERR_UNSUPPORTED;  // its transposed staging needs a workspace
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
