// Host-side helpers shared by the C ABI translation units (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "launch.h"
#include "trinv.h"

#define HIP_TRY(...)                               \
  do {                                             \
    hipError_t _e = (__VA_ARGS__);                  \
    if (_e != hipSuccess) return TRINV_ERR_HIP;    \
  } while (0)

namespace trinv {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Bump allocator over the caller's workspace (base == nullptr: size query).
struct Carve {
  char* base;
  size_t used = 0, cap;
  Carve(void* b, size_t c) : base((char*)b), cap(c) {}
  template <typename T>
  T* take(size_t count) {
    const size_t off = used;
    used = align_up(used + count * sizeof(T));
    return base ? (T*)(base + off) : nullptr;
  }
  bool ok() const { return used <= cap; }
};

// One level of the bottom-up recursion: merges of blocks of order hA.
struct Level {
  int64_t hA, span, nmerge, hB_last;
};

// The "nothing computed" state of *info (nullable).
inline void info_reset(trinv_info* info) {
  if (!info) return;
  info->rel_residual = -1.0;
  info->resid_error_est = 0.0;
  info->resid_error_bound = 0.0;
  info->iterations = 0;
  info->first_bad_index = 0;
}

trinv_opts resolve_opts(const trinv_opts* o);
int default_leaf(int mode, int64_t n);
bool combrit_beta(const trinv_opts& o);
bool valid_leaf(int64_t b);
std::vector<Level> levels_of(int64_t n, int64_t leaf);
// Elements of the T workspace one matrix needs (largest level).
int64_t t_elems(int64_t n, int64_t leaf);

// Off-diagonal products of every level for a strided batch of matrices
// (TC = MFMA type). Tws holds batch * t_elems(n, leaf) elements.
template <typename T, typename TC>
hipError_t run_levels(int64_t n, const T* L, int64_t ldl, T* X, int64_t ldx, int64_t stride, int64_t batch,
                      int64_t leaf, T* Tws, hipStream_t s);

int wait_status(hipStream_t s, const uint64_t* status_dev, int64_t n, int64_t* first_bad);
bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes);
size_t span_bytes(int64_t rows, int64_t cols, int64_t ld, size_t es);

// Top level of algorithm COMBRIT on a beta x beta block grid (combrit.cpp):
// ld is the leading dimension of both L and X; status receives the 1-based
// index of the first zero pivot (all ones if none).
size_t combrit_workspace_bytes(int mode, int64_t n, int beta, int64_t leaf);
template <typename T>
hipError_t combrit_t(int64_t n, const T* L, int64_t ld, T* X, int unit, int beta, int64_t leaf, void* ws,
                     size_t ws_bytes, uint64_t* status, hipStream_t s);

// Mixed-precision path (refine.cpp). Orders above kMaxRefineOrder are
// unsupported: the low-precision products keep 32-bit per-lane byte offsets
// within 256 rows of a plane (256 * 2 bytes * leading dimension < 2^32).
constexpr int64_t kMaxRefineOrder = ((int64_t)1 << 23) - 128;
bool refine_order_ok(int64_t n);
size_t refine_workspace_bytes(int mode, int64_t n, const trinv_opts& o, int64_t leaf);
int refine_inverse(int mode, int64_t n, const double* L, int64_t ldl, double* X, int64_t ldx, const trinv_opts& o,
                   int64_t leaf, void* ws, size_t ws_bytes, hipStream_t s, trinv_info* info);

}  // namespace trinv
