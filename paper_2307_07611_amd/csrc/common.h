// Internal definitions shared by the HIP sources of libtrinv (gfx950 only).
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "profile.h"

namespace trinv {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// Number of XCDs (accelerator complex dies) of an MI355X: workgroups are
// dispatched round-robin over them, each with its own L2.
constexpr int kNumXcd = 8;

// Maps a dispatch index to a logical tile index so that each XCD works on
// runs of `chunk` consecutive logical tiles (which share operand panels in
// that XCD's L2) while the runs rotate over the XCDs in logical order (so a
// heavy-first logical order stays heavy-first on every XCD). XCD x takes runs
// x, x + 8, x + 16, ...: in the column-ordered tile lists of the level
// products these cover the same tile rows of successive columns, so their A
// panels stay in that XCD's L2. Valid for any total; indices past the last
// full round map to themselves.
__device__ __forceinline__ int64_t xcd_remap(int64_t w, int64_t total, int chunk) {
  const int64_t round = (int64_t)kNumXcd * chunk;
  const int64_t full = (total / round) * round;
  if (w >= full) return w;
  const int64_t xcd = w % kNumXcd;
  const int64_t q = w / kNumXcd;
  return (q / chunk) * round + xcd * chunk + (q % chunk);
}

__device__ __forceinline__ int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t imax64(int64_t a, int64_t b) { return a > b ? a : b; }

// Round-to-nearest-even conversions (the hardware conversion instructions).
__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }
__device__ __forceinline__ _Float16 to_f16(float x) { return (_Float16)x; }

// Calls f(integral_constant<int, B>), ..., f(integral_constant<int, E-1>): the
// index is a compile-time constant in every call, so register arrays indexed
// by it never need memory.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

}  // namespace trinv
