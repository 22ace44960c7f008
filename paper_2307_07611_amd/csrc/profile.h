// Launch profiling hooks (internal).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "trinv.h"

namespace trinv {

bool profiling_on();

// Times the launches made on this thread during its lifetime (when profiling
// is enabled) and files them under `cls` with the given algorithmic flops and
// bytes. The timing events travel with the kernel dispatches themselves
// (hipExtLaunchKernel: the first launch's start, the last launch's end), so
// no marker packets sit between the kernels; a scope without launches
// records an empty interval.
class ProfLaunch {
 public:
  ProfLaunch(const char* cls, double flops, double bytes, hipStream_t s);
  ~ProfLaunch();
  ProfLaunch(const ProfLaunch&) = delete;
  ProfLaunch& operator=(const ProfLaunch&) = delete;

 private:
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
  int launched_ = 0;
  ProfLaunch* outer_ = nullptr;
  friend struct LaunchEvents next_launch_events();
};

// Events to attach to the next launch on this thread: both null outside an
// active ProfLaunch scope; else the scope's start event (first launch only)
// and its stop event (every launch: the last one's end closes the interval).
struct LaunchEvents {
  hipEvent_t start, stop;
};
LaunchEvents next_launch_events();

}  // namespace trinv

// Every kernel launch of the library goes through this macro.
#define TRINV_LAUNCH(KERNEL, GRID, BLOCK, LDS, STREAM, ...)                                          \
  do {                                                                                              \
    const ::trinv::LaunchEvents ev_ = ::trinv::next_launch_events();                                \
    if (ev_.stop)                                                                                   \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, STREAM, ev_.start, ev_.stop, 0, __VA_ARGS__); \
    else                                                                                            \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, STREAM, __VA_ARGS__);                            \
  } while (0)
