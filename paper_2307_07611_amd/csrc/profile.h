// Launch profiling hooks (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "trinv.h"

namespace trinv {

bool profiling_on();

// Brackets the launches made during its lifetime with HIP events on stream s
// (when profiling is enabled) and files them under `cls` with the given
// algorithmic flops and bytes.
class ProfLaunch {
 public:
  ProfLaunch(const char* cls, double flops, double bytes, hipStream_t s);
  ~ProfLaunch();
  ProfLaunch(const ProfLaunch&) = delete;
  ProfLaunch& operator=(const ProfLaunch&) = delete;

 private:
  hipStream_t s_;
  long idx_ = -1;
};

}  // namespace trinv
