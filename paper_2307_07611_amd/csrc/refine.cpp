// Mixed-precision path: BF16 / FP16 MFMA products with Newton-Schulz
// refinement (placeholder until the low-precision kernels land).
#include "api_internal.h"

namespace trinv {

size_t refine_workspace_bytes(int, int64_t, const trinv_opts&, int64_t) { return 0; }

int refine_inverse(int, int64_t, const double*, int64_t, double*, int64_t, const trinv_opts&, int64_t, void*, size_t,
                   hipStream_t, trinv_info*) {
  return TRINV_ERR_UNSUPPORTED;
}

}  // namespace trinv
