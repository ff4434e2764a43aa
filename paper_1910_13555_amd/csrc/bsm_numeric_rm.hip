// Numeric kernels: Row-major operands, one problem.
#include "bsm_numeric_core.h"

namespace bsm {

hipError_t launch_numeric_rm(hipStream_t s, const NumParams& p, bool cin) {
  return cin ? launch_kernels<false, true, false>(s, p) : launch_kernels<false, false, false>(s, p);
}

}  // namespace bsm
