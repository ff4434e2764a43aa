// Numeric kernels: Row-major operands, batches (per-problem table).
#include "bsm_numeric_core.h"

namespace bsm {

hipError_t launch_numeric_rm_batch(hipStream_t s, const NumParams& p, bool cin) {
  return cin ? launch_kernels<false, true, true>(s, p) : launch_kernels<false, false, true>(s, p);
}

}  // namespace bsm
