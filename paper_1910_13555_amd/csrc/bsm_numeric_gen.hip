// Numeric kernels: Generic layouts (transposed and split-mode operands, gradients).
#include "bsm_numeric_core.h"

namespace bsm {

hipError_t launch_numeric_gen(hipStream_t s, const NumParams& p, bool batch) {
  return batch ? launch_kernels<true, false, true>(s, p) : launch_kernels<true, false, false>(s, p);
}

}  // namespace bsm
