// float32 instantiations of the batched PCG row kernels (inner solves of the
// mixed-precision refinement): banded pencils (bandwidth <= 64), neighbour entries staged in LDS.
#include "pcg_kernels.hpp"

namespace airga {
KernelSet<float> kernel_set_f32_band(int wclass, bool exact, int cfg) {
  return kernel_set_impl<float, true>(wclass, exact, cfg);
}
}  // namespace airga
