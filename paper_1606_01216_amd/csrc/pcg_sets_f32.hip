// float32 instantiations of the batched PCG row kernels (inner solves of the
// mixed-precision refinement).
#include "pcg_kernels.hpp"

namespace airga {
KernelSet<float> kernel_set_f32(int wclass, bool exact, int cfg) {
  return kernel_set_impl<float>(wclass, exact, cfg);
}
}  // namespace airga
