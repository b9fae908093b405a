// float32 instantiations of the batched PCG row kernels (inner solves of the
// mixed-precision refinement): general sliced-ELL pencils.
#include "pcg_kernels.hpp"

namespace airga {
KernelSet<float> kernel_set_f32_band(int wclass, bool exact, int cfg);

KernelSet<float> kernel_set_f32(int wclass, bool exact, bool band, int cfg) {
  if (wclass == 2) return kernel_set_wide<float>(cfg);
  if (band) return kernel_set_f32_band(wclass, exact, cfg);
  return kernel_set_impl<float, false>(wclass, exact, cfg);
}
}  // namespace airga
