// float64 instantiations of the batched PCG row kernels (plain float64 solves): general sliced-ELL pencils.
#include "pcg_kernels.hpp"

namespace airga {
KernelSet<double> kernel_set_f64_band(int wclass, bool exact, int cfg);

KernelSet<double> kernel_set_f64(int wclass, bool exact, bool band, int cfg) {
  if (wclass == 2) return kernel_set_wide<double>(cfg);
  if (band) return kernel_set_f64_band(wclass, exact, cfg);
  return kernel_set_impl<double, false>(wclass, exact, cfg);
}
}  // namespace airga
