// float64 instantiations of the batched PCG row kernels (plain float64 solves): banded pencils (bandwidth <= 64), neighbour entries staged in LDS.
#include "pcg_kernels.hpp"

namespace airga {
KernelSet<double> kernel_set_f64_band(int wclass, bool exact, int cfg) {
  return kernel_set_impl<double, true>(wclass, exact, cfg);
}
}  // namespace airga
