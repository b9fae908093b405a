// float64 instantiations of the batched PCG row kernels (plain float64 solves).
#include "pcg_kernels.hpp"

namespace airga {
KernelSet<double> kernel_set_f64(int wclass, bool exact, int cfg) {
  return kernel_set_impl<double>(wclass, exact, cfg);
}
}  // namespace airga
