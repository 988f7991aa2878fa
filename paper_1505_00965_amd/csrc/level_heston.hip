// Level-sampler kernels of one variant: Heston, full-truncation Euler.
#include "level_kernels.hpp"

namespace mlmc {

template KernelFn<float> pick_variant<kHeston, float>(int, int, int, int, bool, bool);
template KernelFn<double> pick_variant<kHeston, double>(int, int, int, int, bool, bool);

}  // namespace mlmc
