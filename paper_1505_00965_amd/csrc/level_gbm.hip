// Level-sampler kernels of one variant: GBM, Euler--Maruyama.
#include "level_kernels.hpp"

namespace mlmc {

template KernelFn<float> pick_variant<kGBM, float>(int, int, int, int, bool, bool);
template KernelFn<double> pick_variant<kGBM, double>(int, int, int, int, bool, bool);

}  // namespace mlmc
