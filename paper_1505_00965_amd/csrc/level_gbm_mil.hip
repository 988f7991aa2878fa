// Level-sampler kernels of one variant: GBM, Milstein.
#include "level_kernels.hpp"

namespace mlmc {

template KernelFn<float> pick_variant<kGBMMil, float>(int, int, int, int, bool, bool);
template KernelFn<double> pick_variant<kGBMMil, double>(int, int, int, int, bool, bool);

}  // namespace mlmc
