// Persistent all-levels sampler kernels of one variant: GBM, Milstein.
#include "persistent.hpp"

namespace mlmc {

template PersistentFn pick_persistent_variant<kGBMMil>(int, int, int, bool);

}  // namespace mlmc
