// Persistent all-levels sampler kernels of one variant: GBM, Euler--Maruyama.
#include "persistent.hpp"

namespace mlmc {

template PersistentFn pick_persistent_variant<kGBM>(int, int, int, bool);

}  // namespace mlmc
