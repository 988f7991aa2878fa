// Persistent all-levels sampler kernels of one variant: Heston, full-truncation Euler.
#include "persistent.hpp"

namespace mlmc {

template PersistentFn pick_persistent_variant<kHeston>(int, int, int, bool);

}  // namespace mlmc
