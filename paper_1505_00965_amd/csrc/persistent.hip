// Persistent all-levels form (work table + graph): see run_persistent.
#include "context.hpp"
#include "driver.hpp"

namespace mlmc {

mlmc_status run_persistent(mlmc_ctx* ctx, const mlmc_model&, const mlmc_payoff&,
                           const mlmc_run_opts&, DriverState*, DriverState*)
{
    return fail(ctx, MLMC_EINVAL, "persistent form not available yet");
}

}  // namespace mlmc
