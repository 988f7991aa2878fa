// Device-resident state of the adaptive MLMC driver.
//
// The sampler adds each level's batch sums into that level's spread group
// (one per level, outside this struct); one small fp64 kernel
// (driver_update) folds the groups into batch[l], absorbs them, re-estimates
// E_l and V_l, sets the optimal N_l and the next outstanding batch dN_l, runs
// the bias test and adds a level when needed.  The host only reads this
// struct back to learn what to launch next (or, in the persistent form, only
// the done flag).
#pragma once
#include <stdint.h>

#include "reduce.hpp"

namespace mlmc {

constexpr int kMaxLevels = 16;

struct DriverState {
    // configuration
    double eps, alpha, beta;
    double Ma, Mb;                 // M^alpha, M^beta (computed once by the host)
    int M, L_min, L_max, max_iterations;
    int antithetic, pad_cfg;       // the twin doubles the fine steps of l >= 1
    // progress
    int L, done, converged, iterations;
    double n[kMaxLevels];          // samples absorbed so far
    double dN[kMaxLevels];         // outstanding batch (sampled next)
    double sum1[kMaxLevels], sum2[kMaxLevels];
    double E[kMaxLevels], V[kMaxLevels], C[kMaxLevels], Nopt[kMaxLevels];
    double estimate, var_est, bias_est;
    double alpha_fit, beta_fit, gamma_fit;
    unsigned long long n_nonfinite;
    // persistent form: work table bookkeeping (persistent.hip)
    unsigned int work_head, work_count;
    unsigned int pad0, pad1;
    // number of updates; the host mirror holds 2 seq + done, written last
    unsigned long long seq;
    LevelAcc batch[kMaxLevels];
};

// Configuration of a fresh state (n_pilot outstanding samples on levels
// 0..L_min); passed by value to the kernel that builds the state.
struct DriverInit {
    double eps, alpha, beta, Ma, Mb, n_pilot;
    int M, antithetic, L_min, L_max, max_iterations, pad;
};

// One update launch (driver.hip): with `init`, the run's first update, which
// builds the state itself; start/stop stamp the kernel when both are given.
hipError_t launch_driver_update(DriverState* st, DriverState* mirror, LevelAcc* spread,
                                hipStream_t stream, hipEvent_t start = nullptr,
                                hipEvent_t stop = nullptr, const DriverInit* init = nullptr);
// Wait until the host mirror shows update number `want` (driver.hip).
hipError_t wait_update(hipStream_t stream, const DriverState* h, unsigned long long want);

// Host side: the update count and the done flag as the mirror's last
// written word publishes them (the mirror words of that update are complete).
inline unsigned long long mirror_updates(const DriverState* h)
{
    return *(const volatile unsigned long long*)&h->seq >> 1;
}
inline bool mirror_done(const DriverState* h)
{
    return (*(const volatile unsigned long long*)&h->seq & 1ull) != 0;
}

}  // namespace mlmc
