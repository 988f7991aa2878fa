// Level-sampler kernel arguments and host-side launchers shared by the
// per-level entry points, the driver and the persistent kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mlmc.h"
#include "reduce.hpp"
#include "sampler.hpp"

namespace mlmc {

template <typename Real>
struct LevelArgs {
    StepParams<Real> P;
    uint64_t seed;
    uint64_t offset;      // index of the first sample
    uint64_t N;           // number of samples
    int l;                // level
    int nf;               // fine steps M^l
    uint32_t ngroups;     // ceil(nf / 4): groups of four fine steps
    uint32_t stream;      // Philox stream of the Brownian normals
    LevelAcc* acc;        // (payoff, level) record or spread group receiving the sums
    uint32_t spread_mask = 0;   // block b adds into acc[b & mask]: 0, or kSpread - 1
    double* pf_out;       // optional per-path dump (fp64), else null
    double* pc_out;
    int coupled;          // 0: standard MC (fine path only at level l)
    const float* phi0;    // level 0 with the control variate: phi(0, S0), else null
    uint32_t c2 = 0;      // Philox counter word 2 of every Brownian block of the launch
    uint32_t c2b = 0;     // and of every bridge block (set_counter_words)
    uint32_t split = 1;   // lanes per path (split_lanes); 1: one path per lane
};

// Philox counter word 2 of generator unit u (a block index on one- and
// two-step levels, a sample index otherwise) at level l: l + 256 (u >> 32),
// the same word make_path_key forms.
__host__ __device__ inline uint32_t counter_word2(int l, uint64_t u)
{
    return (uint32_t)l + 256u * (uint32_t)(u >> 32);
}

// Samples per Brownian generator unit: one- and two-step levels share Philox
// blocks (4 / (n_f d) samples each), longer paths own theirs.
__host__ __device__ inline uint64_t samples_per_unit(int nf, int d)
{
    return nf < 4 ? (uint64_t)(4 / (nf * d)) : 1u;
}

// End of the leading part of the sample range [first, end) whose generator
// units (q samples each) share one high word.  A launch covers one such part,
// so counter word 2 is a launch constant; ranges that cross a multiple of
// q 2^32 are split into several launches.
__host__ __device__ inline uint64_t counter_segment_end(uint64_t first, uint64_t end, uint64_t q)
{
    const uint64_t next_unit = ((first / q >> 32) + 1) << 32;
    const uint64_t lim = next_unit * q;
    return lim < end ? lim : end;
}

// Counter words of a launch whose range [offset, offset + N) is one segment;
// d = Brownian dimension.  Bridge blocks of one- and two-step levels are
// numbered by generator block / d, of longer paths by sample.
template <typename Real>
__host__ __device__ inline void set_counter_words(LevelArgs<Real>& a, int d)
{
    const uint64_t u = a.offset / samples_per_unit(a.nf, d);
    a.c2 = counter_word2(a.l, u);
    a.c2b = counter_word2(a.l, a.nf < 4 ? u / (uint64_t)d : u);
}

// Lanes per path for a GBM level whose N paths cannot fill the device: a
// power of two G <= 64 with G <= (num_cu 1024) / N (about four paths' worth
// of lanes per SIMD in all) and n_f / G a multiple of 4, so that every lane
// holds whole generator blocks (and whole coarse steps); 1 when that leaves
// fewer than 4 lanes per path or when the variant is not linear in the path's
// start value (Heston, the conditional digital, the antithetic twin).
__host__ __device__ inline uint32_t split_lanes(int nf, uint64_t N, int num_cu, bool eligible)
{
    if (!eligible || N == 0 || nf < 16) return 1;
    const uint64_t want = (uint64_t)num_cu * 1024 / N;
    uint32_t G = 64;
    while (G > 1 && ((uint64_t)G > want || (uint32_t)(nf / 4) % G != 0)) G >>= 1;
    return G >= 4 ? G : 1;
}

// Host-side conversion of model/payoff to the kernel's parameter block.
template <typename Real>
StepParams<Real> make_step_params(const mlmc_model& m, const mlmc_payoff& p, int l, int M);

// Kernel variant of a model: kGBM, kGBMMil (GBM with the Milstein scheme)
// or kHeston.
int sampler_variant(const mlmc_model& m);

// Launch shape actually used.  `grid` is an upper bound: the launcher lowers
// it to the number of blocks the device holds at once for the chosen kernel
// (num_cu compute units, 0 = no cap), so that no block waits for another to
// finish and the grid-stride loop gives every resident block the same share.
struct LaunchShape {
    int block, ppt, grid;
    int num_cu = 0;
    int split = 1;        // lanes per path (split_lanes)
};

// Enqueue one level's sampler on `stream` (accumulating into args.acc).
// Returns hipSuccess or the launch error.  Shape chosen by the caller.  With
// start/stop events the runtime stamps them when the kernel itself starts and
// ends (hipExtLaunchKernelGGL), so they time the kernel, not the queue: they
// agree with the profiler's kernel durations, where events recorded around
// the launch read ~7% more.  A stamped launch costs ~15 us of queue time
// when only some launches carry stamps.
hipError_t launch_level(const mlmc_model& m, const mlmc_payoff& p, int M, int precision,
                        const void* args, LaunchShape shape, hipStream_t stream,
                        hipEvent_t start = nullptr, hipEvent_t stop = nullptr);

}  // namespace mlmc
