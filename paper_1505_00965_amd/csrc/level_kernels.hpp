// Coupled level-sampler kernels and their per-variant dispatch tables.
//
// One lane owns PPT samples of level l at a time (indices i0 + p * blockDim,
// so dumps are coalesced), advances each coupled fine/coarse pair (and with
// ANTI its antithetic twin) through n_f = M^l fine steps in registers, forms
// Y = P_l - P_{l-1} (eq. (eq:Yldef)) and adds Y, Y^2, P_l, P_l^2, P_{l-1},
// P_{l-1}^2 into fp64 lane sums; blocks walk the sample range with a grid
// stride, then reduce once (reduce.hpp).  The loop trip count is the same for
// every lane of a launch, so waves never diverge in the path loop.
//
// Each sampler variant (MODEL) instantiates its table in a translation unit
// of its own (level_gbm.hip, level_gbm_mil.hip, level_heston.hip), so the
// kernels compile in parallel.
#pragma once
#include "level.hpp"
#include "sampler_impl.hpp"

namespace mlmc {

template <int MODEL, int PAYOFF, typename Real, int M, int PPT, bool ANTI>
__global__ __launch_bounds__(1024) void level_kernel(LevelArgs<Real> a)
{
    double sums[kNumSums] = {0, 0, 0, 0, 0, 0};
    unsigned nonfinite = 0;
    const uint64_t chunk = (uint64_t)blockDim.x * PPT;
    const uint64_t nchunks = (a.N + chunk - 1) / chunk;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x)
        process_chunk<MODEL, PAYOFF, Real, M, PPT, ANTI>(a, c * chunk, sums, nonfinite);
    block_reduce_add(sums, nonfinite, a.acc + (blockIdx.x & a.spread_mask));
}

// Levels with one or two fine steps: samples share generator blocks.
template <int MODEL, int PAYOFF, typename Real, int NF, int M, int PPT, bool ANTI>
__global__ __launch_bounds__(1024) void short_level_kernel(LevelArgs<Real> a)
{
    constexpr int Q = 4 / (NF * (one_factor(MODEL) ? 1 : 2));
    double sums[kNumSums] = {0, 0, 0, 0, 0, 0};
    unsigned nonfinite = 0;
    const uint64_t nblk = short_blocks(a.offset, a.N, Q);
    const uint64_t chunk = (uint64_t)blockDim.x * PPT;
    const uint64_t nchunks = (nblk + chunk - 1) / chunk;
    const FullChunks f = full_chunks(a.offset, a.N, Q, chunk);
    // block-uniform bounds (computed with a vector division): scalar registers.
    // A launch's generator blocks share one counter high word, so chunk
    // indices fit 32 bits and the loop test is a scalar compare.
    const uint32_t lo = __builtin_amdgcn_readfirstlane(f.lo), hi = __builtin_amdgcn_readfirstlane(f.hi);
    const uint32_t n32 = __builtin_amdgcn_readfirstlane((uint32_t)nchunks);
    for (uint32_t c = blockIdx.x; c < n32; c += gridDim.x) {
        const bool full = c >= lo && c < hi;
        process_short<MODEL, PAYOFF, Real, NF, M, PPT, ANTI>(a, (uint64_t)c * chunk, full, sums,
                                                             nonfinite);
    }
    if (NF == 1) copy_y_sums(sums);
    block_reduce_add(sums, nonfinite, a.acc + (blockIdx.x & a.spread_mask));
}

// GBM levels whose paths are too few to fill the device: a.split lanes per
// path (process_split); blocks walk the paths a.split at a time per lane group.
template <int MODEL, int PAYOFF, int M>
__global__ __launch_bounds__(1024) void split_level_kernel(LevelArgs<float> a)
{
    double sums[kNumSums] = {0, 0, 0, 0, 0, 0};
    unsigned nonfinite = 0;
    const uint64_t per_block = blockDim.x / a.split;
    const uint64_t nchunks = (a.N + per_block - 1) / per_block;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x)
        process_split<MODEL, PAYOFF, M>(a, c * per_block, sums, nonfinite);
    block_reduce_add(sums, nonfinite, a.acc + (blockIdx.x & a.spread_mask));
}

template <typename Real>
using KernelFn = void (*)(LevelArgs<Real>);

// nf: 1 or 2 selects the short-level kernel, anything else the general one.
// The antithetic twin exists on coupled levels (n_f >= 2); fp64 paths run
// one sample per lane (register budget); the twin runs at most two.
template <int MODEL, int PAYOFF, typename Real, int M>
KernelFn<Real> pick_ppt(int ppt, int nf, bool anti, bool split)
{
    if constexpr (sizeof(Real) == 4 && MODEL != kHeston && PAYOFF != kDigitalCond) {
        if (split) return split_level_kernel<MODEL, PAYOFF, M>;
    }
    (void)split;
    if constexpr (sizeof(Real) == 8) {
        (void)ppt;
        if (nf == 1) return short_level_kernel<MODEL, PAYOFF, Real, 1, M, 1, false>;
        if constexpr (M == 2) {
            if (nf == 2) return anti ? short_level_kernel<MODEL, PAYOFF, Real, 2, M, 1, true>
                                     : short_level_kernel<MODEL, PAYOFF, Real, 2, M, 1, false>;
        }
        return anti ? level_kernel<MODEL, PAYOFF, Real, M, 1, true>
                    : level_kernel<MODEL, PAYOFF, Real, M, 1, false>;
    } else {
        if (nf == 1) return ppt == 1 ? short_level_kernel<MODEL, PAYOFF, Real, 1, M, 1, false>
                                     : short_level_kernel<MODEL, PAYOFF, Real, 1, M, 2, false>;
        if constexpr (M == 2) {
            if (nf == 2) {
                if (anti) return ppt == 1 ? short_level_kernel<MODEL, PAYOFF, Real, 2, M, 1, true>
                                          : short_level_kernel<MODEL, PAYOFF, Real, 2, M, 2, true>;
                return ppt == 1 ? short_level_kernel<MODEL, PAYOFF, Real, 2, M, 1, false>
                                : short_level_kernel<MODEL, PAYOFF, Real, 2, M, 2, false>;
            }
        }
        if (anti) return ppt == 1 ? level_kernel<MODEL, PAYOFF, Real, M, 1, true>
                                  : level_kernel<MODEL, PAYOFF, Real, M, 2, true>;
        switch (ppt) {
        case 1: return level_kernel<MODEL, PAYOFF, Real, M, 1, false>;
        case 2: return level_kernel<MODEL, PAYOFF, Real, M, 2, false>;
        default: return level_kernel<MODEL, PAYOFF, Real, M, 4, false>;
        }
    }
}

template <int MODEL, int PAYOFF, typename Real>
KernelFn<Real> pick_m(int M, int ppt, int nf, bool anti, bool split)
{
    return M == 2 ? pick_ppt<MODEL, PAYOFF, Real, 2>(ppt, nf, anti, split)
                  : pick_ppt<MODEL, PAYOFF, Real, 4>(ppt, nf, anti, split);
}

// The kernel of one sampler variant for (payoff, M, samples per lane, n_f,
// antithetic, split paths).  Defined here, instantiated once per variant.
template <int MODEL, typename Real>
KernelFn<Real> pick_variant(int payoff, int M, int ppt, int nf, bool anti, bool split)
{
    switch (payoff) {
    case kCall: return pick_m<MODEL, kCall, Real>(M, ppt, nf, anti, split);
    case kAsian: return pick_m<MODEL, kAsian, Real>(M, ppt, nf, anti, split);
    case kLookback: return pick_m<MODEL, kLookback, Real>(M, ppt, nf, anti, split);
    case kDigitalCond: return pick_m<MODEL, kDigitalCond, Real>(M, ppt, nf, anti, split);
    default: return pick_m<MODEL, kDigital, Real>(M, ppt, nf, anti, split);
    }
}

}  // namespace mlmc
