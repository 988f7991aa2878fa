// Coupled level-sampler kernels (one (model, payoff, precision, M, PPT)
// instantiation each) and their launcher.
//
// One lane owns PPT samples of level l at a time (indices i0 + p * blockDim,
// so dumps are coalesced), advances each coupled fine/coarse pair through
// n_f = M^l fine steps in registers, forms Y = P_l - P_{l-1}
// (eq. (eq:Yldef)) and adds Y, Y^2, P_l, P_l^2, P_{l-1}, P_{l-1}^2 into fp64
// lane sums; blocks walk the sample range with a grid stride, then reduce
// once (reduce.hpp).  The loop trip count is the same for every lane of a
// launch, so waves never diverge in the path loop.
#include <cmath>

#include <hip/hip_ext.h>

#include "level.hpp"
#include "sampler_impl.hpp"

namespace mlmc {

template <typename Real>
StepParams<Real> make_step_params(const mlmc_model& m, const mlmc_payoff& p, int l, int M)
{
    StepParams<Real> P;
    double nf = 1.0;
    for (int i = 0; i < l; ++i) nf *= M;
    const double h = m.T / nf, H = M * h;
    P.S0 = (Real)m.S0;
    P.r = (Real)m.r;
    P.sigma = (Real)m.sigma;
    P.kappa = (Real)m.kappa;
    P.theta = (Real)m.theta;
    P.xi = (Real)m.xi;
    P.rho = (Real)m.rho;
    P.rho_c = (Real)std::sqrt(1.0 - m.rho * m.rho);
    P.v0 = (Real)m.v0;
    P.h = (Real)h;
    P.sqh = (Real)std::sqrt(h);
    P.H = (Real)H;
    P.rh = (Real)(m.r * h);
    P.rH = (Real)(m.r * H);
    P.K = (Real)p.K;
    P.payout = (Real)p.payout;
    P.disc = (Real)std::exp(-m.r * m.T);
    P.inv_T = (Real)(1.0 / m.T);
    P.lnu_scale = (Real)(-2.0 * h * std::log(2.0));
    P.asian_scale = (Real)(h / (2.0 * m.T));
    return P;
}
template StepParams<float> make_step_params<float>(const mlmc_model&, const mlmc_payoff&, int, int);
template StepParams<double> make_step_params<double>(const mlmc_model&, const mlmc_payoff&, int, int);

template <int MODEL, int PAYOFF, typename Real, int M, int PPT>
__global__ __launch_bounds__(1024) void level_kernel(LevelArgs<Real> a)
{
    double sums[kNumSums] = {0, 0, 0, 0, 0, 0};
    unsigned nonfinite = 0;
    const uint64_t chunk = (uint64_t)blockDim.x * PPT;
    const uint64_t nchunks = (a.N + chunk - 1) / chunk;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x)
        process_chunk<MODEL, PAYOFF, Real, M, PPT>(a, c * chunk, sums, nonfinite);
    block_reduce_add(sums, nonfinite, a.acc);
}

// Levels with one or two fine steps: samples share generator blocks.
template <int MODEL, int PAYOFF, typename Real, int NF, int M, int PPT>
__global__ __launch_bounds__(1024) void short_level_kernel(LevelArgs<Real> a)
{
    constexpr int Q = 4 / (NF * (MODEL == kGBM ? 1 : 2));
    double sums[kNumSums] = {0, 0, 0, 0, 0, 0};
    unsigned nonfinite = 0;
    const uint64_t nblk = short_blocks(a.offset, a.N, Q);
    const uint64_t chunk = (uint64_t)blockDim.x * PPT;
    const uint64_t nchunks = (nblk + chunk - 1) / chunk;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x)
        process_short<MODEL, PAYOFF, Real, NF, M, PPT>(a, c * chunk, sums, nonfinite);
    block_reduce_add(sums, nonfinite, a.acc);
}

// ------------------------------------------------------------ dispatch
template <typename Real>
using KernelFn = void (*)(LevelArgs<Real>);

// nf: 1 or 2 selects the short-level kernel, anything else the general one.
template <int MODEL, int PAYOFF, typename Real, int M>
static KernelFn<Real> pick_ppt(int ppt, int nf)
{
    if constexpr (sizeof(Real) == 8) {
        (void)ppt;   // fp64 paths: one per lane (register budget)
        if (nf == 1) return short_level_kernel<MODEL, PAYOFF, Real, 1, M, 1>;
        if (nf == 2) return short_level_kernel<MODEL, PAYOFF, Real, 2, M, 1>;
        return level_kernel<MODEL, PAYOFF, Real, M, 1>;
    } else {
        if (nf == 1) return ppt == 1 ? short_level_kernel<MODEL, PAYOFF, Real, 1, M, 1>
                                     : short_level_kernel<MODEL, PAYOFF, Real, 1, M, 2>;
        if (nf == 2) return ppt == 1 ? short_level_kernel<MODEL, PAYOFF, Real, 2, M, 1>
                                     : short_level_kernel<MODEL, PAYOFF, Real, 2, M, 2>;
        switch (ppt) {
        case 1: return level_kernel<MODEL, PAYOFF, Real, M, 1>;
        case 2: return level_kernel<MODEL, PAYOFF, Real, M, 2>;
        default: return level_kernel<MODEL, PAYOFF, Real, M, 4>;
        }
    }
}

template <int MODEL, int PAYOFF, typename Real>
static KernelFn<Real> pick_m(int M, int ppt, int nf)
{
    return M == 2 ? pick_ppt<MODEL, PAYOFF, Real, 2>(ppt, nf)
                  : pick_ppt<MODEL, PAYOFF, Real, 4>(ppt, nf);
}

template <int MODEL, typename Real>
static KernelFn<Real> pick_payoff(int payoff, int M, int ppt, int nf)
{
    switch (payoff) {
    case kCall: return pick_m<MODEL, kCall, Real>(M, ppt, nf);
    case kAsian: return pick_m<MODEL, kAsian, Real>(M, ppt, nf);
    case kLookback: return pick_m<MODEL, kLookback, Real>(M, ppt, nf);
    default: return pick_m<MODEL, kDigital, Real>(M, ppt, nf);
    }
}

template <typename Real>
static KernelFn<Real> pick(int model, int payoff, int M, int ppt, int nf)
{
    return model == kGBM ? pick_payoff<kGBM, Real>(payoff, M, ppt, nf)
                         : pick_payoff<kHeston, Real>(payoff, M, ppt, nf);
}

hipError_t launch_level(const mlmc_model& m, const mlmc_payoff& p, int M, int precision,
                        const void* args, LaunchShape shape, hipStream_t stream, hipEvent_t start,
                        hipEvent_t stop)
{
    dim3 grid(shape.grid), block(shape.block);
    if (precision == 64) {
        const auto& a = *(const LevelArgs<double>*)args;
        auto fn = pick<double>(m.kind, p.kind, M, 1, a.nf);
        hipExtLaunchKernelGGL(fn, grid, block, 0, stream, start, stop, 0, a);
    } else {
        const auto& a = *(const LevelArgs<float>*)args;
        auto fn = pick<float>(m.kind, p.kind, M, shape.ppt, a.nf);
        hipExtLaunchKernelGGL(fn, grid, block, 0, stream, start, stop, 0, a);
    }
    return hipGetLastError();
}

// ------------------------------------------------------- generator probes
__global__ void philox_words_kernel(uint64_t seed, int level, uint64_t s0, uint32_t stream,
                                    uint32_t nblocks, uint64_t npaths, uint32_t* out)
{
    const uint64_t total = npaths * nblocks;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < total;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = t / nblocks;
        const uint32_t j = (uint32_t)(t % nblocks);
        const PathKey k = make_path_key(seed, level, s0 + i, stream);
        const u32x4 w = path_block(k, j);
        uint32_t* o = out + 4 * t;
        o[0] = w.x; o[1] = w.y; o[2] = w.z; o[3] = w.w;
    }
}

// Normals of each path as the sampler reads them (paths needing fewer than
// four share a block: q = 4/total_per_path of them, block s/q).
template <typename Real>
__global__ void normals_kernel(uint64_t seed, int level, uint64_t s0, uint32_t stream,
                               uint32_t nblocks, int total_per_path, uint64_t npaths, double* out)
{
    const uint64_t total = npaths * nblocks;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < total;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = t / nblocks;
        const uint32_t j = (uint32_t)(t % nblocks);
        const uint64_t s = s0 + i;
        const int q = total_per_path < 4 ? 4 / total_per_path : 1;
        const PathKey k = make_path_key(seed, level, s / q, stream);
        const u32x4 w = path_block(k, j);
        Real z[4];
        box_muller(w.x, w.y, z[0], z[1]);
        box_muller(w.z, w.w, z[2], z[3]);
        const int first = q > 1 ? (int)(s % q) * total_per_path : 4 * (int)j;
        for (int n = 0; n < total_per_path && q > 1; ++n)
            out[i * total_per_path + n] = (double)z[first + n];
        for (int w4 = 0; w4 < 4 && q == 1; ++w4) {
            const int n = first + w4;
            if (n < total_per_path) out[i * total_per_path + n] = (double)z[w4];
        }
    }
}

hipError_t launch_philox_words(uint64_t seed, int level, uint64_t s0, uint32_t stream,
                               uint32_t nblocks, uint64_t npaths, uint32_t* out, hipStream_t st)
{
    const uint64_t total = npaths * nblocks;
    const unsigned grid = (unsigned)std::min<uint64_t>((total + 255) / 256, 65536);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(philox_words_kernel, dim3(grid), dim3(256), 0, st, seed, level, s0, stream,
                       nblocks, npaths, out);
    return hipGetLastError();
}

hipError_t launch_normals(uint64_t seed, int level, uint64_t s0, uint32_t stream, int dim,
                          int nsteps, uint64_t npaths, int precision, double* out, hipStream_t st)
{
    const int per_path = nsteps * dim;
    const uint32_t nblocks = (uint32_t)((per_path + 3) / 4);
    const uint64_t total = npaths * nblocks;
    const unsigned grid = (unsigned)std::min<uint64_t>((total + 255) / 256, 65536);
    if (grid == 0) return hipSuccess;
    if (precision == 64)
        hipLaunchKernelGGL(normals_kernel<double>, dim3(grid), dim3(256), 0, st, seed, level, s0,
                           stream, nblocks, per_path, npaths, out);
    else
        hipLaunchKernelGGL(normals_kernel<float>, dim3(grid), dim3(256), 0, st, seed, level, s0,
                           stream, nblocks, per_path, npaths, out);
    return hipGetLastError();
}

}  // namespace mlmc
