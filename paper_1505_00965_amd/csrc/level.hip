// Level-sampler launcher: parameter block, dispatch to the per-variant
// kernel tables, and the generator probes.
#include <cmath>
#include <map>
#include <mutex>
#include <utility>

#include <hip/hip_ext.h>

#include "level_kernels.hpp"

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
    P.c2 = (Real)(0.5 * m.sigma * m.sigma);
    P.rh_m = (Real)((m.r - 0.5 * m.sigma * m.sigma) * h);
    P.rH_m = (Real)((m.r - 0.5 * m.sigma * m.sigma) * H);
    P.K = (Real)p.K;
    P.payout = (Real)p.payout;
    P.disc = (Real)std::exp(-m.r * m.T);
    P.inv_T = (Real)(1.0 / m.T);
    P.lnu_scale = (Real)(-2.0 * h * std::log(2.0));
    P.asian_scale = (Real)(h / (2.0 * m.T));
    P.l0_base = (Real)(m.S0 * (1.0 + m.r * h) - p.K);
    P.l0_slope = (Real)(m.S0 * m.sigma);
    return P;
}
template StepParams<float> make_step_params<float>(const mlmc_model&, const mlmc_payoff&, int, int);
template StepParams<double> make_step_params<double>(const mlmc_model&, const mlmc_payoff&, int, int);

// ------------------------------------------------------------ dispatch
// Instantiated in the per-variant translation units.
extern template KernelFn<float> pick_variant<kGBM, float>(int, int, int, int, bool, bool);
extern template KernelFn<double> pick_variant<kGBM, double>(int, int, int, int, bool, bool);
extern template KernelFn<float> pick_variant<kGBMMil, float>(int, int, int, int, bool, bool);
extern template KernelFn<double> pick_variant<kGBMMil, double>(int, int, int, int, bool, bool);
extern template KernelFn<float> pick_variant<kHeston, float>(int, int, int, int, bool, bool);
extern template KernelFn<double> pick_variant<kHeston, double>(int, int, int, int, bool, bool);

int sampler_variant(const mlmc_model& m)
{
    if (m.kind == MLMC_HESTON) return kHeston;
    return m.scheme == MLMC_MILSTEIN ? kGBMMil : kGBM;
}

template <typename Real>
static KernelFn<Real> pick(const mlmc_model& m, int payoff, int M, int ppt, int nf, bool split)
{
    const bool anti = m.antithetic != 0 && nf > 1;
    switch (sampler_variant(m)) {
    case kGBMMil: return pick_variant<kGBMMil, Real>(payoff, M, ppt, nf, anti, split);
    case kHeston: return pick_variant<kHeston, Real>(payoff, M, ppt, nf, anti, split);
    default: return pick_variant<kGBM, Real>(payoff, M, ppt, nf, anti, split);
    }
}

// Blocks of `fn` with `block` threads that one compute unit holds at once
// (its register count decides), cached per kernel and block size; 0 if the
// runtime cannot say.
static int resident_blocks(const void* fn, int block)
{
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(fn, block);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, block, 0) != hipSuccess) {
        (void)hipGetLastError();
        n = 0;
    }
    cache[key] = n;
    return n;
}

static dim3 resident_grid(const void* fn, const LaunchShape& shape)
{
    int g = shape.grid;
    if (shape.num_cu > 0) {
        const int per_cu = resident_blocks(fn, shape.block);
        if (per_cu > 0 && g > shape.num_cu * per_cu) g = shape.num_cu * per_cu;
    }
    return dim3(g);
}

hipError_t launch_level(const mlmc_model& m, const mlmc_payoff& p, int M, int precision,
                        const void* args, LaunchShape shape, hipStream_t stream, hipEvent_t start,
                        hipEvent_t stop)
{
    dim3 block(shape.block);
    if (precision == 64) {
        const auto& a = *(const LevelArgs<double>*)args;
        auto fn = pick<double>(m, p.kind, M, 1, a.nf, false);
        hipExtLaunchKernelGGL(fn, resident_grid((const void*)fn, shape), block, 0, stream, start,
                              stop, 0, a);
    } else {
        const auto& a = *(const LevelArgs<float>*)args;
        auto fn = pick<float>(m, p.kind, M, shape.ppt, a.nf, a.split > 1);
        hipExtLaunchKernelGGL(fn, resident_grid((const void*)fn, shape), block, 0, stream, start,
                              stop, 0, a);
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
