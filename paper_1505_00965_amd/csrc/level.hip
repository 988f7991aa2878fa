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

#include "level.hpp"

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

// Advance PPT coupled pairs through all fine steps of the level.
template <int MODEL, int PAYOFF, typename Real, int M, int PPT>
__device__ __forceinline__ void simulate(const LevelArgs<Real>& a, const uint64_t (&s)[PPT],
                                         PathPair<Real> (&q)[PPT])
{
    const StepParams<Real>& P = a.P;
    PathKey key[PPT], bkey[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        key[p] = make_path_key(a.seed, a.l, s[p], a.stream);
        bkey[p] = make_path_key(a.seed, a.l, s[p], a.stream + 1u);
        init_pair<Real, MODEL, PAYOFF>(q[p], P);
    }
    const bool coupled = a.coupled && a.l > 0;
    const bool full = a.nf >= 4;
    for (uint32_t g = 0; g < a.ngroups; ++g) {
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            Real dw1[4], dwp[4], e[4];
            if (MODEL == kGBM) {
                const u32x4 w = path_block(key[p], g);
                Real z0, z1, z2, z3;
                box_muller(w.x, w.y, z0, z1);
                box_muller(w.z, w.w, z2, z3);
                dw1[0] = P.sqh * z0; dw1[1] = P.sqh * z1;
                dw1[2] = P.sqh * z2; dw1[3] = P.sqh * z3;
                dwp[0] = dwp[1] = dwp[2] = dwp[3] = Real(0);
            } else {
                const u32x4 wa = path_block(key[p], 2 * g);
                const u32x4 wb = path_block(key[p], 2 * g + 1);
                Real z0, z1, z2, z3, z4, z5, z6, z7;
                box_muller(wa.x, wa.y, z0, z1);
                box_muller(wa.z, wa.w, z2, z3);
                box_muller(wb.x, wb.y, z4, z5);
                box_muller(wb.z, wb.w, z6, z7);
                dw1[0] = P.sqh * z0; dwp[0] = P.sqh * z1;
                dw1[1] = P.sqh * z2; dwp[1] = P.sqh * z3;
                dw1[2] = P.sqh * z4; dwp[2] = P.sqh * z5;
                dw1[3] = P.sqh * z6; dwp[3] = P.sqh * z7;
            }
            if (PAYOFF == kLookback) {
                const u32x4 u = path_block(bkey[p], g);
                e[0] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.x));
                e[1] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.y));
                e[2] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.z));
                e[3] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.w));
            } else {
                e[0] = e[1] = e[2] = e[3] = Real(0);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (full || (int)(4 * g + k) < a.nf) {
                    fine_step<Real, MODEL, PAYOFF>(q[p], P, dw1[k], dwp[k], e[k], k % M, coupled);
                    if (coupled && ((k + 1) % M) == 0) coarse_step<Real, MODEL, PAYOFF>(q[p], P);
                }
            }
        }
    }
}

template <int MODEL, int PAYOFF, typename Real, int M, int PPT>
__global__ __launch_bounds__(1024) void level_kernel(LevelArgs<Real> a)
{
    double sums[kNumSums] = {0, 0, 0, 0, 0, 0};
    unsigned nonfinite = 0;
    const uint64_t chunk = (uint64_t)blockDim.x * PPT;
    const uint64_t nchunks = (a.N + chunk - 1) / chunk;
    const bool coupled = a.coupled && a.l > 0;
    const Real dtf = a.P.h, dtc = a.P.H;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        uint64_t idx[PPT], s[PPT];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            idx[p] = c * chunk + (uint64_t)p * blockDim.x + threadIdx.x;
            s[p] = a.offset + idx[p];
        }
        PathPair<Real> q[PPT];
        simulate<MODEL, PAYOFF, Real, M, PPT>(a, s, q);
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const Real pf = payoff_value<Real, PAYOFF>(a.P, q[p].S, q[p].asum, q[p].acomp, q[p].mn, dtf);
            const Real pc = coupled ? payoff_value<Real, PAYOFF>(a.P, q[p].Sc, q[p].csum, q[p].ccomp,
                                                                q[p].mnc, dtc)
                                    : Real(0);
            if (idx[p] >= a.N) continue;
            const double df = (double)pf, dc = (double)pc;
            if (a.pf_out) {
                a.pf_out[idx[p]] = df;
                a.pc_out[idx[p]] = dc;
            }
            const double y = df - dc;
            if (!isfinite(y)) {
                ++nonfinite;
                continue;
            }
            sums[0] += y;
            sums[1] = __builtin_fma(y, y, sums[1]);
            sums[2] += df;
            sums[3] = __builtin_fma(df, df, sums[3]);
            sums[4] += dc;
            sums[5] = __builtin_fma(dc, dc, sums[5]);
        }
    }
    block_reduce_add(sums, nonfinite, a.acc);
}

// ------------------------------------------------------------ dispatch
template <typename Real>
using KernelFn = void (*)(LevelArgs<Real>);

template <int MODEL, int PAYOFF, typename Real, int M>
static KernelFn<Real> pick_ppt(int ppt)
{
    if constexpr (sizeof(Real) == 8) {
        (void)ppt;   // fp64 paths: one per lane (register budget)
        return level_kernel<MODEL, PAYOFF, Real, M, 1>;
    } else {
        switch (ppt) {
        case 1: return level_kernel<MODEL, PAYOFF, Real, M, 1>;
        case 2: return level_kernel<MODEL, PAYOFF, Real, M, 2>;
        default: return level_kernel<MODEL, PAYOFF, Real, M, 4>;
        }
    }
}

template <int MODEL, int PAYOFF, typename Real>
static KernelFn<Real> pick_m(int M, int ppt)
{
    return M == 2 ? pick_ppt<MODEL, PAYOFF, Real, 2>(ppt) : pick_ppt<MODEL, PAYOFF, Real, 4>(ppt);
}

template <int MODEL, typename Real>
static KernelFn<Real> pick_payoff(int payoff, int M, int ppt)
{
    switch (payoff) {
    case kCall: return pick_m<MODEL, kCall, Real>(M, ppt);
    case kAsian: return pick_m<MODEL, kAsian, Real>(M, ppt);
    case kLookback: return pick_m<MODEL, kLookback, Real>(M, ppt);
    default: return pick_m<MODEL, kDigital, Real>(M, ppt);
    }
}

template <typename Real>
static KernelFn<Real> pick(int model, int payoff, int M, int ppt)
{
    return model == kGBM ? pick_payoff<kGBM, Real>(payoff, M, ppt)
                         : pick_payoff<kHeston, Real>(payoff, M, ppt);
}

hipError_t launch_level(const mlmc_model& m, const mlmc_payoff& p, int M, int precision,
                        const void* args, LaunchShape shape, hipStream_t stream)
{
    dim3 grid(shape.grid), block(shape.block);
    if (precision == 64) {
        auto fn = pick<double>(m.kind, p.kind, M, 1);
        hipLaunchKernelGGL(fn, grid, block, 0, stream, *(const LevelArgs<double>*)args);
    } else {
        auto fn = pick<float>(m.kind, p.kind, M, shape.ppt);
        hipLaunchKernelGGL(fn, grid, block, 0, stream, *(const LevelArgs<float>*)args);
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

template <typename Real>
__global__ void normals_kernel(uint64_t seed, int level, uint64_t s0, uint32_t stream,
                               uint32_t nblocks, int total_per_path, uint64_t npaths, double* out)
{
    const uint64_t total = npaths * nblocks;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < total;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = t / nblocks;
        const uint32_t j = (uint32_t)(t % nblocks);
        const PathKey k = make_path_key(seed, level, s0 + i, stream);
        const u32x4 w = path_block(k, j);
        Real z[4];
        box_muller(w.x, w.y, z[0], z[1]);
        box_muller(w.z, w.w, z[2], z[3]);
        for (int q = 0; q < 4; ++q) {
            const int n = 4 * (int)j + q;
            if (n < total_per_path) out[i * total_per_path + n] = (double)z[q];
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
