// Randomised single-term multilevel estimator (Sec. 7 cites Rhee and
// Glynn's extra randomisation, which removes the bias of a fixed finest
// level).  Every one of the N samples draws its level L from the geometric
// law p_l ~ q^l cut at the finest grid Lc and contributes Z = Y_L / p_L, so
// E[Z] = sum_l E[Y_l] = E[P_Lc] (eq. (eq:mlmc:ident)).
//
// GPU form: one kernel draws the N levels (word i mod 4 of the Philox block
// at counter (0, i / 4, 0, stream 7), inverted against the cumulative law)
// into a per-level histogram; then every level with a non-zero count runs
// the ordinary level sampler on its samples 0 .. n_l - 1, all launches back
// to back into one record per level, and the host forms
//   estimate = (1/N) sum_l S1_l / p_l,  E[Z^2] = (1/N) sum_l S2_l / p_l^2.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "context.hpp"
#include "philox.hpp"

namespace mlmc {

constexpr int kRgLevels = 16;

struct RgLaw {
    double F[kRgLevels];   // cumulative probabilities, F[Lc] = 1
    int Lc;
};

// Draws are integer work decided by one fp64 comparison per bin, made on
// the same exactly representable uniform as the oracle's.
__global__ __launch_bounds__(256) void level_draw_kernel(uint64_t seed, uint64_t N, RgLaw law,
                                                         unsigned long long* counts)
{
    __shared__ unsigned int hist[kRgLevels];
    if (threadIdx.x < kRgLevels) hist[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t nblk = (N + 3) / 4;
    for (uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; b < nblk;
         b += (uint64_t)gridDim.x * blockDim.x) {
        const u32x4 w = path_block(make_path_key(seed, 0, b, kStreamLevelDraw), 0);
        const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (4 * b + k >= N) break;
            const double u = u01d(words[k]);
            int l = 0;
            while (l < law.Lc && !(u < law.F[l])) ++l;
            atomicAdd(&hist[l], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < kRgLevels && hist[threadIdx.x])
        atomicAdd(&counts[threadIdx.x], (unsigned long long)hist[threadIdx.x]);
}

}  // namespace mlmc

using namespace mlmc;

extern "C" {

mlmc_status mlmc_rhee_glynn(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff,
                            int M, int L_cap, double q, uint64_t N, uint64_t seed, int precision,
                            mlmc_rg_result* out)
{
    if (!ctx) return MLMC_EINVAL;
    if (!out) return fail(ctx, MLMC_EINVAL, "out must not be NULL");
    mlmc_status st = check_level_args(ctx, model, payoff, L_cap, M, precision);
    if (st) return st;
    if (L_cap >= kRgLevels) return fail(ctx, MLMC_EINVAL, "L_cap must be at most 15");
    if (!(q > 0.0 && q < 1.0)) return fail(ctx, MLMC_EINVAL, "q must lie in (0, 1)");
    if (N == 0 || N > (1ull << 40)) return fail(ctx, MLMC_EINVAL, "N must be in 1..2^40");
    ctx->err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    std::memset(out, 0, sizeof(*out));
    // the law and its cumulative sums, in the same order as the oracle's
    RgLaw law;
    const double norm = 1.0 - std::pow(q, (double)(L_cap + 1));
    double acc = 0.0;
    for (int l = 0; l <= L_cap; ++l) {
        out->p[l] = (1.0 - q) * std::pow(q, (double)l) / norm;
        acc += out->p[l];
        law.F[l] = acc;
    }
    law.F[L_cap] = 1.0;
    for (int l = L_cap + 1; l < kRgLevels; ++l) law.F[l] = 1.0;
    law.Lc = L_cap;
    // counts in the first 16 words of the scratch record array
    unsigned long long* d_counts = (unsigned long long*)ctx->d_tmp;
    static_assert(3 * MLMC_MAX_LEVELS * sizeof(double) >= kRgLevels * sizeof(unsigned long long),
                  "scratch holds the histogram");
    MLMC_HIP(ctx, hipMemsetAsync(d_counts, 0, kRgLevels * sizeof(unsigned long long), ctx->stream));
    const uint64_t nblk = (N + 3) / 4;
    const unsigned grid = (unsigned)std::min<uint64_t>((nblk + 255) / 256, (uint64_t)ctx->num_cu * 8);
    hipLaunchKernelGGL(level_draw_kernel, dim3(grid), dim3(256), 0, ctx->stream, seed, N, law,
                       d_counts);
    MLMC_HIP(ctx, hipGetLastError());
    MLMC_HIP(ctx, hipMemcpyAsync(ctx->h_tmp, d_counts, kRgLevels * sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, ctx->stream));
    MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::memcpy(out->N, ctx->h_tmp, kRgLevels * sizeof(unsigned long long));
    // every drawn level on the ordinary sampler, one record per level
    static_assert(kRgLevels * kSpread <= kAccSlots, "one spread group per level");
    MLMC_HIP(ctx, zero_records(ctx->d_acc, kRgLevels * kSpread, ctx->stream));
    for (int l = 0; l <= L_cap; ++l) {
        if (!out->N[l]) continue;
        st = enqueue_level(ctx, *model, *payoff, l, M, out->N[l], seed, 0, precision,
                           kStreamNormal, 1, ctx->d_acc + l * kSpread, nullptr, nullptr, nullptr,
                           true);
        if (st) return st;
    }
    MLMC_HIP(ctx, hipMemcpyAsync(ctx->h_acc, ctx->d_acc, kRgLevels * kSpread * sizeof(LevelAcc),
                                 hipMemcpyDeviceToHost, ctx->stream));
    MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    harvest_timing(ctx);
    double z1 = 0.0, z2 = 0.0;
    for (int l = 0; l <= L_cap; ++l) {
        if (!out->N[l]) continue;
        const LevelAcc r = fold_records(ctx->h_acc + l * kSpread, kSpread);
        out->sum_y[l] = r.sum[0];
        out->sum_y2[l] = r.sum[1];
        out->n_nonfinite += r.n_nonfinite;
        out->cost += (double)out->N[l] * level_cost(*model, l, M);
        z1 += r.sum[0] / out->p[l];
        z2 += r.sum[1] / (out->p[l] * out->p[l]);
    }
    out->L_cap = L_cap;
    out->estimate = z1 / (double)N;
    out->variance = z2 / (double)N - out->estimate * out->estimate;
    out->rmse_est = std::sqrt(std::max(out->variance, 0.0) / (double)N);
    out->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (out->n_nonfinite)
        return fail(ctx, MLMC_ENONFINITE, "non-finite samples were left out of the sums");
    return MLMC_OK;
}

}  // extern "C"
