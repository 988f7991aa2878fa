// Adaptive MLMC driver: the fp64 update kernel and the host loops (the
// arithmetic itself is in driver_dev.hpp).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>

#include "context.hpp"
#include "driver.hpp"
#include "driver_dev.hpp"
#include "trace.hpp"

namespace mlmc {

__global__ void optimal_n_kernel(int L, const double* V, const double* C, double eps, double* N)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) optimal_n_dev(L, V, C, eps, N);
}

// A fresh state: zeros, the configuration, n_pilot outstanding samples on
// levels 0..L_min (the host mirror is filled the same way on the host); the
// per-level spread groups cleared.
__global__ void driver_init_kernel(DriverState* st, LevelAcc* spread, DriverInit c)
{
    unsigned long long* g = (unsigned long long*)spread;
    constexpr int kSpreadWords = kMaxLevels * kSpread * (int)sizeof(LevelAcc) / 8;
    for (int i = threadIdx.x; i < kSpreadWords; i += blockDim.x) g[i] = 0ull;
    init_state(*st, c);
}

// has_init: the run's first update, which builds the state itself (the
// spread groups hold the pilot's sums and nothing else).
__global__ __launch_bounds__(512) void driver_update_kernel(DriverState* st, DriverState* mirror,
                                                            LevelAcc* spread, DriverInit c,
                                                            int has_init)
{
    __shared__ DriverState s;
    driver_update_block(st, mirror, s, spread, has_init ? &c : nullptr);
}

// Wait until the host mirror shows update number `want`.  Spinning on the
// mirror saves the completion signal and wake-up of a stream synchronisation;
// the stream is polled as well, so a failed launch ends the wait with its
// error.
hipError_t wait_update(hipStream_t stream, const DriverState* h, unsigned long long want)
{
    auto next_poll = std::chrono::steady_clock::now() + std::chrono::milliseconds(1);
    for (;;) {
        if (mirror_updates(h) >= want) {
            std::atomic_thread_fence(std::memory_order_acquire);
            return hipSuccess;
        }
        // querying the stream costs the runtime work; once a millisecond is enough
        if (std::chrono::steady_clock::now() >= next_poll) {
            next_poll += std::chrono::milliseconds(1);
            const hipError_t e = hipStreamQuery(stream);
            if (e == hipSuccess) {
                std::atomic_thread_fence(std::memory_order_acquire);
                return mirror_updates(h) >= want ? hipSuccess : hipErrorUnknown;
            }
            if (e != hipErrorNotReady) return e;
        }
    }
}

hipError_t launch_driver_update(DriverState* st, DriverState* mirror, LevelAcc* spread,
                                hipStream_t stream, hipEvent_t start, hipEvent_t stop,
                                const DriverInit* init)
{
    const DriverInit c = init ? *init : DriverInit{};
    const int has_init = init ? 1 : 0;
    if (start || stop)
        hipExtLaunchKernelGGL(driver_update_kernel, dim3(1), dim3(512), 0, stream, start, stop, 0, st,
                              mirror, spread, c, has_init);
    else
        hipLaunchKernelGGL(driver_update_kernel, dim3(1), dim3(512), 0, stream, st, mirror, spread, c,
                           has_init);
    return hipGetLastError();
}

void free_driver(mlmc_ctx* ctx)
{
    if (ctx->d_drv) hipFree(ctx->d_drv);
    if (ctx->d_drv_spread) hipFree(ctx->d_drv_spread);
    if (ctx->h_drv) hipHostFree(ctx->h_drv);
    ctx->d_drv = ctx->h_drv = ctx->h_drv_dev = nullptr;
    ctx->d_drv_spread = nullptr;
}

// The mirror's device address is taken last, so it marks a complete set; a
// set left incomplete by a failed allocation is released and made again.
static mlmc_status ensure_driver(mlmc_ctx* ctx)
{
    if (ctx->h_drv_dev) return MLMC_OK;
    free_driver(ctx);
    hipError_t e = hipMalloc(&ctx->d_drv, sizeof(DriverState));
    if (e == hipSuccess)
        e = hipMalloc(&ctx->d_drv_spread, sizeof(LevelAcc) * kMaxLevels * kSpread);
    if (e == hipSuccess) e = hipHostMalloc(&ctx->h_drv, sizeof(DriverState));
    if (e == hipSuccess) e = hipHostGetDevicePointer(&ctx->h_drv_dev, ctx->h_drv, 0);
    if (e != hipSuccess) {
        free_driver(ctx);
        return hip_fail(ctx, e, "driver state allocation");
    }
    return MLMC_OK;
}

// persistent.hip: the device-planned form (start kernel, then the sampler
// and the update-and-plan block per iteration)
mlmc_status run_persistent(mlmc_ctx* ctx, const mlmc_model& m, const mlmc_payoff& p,
                           const mlmc_run_opts& o, DriverState* d_st, DriverState* h_st,
                           const DriverInit& init, bool prepared);

}  // namespace mlmc

using namespace mlmc;

extern "C" {

mlmc_status mlmc_optimal_n(mlmc_ctx* ctx, int L, const double* V, const double* C, double eps,
                           double* N)
{
    if (!ctx) return MLMC_EINVAL;
    if (L < 0 || L >= MLMC_MAX_LEVELS || !V || !C || !N || !(eps > 0))
        return fail(ctx, MLMC_EINVAL, "need 0 <= L < 16, eps > 0 and non-NULL arrays");
    for (int l = 0; l <= L; ++l)
        if (!(V[l] >= 0) || !(C[l] > 0)) return fail(ctx, MLMC_EINVAL, "need V >= 0 and C > 0");
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    const size_t n = (size_t)(L + 1);
    double* dV = ctx->d_tmp;
    double* dC = ctx->d_tmp + MLMC_MAX_LEVELS;
    double* dN = ctx->d_tmp + 2 * MLMC_MAX_LEVELS;
    std::memcpy(ctx->h_tmp, V, n * sizeof(double));
    std::memcpy(ctx->h_tmp + MLMC_MAX_LEVELS, C, n * sizeof(double));
    MLMC_HIP(ctx, hipMemcpyAsync(ctx->d_tmp, ctx->h_tmp, 2 * MLMC_MAX_LEVELS * sizeof(double),
                                 hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(optimal_n_kernel, dim3(1), dim3(64), 0, ctx->stream, L, dV, dC, eps, dN);
    MLMC_HIP(ctx, hipGetLastError());
    MLMC_HIP(ctx, hipMemcpyAsync(ctx->h_tmp + 2 * MLMC_MAX_LEVELS, dN, n * sizeof(double),
                                 hipMemcpyDeviceToHost, ctx->stream));
    MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::memcpy(N, ctx->h_tmp + 2 * MLMC_MAX_LEVELS, n * sizeof(double));
    return MLMC_OK;
}

mlmc_status mlmc_run(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff,
                     const mlmc_run_opts* opts, mlmc_run_result* out)
{
    if (!ctx) return MLMC_EINVAL;
    if (!opts || !out) return fail(ctx, MLMC_EINVAL, "opts and out must not be NULL");
    const mlmc_run_opts& o = *opts;
    mlmc_status st = check_level_args(ctx, model, payoff, 0, o.M, o.precision);
    if (st) return st;
    if (!(o.eps > 0)) return fail(ctx, MLMC_EINVAL, "eps must be > 0");
    if (o.L_min < 1 || o.L_max < o.L_min || o.L_max > 12)
        return fail(ctx, MLMC_EINVAL, "need 1 <= L_min <= L_max <= 12");
    if ((o.M == 4 && o.L_max > 9)) return fail(ctx, MLMC_EINVAL, "L_max too deep for M = 4");
    if (o.n_pilot < 2) return fail(ctx, MLMC_EINVAL, "n_pilot must be >= 2");
    if (o.cv && o.precision != 32)
        return fail(ctx, MLMC_EINVAL, "the control variate runs in fp32 paths only");
    if (o.persistent != 0 && o.persistent != 1)
        return fail(ctx, MLMC_EINVAL, "persistent must be 0 or 1");
    if (o.cv && o.persistent && !cv_tabulated(o.cv))
        return fail(ctx, MLMC_EINVAL,
                    "the device-planned form takes the tabulated control variate (mlmc_cv_set_tabulated)");
    if (model->antithetic && o.persistent)
        return fail(ctx, MLMC_EINVAL, "the antithetic estimator runs with per-level launches only");
    ctx->err.clear();
    const TraceRange run_range("mlmc_run");
    const auto t0 = std::chrono::steady_clock::now();
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    st = ensure_driver(ctx);
    if (st) return st;
    DriverState* h = (DriverState*)ctx->h_drv;
    DriverState* d = (DriverState*)ctx->d_drv;
    std::memset(h, 0, sizeof(DriverState));
    h->eps = o.eps;
    h->alpha = o.alpha > 0 ? o.alpha : 1.0;
    h->beta = o.beta > 0 ? o.beta : 1.0;
    h->Ma = std::pow((double)o.M, h->alpha);
    h->Mb = std::pow((double)o.M, h->beta);
    h->M = o.M;
    h->antithetic = model->antithetic;
    h->L_min = o.L_min;
    h->L_max = o.L_max;
    h->max_iterations = 1000;
    h->L = o.L_min;
    for (int l = 0; l <= o.L_min; ++l) h->dN[l] = (double)o.n_pilot;
    // the device copy from the same few values (a launch costs the host less
    // than a host-to-device copy of the whole state)
    DriverInit init;
    init.eps = h->eps;
    init.alpha = h->alpha;
    init.beta = h->beta;
    init.Ma = h->Ma;
    init.Mb = h->Mb;
    init.n_pilot = (double)o.n_pilot;
    init.M = h->M;
    init.antithetic = h->antithetic;
    init.L_min = h->L_min;
    init.L_max = h->L_max;
    init.max_iterations = h->max_iterations;
    init.pad = 0;
    // When the spread groups are known to hold zeros, the per-level form
    // lets its first update build the state (one launch fewer on the pilot's
    // path), and the device-planned form skips its start kernel if the last
    // call, a device-planned run, left the next run's start prepared;
    // otherwise a kernel clears both first (in the device-planned form, its
    // start kernel).  Until this run ends normally neither is known.
    const bool fused_init = ctx->drv_clean && !o.persistent;
    const bool prepared = ctx->drv_clean && ctx->drv_pilot_ready;
    ctx->drv_clean = false;
    ctx->drv_pilot_ready = false;
    if (!fused_init && !o.persistent) {
        hipLaunchKernelGGL(driver_init_kernel, dim3(1), dim3(256), 0, ctx->stream, d,
                           ctx->d_drv_spread, init);
        MLMC_HIP(ctx, hipGetLastError());
    }
    if (o.persistent) {
        st = run_persistent(ctx, *model, *payoff, o, d, h, init, prepared);
        if (st) return st;
    } else {
        for (int it = 0;; ++it) {
            // the device stops at max_iterations; a host loop past that means
            // the mirror is not being written
            if (it > h->max_iterations + 1)
                return fail(ctx, MLMC_EDEVICE, "driver state did not reach the host");
            const TraceRange iter_range("mlmc_run driver iteration");
            // deepest level first: level 0's launch (the largest, and the
            // dearest for the host when its kernels are timed) is enqueued
            // last, while the deeper levels run
            for (int l = h->L; l >= 0; --l) {
                if (h->dN[l] <= 0) continue;
                const mlmc_cv* cv = (o.cv && (o.cv_levels <= 0 || l < o.cv_levels)) ? o.cv : nullptr;
                st = enqueue_level(ctx, *model, *payoff, l, o.M, (uint64_t)h->dN[l], o.seed,
                                   (uint64_t)h->n[l], o.precision, kStreamNormal, 1,
                                   ctx->d_drv_spread + l * kSpread, nullptr, nullptr, cv, true);
                if (st) return st;
            }
            hipEvent_t t0, t1;
            timed_kernel(ctx, 17, 0.0, 0.0, &t0, &t1);
            MLMC_HIP(ctx, launch_driver_update(d, (DriverState*)ctx->h_drv_dev, ctx->d_drv_spread,
                                               ctx->stream, t0, t1,
                                               (it == 0 && fused_init) ? &init : nullptr));
            MLMC_HIP(ctx, wait_update(ctx->stream, h, (unsigned long long)it + 1));
            if (mirror_done(h)) break;
        }
        // the mirror holds the final state; stamped launches that have
        // finished are read now, the rest (the last update's, usually) by a
        // later harvest: the run does not wait for the stream
        if (!ctx->pending.empty()) harvest_ready(ctx);
    }
    ctx->drv_clean = true;
    const auto t1 = std::chrono::steady_clock::now();
    std::memset(out, 0, sizeof(*out));
    out->estimate = h->estimate;
    out->rmse_est = std::sqrt(h->var_est + h->bias_est * h->bias_est);
    out->wall_s = std::chrono::duration<double>(t1 - t0).count();
    out->L = h->L;
    out->converged = h->converged;
    out->iterations = h->iterations;
    double cost = 0.0;
    for (int l = 0; l <= h->L; ++l) {
        out->N[l] = (uint64_t)h->n[l];
        out->sum_y[l] = h->sum1[l];
        out->sum_y2[l] = h->sum2[l];
        out->E[l] = h->sum1[l] / h->n[l];
        out->V[l] = h->sum2[l] / h->n[l] - out->E[l] * out->E[l];
        out->C[l] = h->C[l];
        cost += h->n[l] * h->C[l];
    }
    out->alpha = h->alpha_fit;
    out->beta = h->beta_fit;
    out->gamma = h->gamma_fit;
    out->cost = cost;
    out->n_nonfinite = h->n_nonfinite;
    if (h->n_nonfinite)
        return fail(ctx, MLMC_ENONFINITE, "non-finite samples were left out of the sums");
    if (!h->converged) {
        if (h->iterations >= h->max_iterations)
            return fail(ctx, MLMC_EDEVICE, "driver did not settle within its iteration limit");
        return fail(ctx, MLMC_ENOTCONV, "L_max reached before the bias test passed");
    }
    return MLMC_OK;
}

}  // extern "C"
