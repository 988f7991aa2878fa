// Device arithmetic of the adaptive MLMC driver (shared by the update
// kernel and the device-resident run loop).
//
// The paper fixes the estimator Y = sum_l Yhat_l (eq. (eq:mlmc:ident)), that
// level variances add (Sec. 5), the cost measure (Sec. 3), and leaves N_l to
// an optimisation over estimated variances (Sec. 5, "Constructive Upper
// Bound"); the complexity theorem sets the target E[(Y - E P)^2] < eps^2.
// Reading used: eps is an RMSE split evenly into bias^2 and variance;
// minimising sum N_l C_l under sum V_l/N_l = eps^2/2 gives
// N_l = ceil(2 eps^-2 sqrt(V_l/C_l) sum_k sqrt(V_k C_k)); costs
// C_0 = 1, C_l = M^l + M^(l-1); estimates floored by the assumed rates from
// l = 2; a level is resampled when its shortfall exceeds 1%; the bias is
// estimated from weak order alpha (eq. (eq:emweak)).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "driver.hpp"

namespace mlmc {

__device__ inline double level_cost_dev(int l, int M, int antithetic)
{
    if (l == 0) return 1.0;
    double a = 1.0;
    for (int i = 0; i < l - 1; ++i) a *= M;
    return (antithetic ? 2.0 : 1.0) * a * M + a;
}

__device__ inline void optimal_n_dev(int L, const double* V, const double* C, double eps, double* N)
{
    double total = 0.0;
    for (int k = 0; k <= L; ++k) total += sqrt(V[k] * C[k]);
    for (int l = 0; l <= L; ++l) N[l] = ceil(2.0 / (eps * eps) * sqrt(V[l] / C[l]) * total);
}

__device__ inline double fit_rate_dev(int L, const double* y, int M)
{
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    int n = 0;
    const double lm = log((double)M);
    for (int l = 1; l <= L; ++l) {
        if (!(y[l] > 0)) continue;
        const double x = l, v = log(y[l]) / lm;
        sx += x; sy += v; sxx += x * x; sxy += x * v; ++n;
    }
    if (n < 2) return nan("");
    return (n * sxy - sx * sy) / (n * sxx - sx * sx);
}

// Absorb the batch, re-plan.  One thread; a handful of fp64 operations.
__device__ __forceinline__ void driver_update_dev(DriverState* st)
{
    const int M = st->M;
    const double Ma = st->Ma, Mb = st->Mb;
    int L = st->L;
    for (int l = 0; l <= L; ++l) {
        if (st->dN[l] > 0) {
            st->sum1[l] += st->batch[l].sum[0];
            st->sum2[l] += st->batch[l].sum[1];
            st->n[l] += st->dN[l];
            st->n_nonfinite += st->batch[l].n_nonfinite;
        }
        for (int k = 0; k < kNumSums; ++k) st->batch[l].sum[k] = 0.0;
        st->batch[l].n_nonfinite = 0;
        st->dN[l] = 0.0;
    }
    st->iterations += 1;
    for (int l = 0; l <= L; ++l) {
        st->C[l] = level_cost_dev(l, M, st->antithetic);
        const double m = st->sum1[l] / st->n[l];
        st->E[l] = fabs(m);
        st->V[l] = st->sum2[l] / st->n[l] - m * m;
        if (st->V[l] < 0) st->V[l] = 0;
    }
    for (int l = 2; l <= L; ++l) {
        if (st->E[l] < st->E[l - 1] / Ma) st->E[l] = st->E[l - 1] / Ma;
        if (st->V[l] < st->V[l - 1] / Mb) st->V[l] = st->V[l - 1] / Mb;
    }
    optimal_n_dev(L, st->V, st->C, st->eps, st->Nopt);
    int more = 0;
    for (int l = 0; l <= L; ++l) {
        const double d = st->Nopt[l] - st->n[l];
        st->dN[l] = (d > 0.01 * st->n[l]) ? d : 0.0;
        if (st->dN[l] > 0) more = 1;
    }
    if (!more) {
        const double rem = fmax(st->E[L], st->E[L - 1] / Ma) / (Ma - 1.0);
        st->bias_est = rem;
        if (rem <= st->eps / sqrt(2.0)) {
            st->converged = 1;
            st->done = 1;
        } else if (L == st->L_max) {
            st->done = 1;
        } else {
            ++L;
            st->V[L] = st->V[L - 1] / Mb;
            st->E[L] = st->E[L - 1] / Ma;
            st->C[L] = level_cost_dev(L, M, st->antithetic);
            st->n[L] = 0;
            st->sum1[L] = 0;
            st->sum2[L] = 0;
            optimal_n_dev(L, st->V, st->C, st->eps, st->Nopt);
            for (int l = 0; l <= L; ++l) {
                const double d = st->Nopt[l] - st->n[l];
                st->dN[l] = (l == L) ? (st->Nopt[l] > 1 ? st->Nopt[l] : 1.0)
                                     : ((d > 0.01 * st->n[l]) ? d : 0.0);
            }
            st->L = L;
        }
    }
    if (st->iterations >= st->max_iterations) st->done = 1;
    if (st->done) {
        // nothing more is sampled: a launch planned from this state is empty
        for (int l = 0; l < kMaxLevels; ++l) st->dN[l] = 0.0;
        double est = 0.0, var = 0.0;
        double absE[kMaxLevels], Vr[kMaxLevels];
        for (int l = 0; l <= st->L; ++l) {
            const double m = st->sum1[l] / st->n[l];
            est += m;
            const double v = st->sum2[l] / st->n[l] - m * m;
            var += (v > 0 ? v : 0) / st->n[l];
            absE[l] = fabs(m);
            Vr[l] = v;
        }
        st->estimate = est;
        st->var_est = var;
        st->alpha_fit = -fit_rate_dev(st->L, absE, M);
        st->beta_fit = -fit_rate_dev(st->L, Vr, M);
        st->gamma_fit = fit_rate_dev(st->L, st->C, M);
    }
}

// The update is a serial chain of a few hundred dependent fp64 operations on
// the state, so the state is staged in LDS (a global round trip per access
// would dominate), updated by one lane, and written back.  The same words go
// to the host's pinned mirror (if any): everything before the batch records
// but `seq` first, then a system-scope fence, then `seq` (there 2 x the
// update count + the done flag), so a host that sees the new word sees the
// whole update, and the done flag of that same update.  Once the state is done the call
// does nothing (no write, `seq` unchanged), so launches queued past the last
// update are harmless.  With `spread` (kMaxLevels spread
// groups, one per level) the block first folds each sampled level's group
// into batch[l] (the sums of Y and Y^2 and the non-finite count), one wave
// per level, and clears it.  Every thread of the block must call it; `s` is
// the block's LDS copy of the state.
__device__ __forceinline__ void driver_update_block(DriverState* st, DriverState* mirror, DriverState& s,
                                                    LevelAcc* spread)
{
    static_assert(sizeof(DriverState) % 8 == 0, "state is copied in 8-byte words");
    static_assert(offsetof(DriverState, seq) % 8 == 0, "seq is one word");
    static_assert(offsetof(DriverState, batch) % 8 == 0, "batch starts a word");
    constexpr int kWords = sizeof(DriverState) / 8;
    constexpr int kSeq = offsetof(DriverState, seq) / 8;
    const unsigned long long* src = (const unsigned long long*)st;
    unsigned long long* w = (unsigned long long*)&s;
    for (int i = threadIdx.x; i < kWords; i += blockDim.x) w[i] = src[i];
    __syncthreads();
    // a finished run stays as it is (block-uniform: every thread reads the
    // same LDS word after the barrier); nothing was sampled since, so the
    // spread groups hold zeros
    if (s.done) return;
    if (spread) {
        static_assert(kSpread == 64, "one lane per record of a group");
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const int nwaves = (int)(blockDim.x >> 6);
        // the update reads sum Y, sum Y^2 and the non-finite count only
        for (int l = wave; l <= s.L; l += nwaves) {    // wave-uniform
            LevelAcc& r = spread[l * kSpread + lane];
            const double y = wave_sum(r.sum[0]);
            const double y2 = wave_sum(r.sum[1]);
            const double c = wave_sum((double)r.n_nonfinite);
#pragma unroll
            for (int k = 0; k < kNumSums; ++k) r.sum[k] = 0.0;
            r.n_nonfinite = 0;
            if (lane == 0) {
                s.batch[l].sum[0] += y;
                s.batch[l].sum[1] += y2;
                s.batch[l].n_nonfinite += (unsigned long long)c;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        driver_update_dev(&s);
        s.seq += 1;
    }
    __syncthreads();
    // the host waits for the mirror: publish it first; the device copy is
    // read by the next update only, which the stream orders after this one
    if (mirror) {
        // the host never reads the batch records: every word before them
        constexpr int kMirrorWords = offsetof(DriverState, batch) / 8;
        static_assert(kSeq < kMirrorWords, "seq precedes the batch records");
        volatile unsigned long long* h = (volatile unsigned long long*)mirror;
        for (int i = threadIdx.x; i < kMirrorWords; i += blockDim.x)
            if (i != kSeq) h[i] = w[i];
        __threadfence_system();
        __syncthreads();
        // the published word carries the done flag beside the update count
        if (threadIdx.x == 0) h[kSeq] = 2ull * w[kSeq] + (s.done ? 1ull : 0ull);
    }
    unsigned long long* dst = (unsigned long long*)st;
    for (int i = threadIdx.x; i < kWords; i += blockDim.x) dst[i] = w[i];
}

}  // namespace mlmc
