// Device arithmetic of the adaptive MLMC driver (the update kernel and the
// optimal-N entry point).
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

// A fresh state in `s` (global or LDS): zeros, the configuration, the pilot
// batch.  Every thread of the block must call it; it ends with a barrier.
__device__ __forceinline__ void init_state(DriverState& s, const DriverInit& c)
{
    static_assert(sizeof(DriverState) % 8 == 0, "state is cleared in 8-byte words");
    unsigned long long* w = (unsigned long long*)&s;
    for (int i = threadIdx.x; i < (int)(sizeof(DriverState) / 8); i += blockDim.x) w[i] = 0ull;
    __syncthreads();
    if (threadIdx.x == 0) {
        s.eps = c.eps;
        s.alpha = c.alpha;
        s.beta = c.beta;
        s.Ma = c.Ma;
        s.Mb = c.Mb;
        s.M = c.M;
        s.antithetic = c.antithetic;
        s.L_min = c.L_min;
        s.L_max = c.L_max;
        s.max_iterations = c.max_iterations;
        s.L = c.L_min;
        for (int l = 0; l <= c.L_min; ++l) s.dN[l] = c.n_pilot;
    }
    __syncthreads();
}

// Value of lane l (wave-uniform l) of a per-lane double.
__device__ __forceinline__ double lane_f64(double v, int l)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, l);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// sum_{k <= L} v_k in level order (the order of the one-lane loops above),
// so every sum over levels rounds as optimal_n_dev and fit_rate_dev round it.
__device__ __forceinline__ double ordered_sum(double v, int L)
{
    double t = 0.0;
    for (int k = 0; k <= L; ++k) t += lane_f64(v, k);
    return t;
}

// Absorb the batch, re-plan: the first wave of the block, lane l holding
// level l.  The per-level formulas run side by side; what couples levels
// (the floors from the level below, the sums over levels, the bias test)
// takes the levels in order, so every result is the one-lane loop's, bit
// for bit.  `s` is the block's LDS copy of the state; all 64 lanes call it.
__device__ __forceinline__ void driver_update_wave(DriverState& s)
{
    static_assert(kMaxLevels <= 64, "one lane per level");
    const int lane = (int)(threadIdx.x & 63);
    const int li = lane < kMaxLevels ? lane : kMaxLevels - 1;   // in-bounds index
    const int M = s.M;
    const double Ma = s.Ma, Mb = s.Mb, eps = s.eps;
    const int L0 = __builtin_amdgcn_readfirstlane(s.L);   // the same word in every lane
    bool in = lane <= L0;
    double n = s.n[li], dN = s.dN[li], sum1 = s.sum1[li], sum2 = s.sum2[li];
    double E = s.E[li], V = s.V[li], C = s.C[li], Nopt = s.Nopt[li];
    // absorb the batch (every level's record is cleared)
    unsigned long long nonfinite = 0;
    if (in && dN > 0) {
        sum1 += s.batch[li].sum[0];
        sum2 += s.batch[li].sum[1];
        n += dN;
        nonfinite = s.batch[li].n_nonfinite;
    }
    if (in) dN = 0.0;
    // estimates, then the floors from the level below (l >= 2, in order)
    double m = 0.0;
    if (in) {
        C = level_cost_dev(lane, M, s.antithetic);
        m = sum1 / n;
        E = fabs(m);
        V = sum2 / n - m * m;
        if (V < 0) V = 0;
    }
    for (int l = 2; l <= L0; ++l) {
        const double Ep = lane_f64(E, l - 1), Vp = lane_f64(V, l - 1);
        if (lane == l) {
            if (E < Ep / Ma) E = Ep / Ma;
            if (V < Vp / Mb) V = Vp / Mb;
        }
    }
    // optimal N_l, the outstanding batch
    double total = ordered_sum(in ? sqrt(V * C) : 0.0, L0);
    if (in) Nopt = ceil(2.0 / (eps * eps) * sqrt(V / C) * total);
    if (in) {
        const double d = Nopt - n;
        dN = (d > 0.01 * n) ? d : 0.0;
    }
    const bool more = __ballot(in && dN > 0) != 0;
    int L = L0;
    int done = s.done, converged = s.converged;
    if (!more) {
        const double EL = lane_f64(E, L), EL1 = lane_f64(E, L - 1);
        const double rem = fmax(EL, EL1 / Ma) / (Ma - 1.0);
        if (lane == 0) s.bias_est = rem;
        if (rem <= eps / sqrt(2.0)) {
            converged = 1;
            done = 1;
        } else if (L == __builtin_amdgcn_readfirstlane(s.L_max)) {
            done = 1;
        } else {
            const double VL = lane_f64(V, L);
            ++L;
            in = lane <= L;
            if (lane == L) {
                V = VL / Mb;
                E = EL / Ma;
                C = level_cost_dev(L, M, s.antithetic);
                n = 0;
                sum1 = 0;
                sum2 = 0;
            }
            total = ordered_sum(in ? sqrt(V * C) : 0.0, L);
            if (in) {
                Nopt = ceil(2.0 / (eps * eps) * sqrt(V / C) * total);
                const double d = Nopt - n;
                dN = (lane == L) ? (Nopt > 1 ? Nopt : 1.0) : ((d > 0.01 * n) ? d : 0.0);
            }
        }
    }
    const int iterations = s.iterations + 1;
    if (iterations >= s.max_iterations) done = 1;
    // the non-finite counts of the absorbed levels, in any order (integers)
    unsigned long long nf_total = 0;
    for (int l = 0; l <= L0; ++l)
        nf_total += ((unsigned long long)__builtin_amdgcn_readlane((unsigned)(nonfinite >> 32), l) << 32) |
                    __builtin_amdgcn_readlane((unsigned)nonfinite, l);
    if (done) {
        // nothing more is sampled: a launch planned from this state is empty
        dN = 0.0;
        const double mr = in ? sum1 / n : 0.0;
        const double v = in ? sum2 / n - mr * mr : 0.0;
        const double est = ordered_sum(mr, L);
        const double var = ordered_sum(in ? (v > 0 ? v : 0) / n : 0.0, L);
        // fitted rates over l = 1..L of |E_l|, V_l and C_l
        const double lm = log((double)M);
        double rate[3];
        for (int f = 0; f < 3; ++f) {
            const double y = f == 0 ? fabs(mr) : (f == 1 ? v : C);
            const bool use = in && lane >= 1 && y > 0;
            const double vy = use ? log(y) / lm : 0.0;
            const unsigned long long used = __ballot(use);
            double sx = 0, sy = 0, sxx = 0, sxy = 0;
            int cnt = 0;
            for (int l = 1; l <= L; ++l) {
                if (!((used >> l) & 1ull)) continue;
                const double x = l, w = lane_f64(vy, l);
                sx += x; sy += w; sxx += x * x; sxy += x * w; ++cnt;
            }
            rate[f] = cnt < 2 ? nan("") : (cnt * sxy - sx * sy) / (cnt * sxx - sx * sx);
        }
        if (lane == 0) {
            s.estimate = est;
            s.var_est = var;
            s.alpha_fit = -rate[0];
            s.beta_fit = -rate[1];
            s.gamma_fit = rate[2];
        }
    }
    // write back: every level the update touched (the finished state has
    // no outstanding batch on any level)
    if (lane < kMaxLevels) {
        if (lane <= L) {
            s.n[lane] = n;
            s.sum1[lane] = sum1;
            s.sum2[lane] = sum2;
            s.E[lane] = E;
            s.V[lane] = V;
            s.C[lane] = C;
            s.Nopt[lane] = Nopt;
        }
        if (lane <= L || done) s.dN[lane] = lane <= L ? dN : 0.0;
        if (lane <= L0) {
#pragma unroll
            for (int k = 0; k < kNumSums; ++k) s.batch[lane].sum[k] = 0.0;
            s.batch[lane].n_nonfinite = 0;
        }
    }
    if (lane == 0) {
        s.n_nonfinite += nf_total;
        s.iterations = iterations;
        s.L = L;
        s.done = done;
        s.converged = converged;
    }
}

// The update is a chain of a few hundred dependent fp64 operations on the
// state, so the state is staged in LDS (a global round trip per access
// would dominate), updated by the first wave (one lane per level), and
// written back.  update_state and publish_state are its last two steps;
// driver_update_block is the whole update of the per-level form, and the
// device-planned form's kernel (persistent.hip) composes the steps itself.

// The first wave updates `s` (LDS) and counts the update; ends with a barrier.
__device__ __forceinline__ void update_state(DriverState& s)
{
    if (threadIdx.x < 64) driver_update_wave(s);
    if (threadIdx.x == 0) s.seq += 1;
    __syncthreads();
}

// Write the updated state `s` back to `st`, and to the host's pinned mirror
// (if any): with mirror_each, or once the state is done, everything before
// the batch records but `seq` first, then a system-scope fence, then `seq`
// (there 2 x the update count + the done flag), so a host that sees the new
// word sees the whole update, and the done flag of that same update;
// otherwise `seq` alone (for a host that reads the state at the end only).
// `seq` is a relaxed system-scope store: nothing waits for it, the kernel's
// end makes it visible.  Every thread of the block must call it.
__device__ __forceinline__ void publish_state(DriverState* st, DriverState* mirror, const DriverState& s,
                                              bool mirror_each)
{
    static_assert(sizeof(DriverState) % 8 == 0, "state is copied in 8-byte words");
    static_assert(offsetof(DriverState, seq) % 8 == 0, "seq is one word");
    static_assert(offsetof(DriverState, batch) % 8 == 0, "batch starts a word");
    constexpr int kWords = sizeof(DriverState) / 8;
    constexpr int kSeq = offsetof(DriverState, seq) / 8;
    const unsigned long long* w = (const unsigned long long*)&s;
    // the host waits for the mirror: publish it first; the device copy is
    // read by the next update only, which the stream orders after this one
    if (mirror) {
        // the host never reads the batch records: every word before them
        constexpr int kMirrorWords = offsetof(DriverState, batch) / 8;
        static_assert(kSeq < kMirrorWords, "seq precedes the batch records");
        unsigned long long* h = (unsigned long long*)mirror;
        if (mirror_each || s.done) {    // block-uniform (LDS after a barrier)
            for (int i = threadIdx.x; i < kMirrorWords; i += blockDim.x)
                if (i != kSeq) ((volatile unsigned long long*)h)[i] = w[i];
            __threadfence_system();
            __syncthreads();
        }
        // the published word carries the done flag beside the update count
        if (threadIdx.x == 0)
            __hip_atomic_store(&h[kSeq], 2ull * w[kSeq] + (s.done ? 1ull : 0ull), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
    }
    unsigned long long* dst = (unsigned long long*)st;
    for (int i = threadIdx.x; i < kWords; i += blockDim.x) dst[i] = w[i];
}

// The whole update of the per-level form.  Once the state is done the call
// does nothing (no write, `seq` unchanged), so launches queued past the last
// update are harmless.  With `spread` (kMaxLevels spread groups, one per
// level) the block first folds each sampled level's group into batch[l]
// (the sums of Y and Y^2 and the non-finite count), one wave per level, and
// clears it.  With `init` the state is built fresh in `s` instead of read
// (the first update of a run whose groups hold only the pilot's sums).
// Every thread of the block must call it; `s` is the block's LDS copy of the
// state.
__device__ __forceinline__ void driver_update_block(DriverState* st, DriverState* mirror, DriverState& s,
                                                    LevelAcc* spread, const DriverInit* init = nullptr)
{
    constexpr int kWords = sizeof(DriverState) / 8;
    const unsigned long long* src = (const unsigned long long*)st;
    unsigned long long* w = (unsigned long long*)&s;
    if (init) {
        init_state(s, *init);    // the run's first update: a fresh state
    } else {
        for (int i = threadIdx.x; i < kWords; i += blockDim.x) w[i] = src[i];
        __syncthreads();
    }
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
    update_state(s);
    publish_state(st, mirror, s, true);
}

// Sums of the spread groups per level (sum Y, sum Y^2 and the non-finite
// count), staged in LDS by the device-planned update.
struct GroupSums {
    double y[kMaxLevels], y2[kMaxLevels], c[kMaxLevels];
};

// Zero the spread groups of levels 0..L (every word of their records).
__device__ __forceinline__ void clear_groups(LevelAcc* spread, int L)
{
    static_assert(sizeof(LevelAcc) % 8 == 0, "records are cleared in 8-byte words");
    unsigned long long* w = (unsigned long long*)spread;
    const int n = (L + 1) * kSpread * (int)(sizeof(LevelAcc) / 8);
    for (int i = threadIdx.x; i < n; i += blockDim.x) w[i] = 0ull;
}

}  // namespace mlmc
