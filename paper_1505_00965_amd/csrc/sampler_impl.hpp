// Path loop shared by the per-level kernel and the persistent kernel.
#pragma once
#include "level.hpp"

namespace mlmc {

// Add one sample's payoffs into the lane sums (and the optional dump).
template <typename Real>
__device__ __forceinline__ void accumulate(const LevelArgs<Real>& a, uint64_t idx, Real pf, Real pc,
                                           double (&sums)[kNumSums], unsigned& nonfinite)
{
    const double df = (double)pf, dc = (double)pc;
    if (a.pf_out) {
        a.pf_out[idx] = df;
        a.pc_out[idx] = dc;
    }
    const double y = df - dc;
    if (!isfinite(y)) {
        ++nonfinite;
        return;
    }
    sums[0] += y;
    sums[1] = __builtin_fma(y, y, sums[1]);
    sums[2] += df;
    sums[3] = __builtin_fma(df, df, sums[3]);
    sums[4] += dc;
    sums[5] = __builtin_fma(dc, dc, sums[5]);
}

// Advance PPT coupled pairs through all n_f >= 4 fine steps of the level.
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
    // n_f >= 4 here (a multiple of 4): every group holds four fine steps
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
                fine_step<Real, MODEL, PAYOFF>(q[p], P, dw1[k], dwp[k], e[k], k % M, coupled);
                if (coupled && ((k + 1) % M) == 0) coarse_step<Real, MODEL, PAYOFF>(q[p], P);
            }
        }
    }
}

// Samples base + p * blockDim + threadIdx (p < PPT) of the range described
// by a (a.offset + index, index < a.N): simulate, then add into the lane sums.
template <int MODEL, int PAYOFF, typename Real, int M, int PPT>
__device__ __forceinline__ void process_chunk(const LevelArgs<Real>& a, uint64_t base,
                                              double (&sums)[kNumSums], unsigned& nonfinite)
{
    const bool coupled = a.coupled && a.l > 0;
    const Real dtf = a.P.h, dtc = a.P.H;
    {
        uint64_t idx[PPT], s[PPT];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            idx[p] = base + (uint64_t)p * blockDim.x + threadIdx.x;
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
            accumulate(a, idx[p], pf, pc, sums, nonfinite);
        }
    }
}

// Levels with n_f = NF in {1, 2}: Q = 4/(NF d) consecutive samples share one
// generator block (d = 1 for GBM, 2 for Heston), as do 4/NF samples one
// bridge block.  A lane takes PPT blocks, i.e. Q * PPT samples; block B of
// the level covers samples Q B .. Q B + Q - 1 (those outside
// [offset, offset + N) are computed and dropped).  blk_base indexes blocks
// from B0 = offset / Q.
template <int MODEL, int PAYOFF, typename Real, int NF, int M, int PPT>
__device__ __forceinline__ void process_short(const LevelArgs<Real>& a, uint64_t blk_base,
                                              double (&sums)[kNumSums], unsigned& nonfinite)
{
    constexpr int D = (MODEL == kGBM) ? 1 : 2;
    constexpr int T = NF * D;             // normals per sample: 1, 2 or 4
    constexpr int Q = 4 / T;              // samples per generator block
    constexpr int QU = 4 / NF;            // samples per bridge block
    const StepParams<Real>& P = a.P;
    const bool coupled = a.coupled && a.l > 0;   // NF == 2 with M == 2 only
    const uint64_t B0 = a.offset / Q;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const uint64_t B = B0 + blk_base + (uint64_t)p * blockDim.x + threadIdx.x;
        const u32x4 w = path_block(make_path_key(a.seed, a.l, B, a.stream), 0);
        Real z[4];
        box_muller(w.x, w.y, z[0], z[1]);
        box_muller(w.z, w.w, z[2], z[3]);
        Real e[4] = {Real(0), Real(0), Real(0), Real(0)};
        if (PAYOFF == kLookback) {
            // every sample of this generator block reads bridge block B / D
            const u32x4 u = path_block(make_path_key(a.seed, a.l, B / D, a.stream + 1u), 0);
            e[0] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.x));
            e[1] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.y));
            e[2] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.z));
            e[3] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.w));
        }
#pragma unroll
        for (int r = 0; r < Q; ++r) {
            const uint64_t s = B * Q + r;
            PathPair<Real> q;
            init_pair<Real, MODEL, PAYOFF>(q, P);
            const int ub = (int)(s % QU) * NF;   // first bridge word of the sample
#pragma unroll
            for (int k = 0; k < NF; ++k) {
                const Real dw1 = P.sqh * z[r * T + k * D];
                const Real dwp = (D == 2) ? P.sqh * z[r * T + k * D + 1] : Real(0);
                fine_step<Real, MODEL, PAYOFF>(q, P, dw1, dwp, e[(ub + k) & 3], k % M, coupled);
            }
            if (NF == 2 && coupled) coarse_step<Real, MODEL, PAYOFF>(q, P);
            Real pf = payoff_value<Real, PAYOFF>(P, q.S, q.asum, q.acomp, q.mn, P.h);
            // level 0 with the control variate: every sample starts at (0, S0)
            if (NF == 1 && a.phi0) pf -= (Real)(*a.phi0) * (P.sqh * z[r * T]);
            const Real pc = coupled ? payoff_value<Real, PAYOFF>(P, q.Sc, q.csum, q.ccomp, q.mnc, P.H)
                                    : Real(0);
            if (s < a.offset || s - a.offset >= a.N) continue;
            accumulate(a, s - a.offset, pf, pc, sums, nonfinite);
        }
    }
}

// Number of generator blocks a short level's range [offset, offset + N) touches.
__host__ __device__ inline uint64_t short_blocks(uint64_t offset, uint64_t N, int q)
{
    if (N == 0) return 0;
    return (offset + N - 1) / q - offset / q + 1;
}

}  // namespace mlmc
