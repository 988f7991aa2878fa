// Path loop shared by the per-level kernel and the persistent kernel.
#pragma once
#include <type_traits>

#include "level.hpp"

namespace mlmc {

// Add one sample's payoffs into the lane sums.
template <typename Real>
__device__ __forceinline__ void add_sample(Real pf, Real pc, double (&sums)[kNumSums],
                                           unsigned& nonfinite)
{
    const double df = (double)pf, dc = (double)pc;
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

// One-step samples have no coarse payoff, so y = P_f: only the sums of y are
// kept per lane, and the P_f sums are copied from them once per block
// (copy_y_sums) before the reduction.
__device__ __forceinline__ void add_y(double y, double (&sums)[kNumSums], unsigned& nonfinite)
{
    if (!isfinite(y)) {
        ++nonfinite;
        return;
    }
    sums[0] += y;
    sums[1] = __builtin_fma(y, y, sums[1]);
}

__device__ __forceinline__ void copy_y_sums(double (&sums)[kNumSums])
{
    sums[2] = sums[0];
    sums[3] = sums[1];
}

// add_sample plus the optional per-sample dump.
template <typename Real>
__device__ __forceinline__ void accumulate(const LevelArgs<Real>& a, uint64_t idx, Real pf, Real pc,
                                           double (&sums)[kNumSums], unsigned& nonfinite)
{
    if (a.pf_out) {
        a.pf_out[idx] = (double)pf;
        a.pc_out[idx] = (double)pc;
    }
    add_sample(pf, pc, sums, nonfinite);
}

// Position of the antithetic twin's k-th increment inside a group of four:
// the increments of every coarse step (M of them) in reverse order.
template <int M>
__host__ __device__ constexpr int twin_index(int k) { return (k / M) * M + (M - 1 - k % M); }

// The twin runs its own coarse path only where the coarse payoff depends on
// the fine increments' order (the lookback's refined minimum); elsewhere the
// twin's coarse path equals the coupled one up to summation order.
template <int PAYOFF>
__host__ __device__ constexpr bool twin_coarse()
{
    return PAYOFF == kLookback || PAYOFF == kDigitalCond;
}

// Generator block g of a path (four fine steps): its increments, advanced
// through q's fine and coarse paths; with ANTI also through the antithetic
// twin qa (same generator words, the increments reversed inside every
// coarse step).
template <int MODEL, int PAYOFF, typename Real, int M, bool ANTI>
__device__ __forceinline__ void advance_group(const StepParams<Real>& P, const PathKey& key,
                                              const PathKey& bkey, uint32_t g, PathPair<Real>& q,
                                              PathPair<Real>& qa)
{
    Real dw1[4], dwp[4], e[4];
    if (one_factor(MODEL)) {
        const u32x4 w = path_block(key, g);
        brownian_pair(w.x, w.y, P, dw1[0], dw1[1]);
        brownian_pair(w.z, w.w, P, dw1[2], dw1[3]);
        dwp[0] = dwp[1] = dwp[2] = dwp[3] = Real(0);
    } else {
        const u32x4 wa = path_block(key, 2 * g);
        const u32x4 wb = path_block(key, 2 * g + 1);
        brownian_pair(wa.x, wa.y, P, dw1[0], dwp[0]);
        brownian_pair(wa.z, wa.w, P, dw1[1], dwp[1]);
        brownian_pair(wb.x, wb.y, P, dw1[2], dwp[2]);
        brownian_pair(wb.z, wb.w, P, dw1[3], dwp[3]);
    }
    if (PAYOFF == kLookback) {
        const u32x4 u = path_block(bkey, g);
        e[0] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.x));
        e[1] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.y));
        e[2] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.z));
        e[3] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.w));
    } else {
        e[0] = e[1] = e[2] = e[3] = Real(0);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        fine_step<Real, MODEL, PAYOFF>(q, P, dw1[k], dwp[k], e[k], k % M, true);
        if (((k + 1) % M) == 0) coarse_step<Real, MODEL, PAYOFF>(q, P);
    }
    if (ANTI) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            constexpr bool tc = twin_coarse<PAYOFF>();
            const int j = twin_index<M>(k);
            fine_step<Real, MODEL, PAYOFF>(qa, P, dw1[j], dwp[j], e[j], k % M, tc);
            if (tc && ((k + 1) % M) == 0) coarse_step<Real, MODEL, PAYOFF>(qa, P);
        }
    }
}

// Advance PPT coupled pairs through all n_f >= 4 fine steps of the level;
// with ANTI also each pair's antithetic twin qa.
template <int MODEL, int PAYOFF, typename Real, int M, int PPT, bool ANTI>
__device__ __forceinline__ void simulate(const LevelArgs<Real>& a, const uint64_t (&s)[PPT],
                                         PathPair<Real> (&q)[PPT], PathPair<Real> (&qa)[PPT])
{
    const StepParams<Real>& P = a.P;
    PathKey key[PPT], bkey[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        key[p] = PathKey{(uint32_t)a.seed, (uint32_t)(a.seed >> 32), (uint32_t)s[p], a.c2, a.stream};
        bkey[p] = PathKey{(uint32_t)a.seed, (uint32_t)(a.seed >> 32), (uint32_t)s[p], a.c2b,
                          a.stream + 1u};
        init_pair<Real, MODEL, PAYOFF>(q[p], P);
        if (ANTI) init_pair<Real, MODEL, PAYOFF>(qa[p], P);
    }
    // n_f >= 4 here (a multiple of 4): every group holds four fine steps.
    // The coarse path is advanced even when the caller drops it (standard
    // Monte Carlo at one level): a per-step choice would cost more lane
    // operations on the coupled levels than the coarse steps cost there.
    for (uint32_t g = 0; g < a.ngroups; ++g) {
#pragma unroll
        for (int p = 0; p < PPT; ++p)
            advance_group<MODEL, PAYOFF, Real, M, ANTI>(P, key[p], bkey[p], g, q[p], qa[p]);
    }
}

// Fine and coarse payoffs of a pair; with ANTI the averages over the pair
// and its twin pair (the twin's coarse payoff is the pair's own unless the
// twin runs a coarse path of its own).
template <int MODEL, int PAYOFF, typename Real>
__device__ __forceinline__ Real fine_payoff(const StepParams<Real>& P, const PathPair<Real>& q)
{
    if constexpr (PAYOFF == kDigitalCond) return cond_digital_fine<Real, MODEL>(P, q);
    else return payoff_value<Real, PAYOFF>(P, q.S, q.asum, q.acomp, q.mn, P.h);
}

template <int MODEL, int PAYOFF, typename Real>
__device__ __forceinline__ Real coarse_payoff(const StepParams<Real>& P, const PathPair<Real>& q)
{
    if constexpr (PAYOFF == kDigitalCond) return cond_digital_coarse<Real, MODEL>(P, q);
    else return payoff_value<Real, PAYOFF>(P, q.Sc, q.csum, q.ccomp, q.mnc, P.H);
}

template <int MODEL, int PAYOFF, typename Real, bool ANTI>
__device__ __forceinline__ void pair_payoffs(const StepParams<Real>& P, const PathPair<Real>& q,
                                             const PathPair<Real>& qa, bool coupled, Real& pf,
                                             Real& pc)
{
    pf = fine_payoff<MODEL, PAYOFF>(P, q);
    pc = coupled ? coarse_payoff<MODEL, PAYOFF>(P, q) : Real(0);
    if (ANTI) {
        pf = Real(0.5) * (pf + fine_payoff<MODEL, PAYOFF>(P, qa));
        if (twin_coarse<PAYOFF>()) pc = Real(0.5) * (pc + coarse_payoff<MODEL, PAYOFF>(P, qa));
    }
}

// Samples base + p * blockDim + threadIdx (p < PPT) of the range described
// by a (a.offset + index, index < a.N): simulate, then add into the lane sums.
// a.c2 and a.c2b are the counter words of the whole range (set_counter_words):
// the range lies within one segment of counter_segment_end.
template <int MODEL, int PAYOFF, typename Real, int M, int PPT, bool ANTI>
__device__ __forceinline__ void process_chunk(const LevelArgs<Real>& a, uint64_t base,
                                              double (&sums)[kNumSums], unsigned& nonfinite)
{
    const bool coupled = a.coupled && a.l > 0;
    uint64_t idx[PPT], s[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        idx[p] = base + (uint64_t)p * blockDim.x + threadIdx.x;
        s[p] = a.offset + idx[p];
    }
    PathPair<Real> q[PPT], qa[PPT];
    simulate<MODEL, PAYOFF, Real, M, PPT, ANTI>(a, s, q, qa);
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        Real pf, pc;
        pair_payoffs<MODEL, PAYOFF, Real, ANTI>(a.P, q[p], qa[p], coupled, pf, pc);
        if (idx[p] >= a.N) continue;
        accumulate(a, idx[p], pf, pc, sums, nonfinite);
    }
}

// GBM paths split across G = a.split consecutive lanes (a power of two up to
// 64), for levels whose paths are too few to fill the device.  Lane j of a
// path runs fine steps [j n_f/G, (j+1) n_f/G) from a unit start: the Euler
// and Milstein GBM steps, both coarse constructions and every payoff
// functional are linear in the start value (the terminal value is a product
// of segment factors, the sum of S_n adds the next segment's sum scaled by
// the product so far, the bridge minima scale the same way).  The segment
// summaries (P, Sigma, m) of fine and coarse path combine in path order,
// (P1, S1, m1) o (P2, S2, m2) = (P1 P2, S1 + P1 S2, min(m1, P1 m2)), in fp64
// over a shuffle tree, and the path's first lane forms the payoffs at scale
// S0.  n_f / G is a multiple of 4, so segments hold whole generator blocks
// and whole coarse steps.  base indexes paths; a block takes blockDim / G.
template <int MODEL, int PAYOFF, int M>
__device__ __forceinline__ void process_split(const LevelArgs<float>& a, uint64_t base,
                                              double (&sums)[kNumSums], unsigned& nonfinite)
{
    static_assert(MODEL != kHeston, "the variance step is not linear in the start value");
    static_assert(PAYOFF != kDigitalCond, "the conditional payoff needs the last step's state");
    const int G = (int)a.split;
    const int seg = (int)threadIdx.x & (G - 1);
    const uint64_t idx = base + threadIdx.x / (uint32_t)G;
    const uint64_t s = a.offset + idx;
    const bool coupled = a.coupled && a.l > 0;
    const StepParams<float>& P = a.P;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const PathKey key{k0, k1, (uint32_t)s, a.c2, a.stream};
    const PathKey bkey{k0, k1, (uint32_t)s, a.c2b, a.stream + 1u};
    PathPair<float> q, qa;
    init_pair<float, MODEL, PAYOFF>(q, P);
    q.S = 1.0f;
    q.Sc = 1.0f;
    const uint32_t per = a.ngroups / (uint32_t)G;     // generator blocks per lane
    for (uint32_t g = (uint32_t)seg * per; g < (uint32_t)(seg + 1) * per; ++g)
        advance_group<MODEL, PAYOFF, float, M, false>(P, key, bkey, g, q, qa);
    double pf = q.S, sf = (double)q.asum - (double)q.acomp, mf = q.mn;
    double pc = q.Sc, sc = (double)q.csum - (double)q.ccomp, mc = q.mnc;
    for (int off = 1; off < G; off <<= 1) {
        const double pf2 = __shfl_down(pf, off, G), pc2 = __shfl_down(pc, off, G);
        double sf2 = 0, sc2 = 0, mf2 = 0, mc2 = 0;
        if (PAYOFF == kAsian) {
            sf2 = __shfl_down(sf, off, G);
            sc2 = __shfl_down(sc, off, G);
        }
        if (PAYOFF == kLookback) {
            mf2 = __shfl_down(mf, off, G);
            mc2 = __shfl_down(mc, off, G);
        }
        if ((seg & (2 * off - 1)) == 0) {
            if (PAYOFF == kAsian) {
                sf = __builtin_fma(pf, sf2, sf);
                sc = __builtin_fma(pc, sc2, sc);
            }
            if (PAYOFF == kLookback) {
                const double a1 = pf * mf2, a2 = pc * mc2;
                mf = a1 < mf ? a1 : mf;
                mc = a2 < mc ? a2 : mc;
            }
            pf *= pf2;
            pc *= pc2;
        }
    }
    if (seg != 0) return;
    const double S0 = (double)P.S0;
    const float vf = payoff_value<float, PAYOFF>(P, (float)(S0 * pf), (float)(S0 * sf), 0.0f,
                                                 (float)(S0 * mf), P.h);
    const float vc = coupled ? payoff_value<float, PAYOFF>(P, (float)(S0 * pc), (float)(S0 * sc),
                                                           0.0f, (float)(S0 * mc), P.H)
                             : 0.0f;
    if (idx < a.N) accumulate(a, idx, vf, vc, sums, nonfinite);
}

// Levels with n_f = NF in {1, 2}: Q = 4/(NF d) consecutive samples share one
// generator block (d = 1 for GBM, 2 for Heston), as do 4/NF samples one
// bridge block.  A lane takes PPT blocks, i.e. Q * PPT samples; block B of
// the level covers samples Q B .. Q B + Q - 1 (those outside
// [offset, offset + N) are computed and dropped).  blk_base indexes blocks
// from B0 = offset / Q.
//
// Level 0 (NF = 1, no coarse path) is the busiest launch of an adaptive run
// and costs ~25 lane operations per sample, so its bookkeeping is per lane
// chunk rather than per sample: the chunk's sums of y and y^2 go into the
// lane sums at once when every sample of the block's chunk lies in the range
// (`full`, a block-uniform flag from full_chunks) and the fp64 sum of squares
// is finite (y^2 of an fp32 value cannot overflow fp64,
// so that sum is finite exactly when every y is); otherwise the chunk is
// added sample by sample with the range and finiteness checks.  y = P_f
// there: the P_f sums are left to copy_y_sums and the P_c sums stay zero.
// Level 0 of a GBM Euler call in fp32 paths: process_short folds the step into the payoff.
template <int MODEL, int PAYOFF, typename Real, int NF, bool ANTI>
constexpr bool kFusedLevel0 = NF == 1 && MODEL == kGBM && PAYOFF == kCall && !ANTI &&
                              std::is_same<Real, float>::value;

template <int MODEL, int PAYOFF, typename Real, int NF, int M, int PPT, bool ANTI>
__device__ __forceinline__ void process_short(const LevelArgs<Real>& a, uint64_t blk_base, bool full,
                                              double (&sums)[kNumSums], unsigned& nonfinite)
{
    static_assert(!ANTI || (NF == 2 && M == 2), "the twin exists on coupled levels only");
    constexpr int D = one_factor(MODEL) ? 1 : 2;
    constexpr int T = NF * D;             // normals per sample: 1, 2 or 4
    constexpr int Q = 4 / T;              // samples per generator block
    constexpr int QU = 4 / NF;            // samples per bridge block
    const StepParams<Real>& P = a.P;
    const bool coupled = a.coupled && a.l > 0;   // NF == 2 with M == 2 only
    const uint64_t B0 = a.offset / Q;
    uint64_t B[PPT];
    Real pf[PPT][Q], pc[PPT][Q], dwf[PPT][Q];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        B[p] = B0 + blk_base + (uint64_t)p * blockDim.x + threadIdx.x;
        const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
        const u32x4 w = path_block(PathKey{k0, k1, (uint32_t)B[p], a.c2, a.stream}, 0);
        Real dw[4];
        brownian_pair(w.x, w.y, P, dw[0], dw[1]);
        brownian_pair(w.z, w.w, P, dw[2], dw[3]);
        Real e[4] = {Real(0), Real(0), Real(0), Real(0)};
        if (PAYOFF == kLookback) {
            // every sample of this generator block reads bridge block B / D
            const u32x4 u =
                path_block(PathKey{k0, k1, (uint32_t)(B[p] / D), a.c2b, a.stream + 1u}, 0);
            e[0] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.x));
            e[1] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.y));
            e[2] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.z));
            e[3] = P.lnu_scale * flog2<Real>(uniform01<Real>(u.w));
        }
#pragma unroll
        for (int r = 0; r < Q; ++r) {
            if constexpr (kFusedLevel0<MODEL, PAYOFF, Real, NF, ANTI>) {
                // level 0 of a GBM Euler call: the one step and the payoff fold
                // into S_1 - K = (S0 (1 + r T) - K) + S0 sigma dW, one fma
                const Real u = fmaT(P.l0_slope, dw[r], P.l0_base);
                pf[p][r] = fmaT(P.disc, fmaxT(u, Real(0)), u - u);   // u - u: NaN if u overflowed
                pc[p][r] = Real(0);
                dwf[p][r] = dw[r];
                continue;
            }
            const uint64_t s = B[p] * Q + r;
            PathPair<Real> q;
            init_pair<Real, MODEL, PAYOFF>(q, P);
            const int ub = (int)(s % QU) * NF;   // first bridge word of the sample
#pragma unroll
            for (int k = 0; k < NF; ++k) {
                const Real dw1 = dw[r * T + k * D];
                const Real dwp = (D == 2) ? dw[r * T + k * D + 1] : Real(0);
                fine_step<Real, MODEL, PAYOFF>(q, P, dw1, dwp, e[(ub + k) & 3], k % M, coupled);
            }
            if (NF == 2 && coupled) coarse_step<Real, MODEL, PAYOFF>(q, P);
            PathPair<Real> qa;
            if (ANTI) {
                // the twin takes the two increments (and bridge words) swapped
                constexpr bool tc = twin_coarse<PAYOFF>();
                init_pair<Real, MODEL, PAYOFF>(qa, P);
#pragma unroll
                for (int k = 0; k < NF; ++k) {
                    const int j = NF - 1 - k;
                    const Real dw1 = dw[r * T + j * D];
                    const Real dwp = (D == 2) ? dw[r * T + j * D + 1] : Real(0);
                    fine_step<Real, MODEL, PAYOFF>(qa, P, dw1, dwp, e[(ub + j) & 3], k % M, tc);
                }
                if (tc) coarse_step<Real, MODEL, PAYOFF>(qa, P);
            }
            pair_payoffs<MODEL, PAYOFF, Real, ANTI>(P, q, qa, coupled, pf[p][r], pc[p][r]);
            dwf[p][r] = dw[r * T];
        }
    }
    // level 0 with the control variate: every sample starts at (0, S0), so
    // the martingale term is the one value phi(0, S0) times the increment
    if (NF == 1 && a.phi0) {
        const Real c = (Real)*a.phi0;
#pragma unroll
        for (int p = 0; p < PPT; ++p)
#pragma unroll
            for (int r = 0; r < Q; ++r) pf[p][r] = fmaT(-c, dwf[p][r], pf[p][r]);
    }
    if (a.pf_out) {
#pragma unroll
        for (int p = 0; p < PPT; ++p)
#pragma unroll
            for (int r = 0; r < Q; ++r) {
                const uint64_t s = B[p] * Q + r;
                if (s < a.offset || s - a.offset >= a.N) continue;
                a.pf_out[s - a.offset] = (double)pf[p][r];
                a.pc_out[s - a.offset] = (double)pc[p][r];
            }
    }
    if (NF == 1) {
        double cy = (double)pf[0][0];
        double cy2 = cy * cy;
#pragma unroll
        for (int p = 0; p < PPT; ++p)
#pragma unroll
            for (int r = 0; r < Q; ++r) {
                if (p == 0 && r == 0) continue;
                const double y = (double)pf[p][r];
                cy += y;
                cy2 = __builtin_fma(y, y, cy2);
            }
        if (full && isfinite(cy2)) {
            sums[0] += cy;
            sums[1] += cy2;
            return;
        }
    }
#pragma unroll
    for (int p = 0; p < PPT; ++p)
#pragma unroll
        for (int r = 0; r < Q; ++r) {
            const uint64_t s = B[p] * Q + r;
            if (s < a.offset || s - a.offset >= a.N) continue;
            if (NF == 1) add_y((double)pf[p][r], sums, nonfinite);
            else add_sample(pf[p][r], pc[p][r], sums, nonfinite);
        }
}

// Chunks of `chunk` generator blocks (q samples each) of the range
// [offset, offset + N) whose samples all lie in the range: [lo, hi), counted
// from the chunk of block offset / q.  A launch covers generator units that
// share one counter high word, so chunk indices fit 32 bits and the test is
// two scalar compares.
struct FullChunks {
    uint32_t lo, hi;
};
__host__ __device__ inline FullChunks full_chunks(uint64_t offset, uint64_t N, int q, uint64_t chunk)
{
    const uint64_t b0 = offset / (uint64_t)q;
    const uint64_t bend = (offset + N) / (uint64_t)q;   // blocks wholly before the end
    FullChunks f;
    f.lo = b0 * (uint64_t)q == offset ? 0u : 1u;
    f.hi = (uint32_t)((bend - b0) / chunk);
    return f;
}

// Number of generator blocks a short level's range [offset, offset + N) touches.
__host__ __device__ inline uint64_t short_blocks(uint64_t offset, uint64_t N, int q)
{
    if (N == 0) return 0;
    return (offset + N - 1) / q - offset / q + 1;
}

}  // namespace mlmc
