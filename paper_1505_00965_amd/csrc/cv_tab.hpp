// Samplers with the learned control variate read from its table (and the
// increments of a sample's generator group): the device functions of the
// per-level kernels in cv.hip and of the persistent all-levels sampler.
// Each payoff is replaced by P - sum_n phi(t_n, X_n) dW1_n on its own grid,
// fine increments for the fine path and summed coarse ones for the coarse
// path, phi at the left point of each step (Sec. 5, "Exploiting
// Structure"): the level means are unchanged.
#pragma once
#include <hip/hip_runtime.h>

#include "cv.hpp"
#include "sampler_impl.hpp"

namespace mlmc {

using cvnet::TableSpec;
using cvnet::table_phi;

// ------------------------------------------------------- sampler with cv
// Four fine increments of group g of sample s, either from the sample's own
// generator blocks (n_f >= 4) or from a block shared with q - 1 neighbours.
template <int MODEL, int PAYOFF>
__device__ __forceinline__ void fetch_group(const LevelArgs<float>& a, uint64_t s, uint32_t g,
                                            float (&dw1)[4], float (&dwp)[4], float (&e)[4])
{
    const StepParams<float>& P = a.P;
    constexpr int D = (MODEL == kGBM) ? 1 : 2;
    const PathKey key = make_path_key(a.seed, a.l, s, a.stream);
    if (a.nf >= 4) {
        if (MODEL == kGBM) {
            const u32x4 w = path_block(key, g);
            brownian_pair(w.x, w.y, P, dw1[0], dw1[1]);
            brownian_pair(w.z, w.w, P, dw1[2], dw1[3]);
            for (int k = 0; k < 4; ++k) dwp[k] = 0.0f;
        } else {
            const u32x4 wa = path_block(key, 2 * g), wb = path_block(key, 2 * g + 1);
            brownian_pair(wa.x, wa.y, P, dw1[0], dwp[0]);
            brownian_pair(wa.z, wa.w, P, dw1[1], dwp[1]);
            brownian_pair(wb.x, wb.y, P, dw1[2], dwp[2]);
            brownian_pair(wb.z, wb.w, P, dw1[3], dwp[3]);
        }
        if (PAYOFF == kLookback) {
            const u32x4 u = path_block(make_path_key(a.seed, a.l, s, a.stream + 1u), g);
            e[0] = P.lnu_scale * flog2<float>(u01f(u.x));
            e[1] = P.lnu_scale * flog2<float>(u01f(u.y));
            e[2] = P.lnu_scale * flog2<float>(u01f(u.z));
            e[3] = P.lnu_scale * flog2<float>(u01f(u.w));
        }
        return;
    }
    const int T = a.nf * D, q = 4 / T;
    const u32x4 w = path_block(make_path_key(a.seed, a.l, s / q, a.stream), 0);
    float z[4];
    brownian_pair(w.x, w.y, P, z[0], z[1]);
    brownian_pair(w.z, w.w, P, z[2], z[3]);
    const int base = (int)(s % q) * T;
    for (int k = 0; k < 4; ++k) {
        const int i1 = (base + k * D) & 3, i2 = (base + k * D + 1) & 3;
        const float z1 = i1 == 0 ? z[0] : i1 == 1 ? z[1] : i1 == 2 ? z[2] : z[3];
        const float z2 = i2 == 0 ? z[0] : i2 == 1 ? z[1] : i2 == 2 ? z[2] : z[3];
        dw1[k] = z1;
        dwp[k] = D == 2 ? z2 : 0.0f;
    }
    if (PAYOFF == kLookback) {
        const int qu = 4 / a.nf;
        const u32x4 u = path_block(make_path_key(a.seed, a.l, s / qu, a.stream + 1u), 0);
        const int ub = (int)(s % qu) * a.nf;
        for (int k = 0; k < 4; ++k) {
            const int iw = (ub + k) & 3;
            const uint32_t word = iw == 0 ? u.x : iw == 1 ? u.y : iw == 2 ? u.z : u.w;
            e[k] = P.lnu_scale * flog2<float>(u01f(word));
        }
    }
}

// ------------------------------------------------- sampler with the table
// The rows of the table a level reads, in LDS: lr = min(n_f, rows) rows, LDS
// row r being table row r rows / lr; step n of the level reads LDS row
// floor(n lr / n_f), i.e. table row floor(n rows / n_f).
struct TabView {
    const float* tab;
    TableSpec t;
    int lr, nf;
};

__device__ __forceinline__ int tab_row(const TabView& v, int n)
{
    return (int)(((unsigned)n * (unsigned)v.lr) / (unsigned)v.nf);
}

// Copy the level's rows into s_tab and describe them.
__device__ __forceinline__ TabView load_level_table(float* s_tab, const float* table,
                                                    const TableSpec& t, int nf)
{
    const int lr = nf < t.rows ? nf : t.rows;
    const int rstep = t.rows / lr, rowlen4 = t.ns * t.nv / 4;   // rows hold whole float4s
    const float4* src = reinterpret_cast<const float4*>(table);
    float4* dst = reinterpret_cast<float4*>(s_tab);
    // unrolled so that a thread's loads are in flight together (one L2
    // round trip for the whole copy, not one per element)
#pragma unroll 8
    for (int i = threadIdx.x; i < lr * rowlen4; i += blockDim.x) {
        const int r = i / rowlen4, c = i - r * rowlen4;
        dst[i] = src[r * rstep * rowlen4 + c];
    }
    __syncthreads();
    return TabView{s_tab, t, lr, nf};
}

// Generator block g (four fine steps) of a coupled pair with the tabulated
// control variate: the steps as in advance_group, then phi at the left point
// of each of the four fine steps and of each coarse step the block opens,
// read in one go (the lookups wait on LDS once per block, not once per step)
// and added to the pair's sums in step order.
template <int MODEL, int PAYOFF, int M>
__device__ __forceinline__ void advance_group_tab(const StepParams<float>& P, const PathKey& key,
                                                  const PathKey& bkey, uint32_t g, PathPair<float>& q,
                                                  const TabView& tv)
{
    float dw1[4], dwp[4], e[4];
    if (one_factor(MODEL)) {
        const u32x4 w = path_block(key, g);
        brownian_pair(w.x, w.y, P, dw1[0], dw1[1]);
        brownian_pair(w.z, w.w, P, dw1[2], dw1[3]);
        dwp[0] = dwp[1] = dwp[2] = dwp[3] = 0.0f;
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
        e[0] = P.lnu_scale * flog2<float>(u01f(u.x));
        e[1] = P.lnu_scale * flog2<float>(u01f(u.y));
        e[2] = P.lnu_scale * flog2<float>(u01f(u.z));
        e[3] = P.lnu_scale * flog2<float>(u01f(u.w));
    } else {
        e[0] = e[1] = e[2] = e[3] = 0.0f;
    }
    constexpr int NC = 4 / M;
    float sf[4], vf[4], sc[NC], vc[NC], wc[NC];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        sf[k] = q.S;
        vf[k] = q.v;
        if (k % M == 0) {
            sc[k / M] = q.Sc;
            vc[k / M] = q.vc;
        }
        fine_step<float, MODEL, PAYOFF>(q, P, dw1[k], dwp[k], e[k], k % M, true);
        if ((k + 1) % M == 0) {
            wc[k / M] = q.dw1c;
            coarse_step<float, MODEL, PAYOFF>(q, P);
        }
    }
    const int n0 = 4 * (int)g;
    float pf[4], pcs[NC];
#pragma unroll
    for (int k = 0; k < 4; ++k) pf[k] = table_phi(tv.tab, tv.t, tab_row(tv, n0 + k), sf[k], vf[k]);
#pragma unroll
    for (int c = 0; c < NC; ++c) pcs[c] = table_phi(tv.tab, tv.t, tab_row(tv, n0 + c * M), sc[c], vc[c]);
#pragma unroll
    for (int k = 0; k < 4; ++k) q.cvf = __builtin_fmaf(pf[k], dw1[k], q.cvf);
#pragma unroll
    for (int c = 0; c < NC; ++c) q.cvc = __builtin_fmaf(pcs[c], wc[c], q.cvc);
}

// One chunk of blockDim x PPT samples from index `base` (levels with
// n_f >= 4): PPT samples per lane, each advanced group by group with the
// table's control-variate terms, then payoffs into the lane sums.
template <int MODEL, int PAYOFF, int M, int PPT>
__device__ __forceinline__ void process_chunk_tab(const LevelArgs<float>& a, uint64_t base,
                                                  const TabView& tv, double (&sums)[kNumSums],
                                                  unsigned& nonfinite)
{
    const StepParams<float>& P = a.P;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    uint64_t idx[PPT];
    PathKey key[PPT], bkey[PPT];
    PathPair<float> q[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        idx[p] = base + (uint64_t)p * blockDim.x + threadIdx.x;
        const uint32_t s = (uint32_t)(a.offset + idx[p]);
        key[p] = PathKey{k0, k1, s, a.c2, a.stream};
        bkey[p] = PathKey{k0, k1, s, a.c2b, a.stream + 1u};
        init_pair<float, MODEL, PAYOFF>(q[p], P);
    }
    for (uint32_t g = 0; g < a.ngroups; ++g) {
#pragma unroll
        for (int p = 0; p < PPT; ++p)
            advance_group_tab<MODEL, PAYOFF, M>(P, key[p], bkey[p], g, q[p], tv);
    }
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const float pf = payoff_value<float, PAYOFF>(P, q[p].S, q[p].asum, q[p].acomp, q[p].mn, P.h) -
                         q[p].cvf;
        const float pc =
            payoff_value<float, PAYOFF>(P, q[p].Sc, q[p].csum, q[p].ccomp, q[p].mnc, P.H) - q[p].cvc;
        if (idx[p] < a.N) accumulate(a, idx[p], pf, pc, sums, nonfinite);
    }
}

// GBM levels whose paths are too few to fill the device: G = a.split lanes
// per path.  Pass 1 is process_split's: every lane runs its segment of n_f/G
// fine steps from a unit start and the segment summaries (product, sum of S,
// bridge minimum; fine and coarse) are composed, here by an inclusive scan in
// path order, so lane j also learns the product of the segments before it,
// i.e. its segment's true start.  Pass 2: each lane runs its segment again
// from that start (the same generator blocks) for the control-variate terms;
// their sums over the path's lanes complete the two control-variate sums,
// and the last lane forms the payoffs.
template <int PAYOFF, int M>
__device__ __forceinline__ void process_split_tab(const LevelArgs<float>& a, uint64_t base,
                                                  const TabView& tv, double (&sums)[kNumSums],
                                                  unsigned& nonfinite)
{
    const int G = (int)a.split;
    const int seg = (int)threadIdx.x & (G - 1);
    const uint64_t idx = base + threadIdx.x / (uint32_t)G;
    const uint64_t s = a.offset + idx;
    const StepParams<float>& P = a.P;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const PathKey key{k0, k1, (uint32_t)s, a.c2, a.stream};
    const PathKey bkey{k0, k1, (uint32_t)s, a.c2b, a.stream + 1u};
    PathPair<float> q, qa;
    init_pair<float, kGBM, PAYOFF>(q, P);
    q.S = 1.0f;
    q.Sc = 1.0f;
    const uint32_t per = a.ngroups / (uint32_t)G;
    const uint32_t g0 = (uint32_t)seg * per;
    for (uint32_t g = g0; g < g0 + per; ++g)
        advance_group<kGBM, PAYOFF, float, M, false>(P, key, bkey, g, q, qa);
    double pf = q.S, sf = (double)q.asum - (double)q.acomp, mf = q.mn;
    double pc = q.Sc, sc = (double)q.csum - (double)q.ccomp, mc = q.mnc;
    // inclusive scan: lane j holds the composition of segments 0..j
    for (int off = 1; off < G; off <<= 1) {
        const double pf2 = __shfl_up(pf, off, G), pc2 = __shfl_up(pc, off, G);
        double sf2 = 0, sc2 = 0, mf2 = 0, mc2 = 0;
        if (PAYOFF == kAsian) {
            sf2 = __shfl_up(sf, off, G);
            sc2 = __shfl_up(sc, off, G);
        }
        if (PAYOFF == kLookback) {
            mf2 = __shfl_up(mf, off, G);
            mc2 = __shfl_up(mc, off, G);
        }
        if (seg >= off) {      // (earlier segments) o (this one)
            if (PAYOFF == kAsian) {
                sf = __builtin_fma(pf2, sf, sf2);
                sc = __builtin_fma(pc2, sc, sc2);
            }
            if (PAYOFF == kLookback) {
                const double a1 = pf2 * mf, a2 = pc2 * mc;
                mf = a1 < mf2 ? a1 : mf2;
                mc = a2 < mc2 ? a2 : mc2;
            }
            pf *= pf2;
            pc *= pc2;
        }
    }
    // start of this lane's segment: the product of the segments before it
    const double before_f = __shfl_up(pf, 1, G), before_c = __shfl_up(pc, 1, G);
    const double S0 = (double)P.S0;
    PathPair<float> r;
    init_pair<float, kGBM, kCall>(r, P);
    r.S = (float)(S0 * (seg ? before_f : 1.0));
    r.Sc = (float)(S0 * (seg ? before_c : 1.0));
    for (uint32_t g = g0; g < g0 + per; ++g) advance_group_tab<kGBM, kCall, M>(P, key, bkey, g, r, tv);
    double cf = r.cvf, cc = r.cvc;
    for (int off = 1; off < G; off <<= 1) {
        cf += __shfl_xor(cf, off, G);
        cc += __shfl_xor(cc, off, G);
    }
    if (seg != G - 1) return;
    const float vf = payoff_value<float, PAYOFF>(P, (float)(S0 * pf), (float)(S0 * sf), 0.0f,
                                                 (float)(S0 * mf), P.h) - (float)cf;
    const float vc = payoff_value<float, PAYOFF>(P, (float)(S0 * pc), (float)(S0 * sc), 0.0f,
                                                 (float)(S0 * mc), P.H) - (float)cc;
    if (idx < a.N) accumulate(a, idx, vf, vc, sums, nonfinite);
}

// One chunk of blockDim samples from index `base` on a level with n_f < 4
// (level 1 at M = 2): samples share generator blocks (fetch_group), one
// sample per lane.
template <int MODEL, int PAYOFF, int M>
__device__ __forceinline__ void process_short_tab(const LevelArgs<float>& a, uint64_t base,
                                                  const TabView& tv, double (&sums)[kNumSums],
                                                  unsigned& nonfinite)
{
    const StepParams<float>& P = a.P;
    const uint64_t idx = base + threadIdx.x;
    const uint64_t s = a.offset + idx;
    PathPair<float> q;
    init_pair<float, MODEL, PAYOFF>(q, P);
    float phic = 0.0f;
    float dw1[4], dwp[4], e[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    fetch_group<MODEL, PAYOFF>(a, s, 0, dw1, dwp, e);
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        if (n >= a.nf) break;
        const int row = tab_row(tv, n);
        q.cvf = __builtin_fmaf(table_phi(tv.tab, tv.t, row, q.S, q.v), dw1[n], q.cvf);
        if ((n & (M - 1)) == 0) phic = table_phi(tv.tab, tv.t, row, q.Sc, q.vc);
        fine_step<float, MODEL, PAYOFF>(q, P, dw1[n], dwp[n], e[n], n & (M - 1), true);
        if (((n + 1) & (M - 1)) == 0) {
            q.cvc = __builtin_fmaf(phic, q.dw1c, q.cvc);
            coarse_step<float, MODEL, PAYOFF>(q, P);
        }
    }
    const float pf = payoff_value<float, PAYOFF>(P, q.S, q.asum, q.acomp, q.mn, P.h) - q.cvf;
    const float pc = payoff_value<float, PAYOFF>(P, q.Sc, q.csum, q.ccomp, q.mnc, P.H) - q.cvc;
    if (idx < a.N) accumulate(a, idx, pf, pc, sums, nonfinite);
}

// Host (cv.hip): the tabulated control variate's table for model m on
// stream st (built, with phi(0, S0) from it, if the parameters, the model or
// the stream changed), its grid, phi(0, S0), and the LDS bytes of the rows a
// level of max_nf fine steps reads (the most any level up to it reads).
hipError_t cv_table_view(const mlmc_cv* cv, const mlmc_model& m, hipStream_t st, int max_nf,
                         const float** table, TableSpec* spec, const float** phi0,
                         size_t* lds_bytes);

}  // namespace mlmc
