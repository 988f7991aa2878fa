// Learned control variate: parameters, the sampler with the control variate
// (forward), the training backward pass, and Adam -- all device kernels.
//
// Level estimators with the control variate (eqs. (eq:mlmc:Yzero),
// (eq:Yldef) with each payoff replaced by P - sum_n phi(t_n, X_n) dW1_n on
// its own grid): the fine path uses its fine increments, the coarse path its
// coarse (summed) increments, both evaluated at the left point of each step.
// At t = 0 every sample sits at (0, S0), so level 0 needs only the one value
// phi(0, S0), computed once per launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "context.hpp"
#include "cv.hpp"
#include "cv_tab.hpp"
#include "sampler_impl.hpp"
#include "trace.hpp"

using namespace mlmc::cvnet;

struct mlmc_cv {
    mlmc_ctx* ctx = nullptr;
    int D = 2;                    // network inputs
    int np = 0;                   // parameter count
    float* d_params = nullptr;    // fp32 master
    float* d_m1 = nullptr;        // Adam moments
    float* d_m2 = nullptr;
    bf16x8* d_afwd = nullptr;     // bf16 W2 operands (forward), 8 x 64 entries
    bf16x8* d_abwd = nullptr;     // bf16 W2 operands (backward, permuted)
    float* d_phi0 = nullptr;      // [0] phi(0, S0), [1] its tabulated value: see cv_ensure_phi0
    int adam_t = 0;
    uint64_t version = 0;         // bumped by every parameter change
    uint64_t phi0_version[2] = {~0ull, ~0ull};
    mlmc_model phi0_model[2]{};
    hipStream_t phi0_stream[2] = {nullptr, nullptr};
    // tabulated network (estimation launches only; training evaluates it)
    int tabulated = 0;
    float* d_table = nullptr;
    size_t table_cap = 0;         // floats allocated
    uint64_t table_version = ~0ull;
    mlmc_model table_model{};
    hipStream_t table_stream = nullptr;
    // training scratch
    float* d_gpart = nullptr;     // per-block gradient partials
    int gpart_blocks = 0;
    double* d_y = nullptr;        // per-sample Y of a training batch (all levels)
    float* d_w = nullptr;         // per-sample loss weights
    double* d_loss = nullptr;     // loss and per-level variances
    uint64_t batch_cap = 0;
    float* d_fpart = nullptr;     // forward runs' partial sums of one level
    uint64_t fpart_cap = 0;       // floats allocated
};

namespace mlmc {

// ------------------------------------------------------------ parameters
// Xavier-uniform weights from the init stream: parameter i takes word i % 4
// of generator block i / 4 at (sample 0, level 0); biases zero.
__global__ void cv_init_kernel(float* params, int D, uint64_t seed)
{
    const int np = nparams(D);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    float a = 0.0f;
    if (i < off_b1(D)) a = sqrtf(6.0f / (float)(D + H));
    else if (i >= off_W2(D) && i < off_b2(D)) a = sqrtf(6.0f / (float)(2 * H));
    else if (i >= off_w3(D) && i < off_b3(D)) a = sqrtf(6.0f / (float)(H + 1));
    if (a == 0.0f) {
        params[i] = 0.0f;
        return;
    }
    const u32x4 w = path_block(make_path_key(seed, 0, 0, kStreamInit), (uint32_t)(i / 4));
    const uint32_t word = (i % 4 == 0) ? w.x : (i % 4 == 1) ? w.y : (i % 4 == 2) ? w.z : w.w;
    params[i] = a * (2.0f * (float)u01d(word) - 1.0f);
}

// Row of the permuted backward operand: physical row rho of e1 = W2^T d2
// holds logical unit unit_of_row(rho), chosen so that e1's accumulator
// registers line up with the forward pass's layer-1 slots (unit_b).
__host__ __device__ inline int unit_of_row(int rho)
{
    const int kt = rho / 32, rem = rho % 32;
    const int h = (rem % 8) / 4;
    const int r = 4 * (rem / 8) + rem % 4;
    return 32 * kt + 16 * (r / 8) + 8 * h + r % 8;
}

// Contraction position kappa of e1's B operand (d2 straight from the layer-2
// accumulators) holds logical output unit j_of_pos(kappa).
__host__ __device__ inline int j_of_pos(int kappa)
{
    const int kb = kappa / 16, rem = kappa % 16;
    const int h = rem / 8, i = rem % 8;
    const int t = 8 * kb + i;            // register order within the half
    return row_d(h, t / 16, t % 16);
}

// bf16 operand arrays from the fp32 W2 (round to nearest even).
__global__ void cv_prepare_kernel(const float* params, int D, bf16x8* afwd, bf16x8* abwd)
{
    const float* W2 = params + off_W2(D);
    const int t = threadIdx.x;            // 64 lanes x 8 operand sets
    for (int idx = t; idx < 8 * 64; idx += blockDim.x) {
        const int set = idx / 64, lane = idx % 64;
        const int hi = lane / 32;
        const int tile = set / 4, kb = set % 4;
        bf16x8 f, b;
        for (int i = 0; i < 8; ++i) {
            const int j = 32 * tile + lane % 32, k = 16 * kb + 8 * hi + i;
            f[i] = (__bf16)W2[j * H + k];
            // backward: row rho = 32 tile + lane % 32, position kappa = k
            const int rho = 32 * tile + lane % 32;
            b[i] = (__bf16)W2[j_of_pos(k) * H + unit_of_row(rho)];
        }
        afwd[idx] = f;
        abwd[idx] = b;
    }
}

struct CvKernelArgs {
    const float* params;
    const bf16x8* afwd;
    NetConsts nc;
    int D;
};

// Grid of the tabulated network for a model (host): 256 time rows x 32 stock
// values for GBM; 16 rows x 16 stock values x 32 variances for Heston (32 KiB
// of fp32 either way; a level's sampler copies the rows it reads into LDS).
// Stock values span S0 exp(+-4 sref sqrt T) (sref = sigma, or sqrt(theta) for
// Heston), variances [0, 4 max(theta, v0)].  The network varies slowly in S
// at these scales; Heston's variance axis and the time rows of deep levels
// decide how much of its variance reduction the table keeps.
struct TableGrid {
    int rows, ns, nv;
    double s_lo, s_hi, v_lo, v_hi;
};

static TableGrid table_grid(const mlmc_model& m)
{
    TableGrid g;
    const bool heston = m.kind == MLMC_HESTON;
    const double sref = heston ? std::sqrt(m.theta) : m.sigma;
    const double w = 4.0 * sref * std::sqrt(m.T);
    g.rows = heston ? 16 : 256;
    g.ns = heston ? 16 : 32;
    g.nv = heston ? 32 : 1;
    g.s_lo = m.S0 * std::exp(-w);
    g.s_hi = m.S0 * std::exp(w);
    g.v_lo = 0.0;
    g.v_hi = heston ? 4.0 * std::max(m.theta, m.v0) : 1.0;
    return g;
}

static TableSpec table_spec(const TableGrid& g)
{
    TableSpec t;
    t.rows = g.rows;
    t.ns = g.ns;
    t.nv = g.nv;
    t.s_lo = (float)g.s_lo;
    t.s_inv = (float)((g.ns - 1) / (g.s_hi - g.s_lo));
    t.v_lo = (float)g.v_lo;
    t.v_inv = g.nv > 1 ? (float)((g.nv - 1) / (g.v_hi - g.v_lo)) : 0.0f;
    return t;
}

static size_t table_size(const TableGrid& g) { return (size_t)g.rows * g.ns * g.nv; }

// Fill the table: point p = (row j, variance k, stock i), p = (j nv + k) ns + i,
// holds phi(j T / rows, S_i, v_k) from the network (64 points per wave
// through phi_eval; every lane of a wave evaluates, lanes past the end drop
// their value).
template <int D>
__global__ void cv_table_kernel(CvKernelArgs c, TableGrid g, float* tab)
{
    __shared__ NetShared sh;
    __shared__ bf16x8 s_afwd[8 * 64];
    load_shared<D>(sh, c.params, c.nc);
    for (int i = threadIdx.x; i < 8 * 64; i += blockDim.x) s_afwd[i] = c.afwd[i];
    __syncthreads();
    const int npts = g.rows * g.nv * g.ns;
    const double ds = (g.s_hi - g.s_lo) / (g.ns - 1);
    const double dv = g.nv > 1 ? (g.v_hi - g.v_lo) / (g.nv - 1) : 0.0;
    for (int base = blockIdx.x * blockDim.x; base < npts; base += gridDim.x * blockDim.x) {
        const int p = min(base + (int)threadIdx.x, npts - 1);
        const int i = p % g.ns, jk = p / g.ns;
        const int k = jk % g.nv, j = jk / g.nv;
        const float S = (float)(g.s_lo + i * ds);
        const float v = (float)(g.v_lo + k * dv);
        const float x0 = (float)j / (float)g.rows;
        // a wave may span two time rows: every lane brings its own time
        const float phi = phi_eval<D, true>(sh, s_afwd, x0, S, v);
        if (base + (int)threadIdx.x < npts) tab[p] = phi;
    }
}

// phi at (0, S0, v0) read from the table (level 0 of the tabulated form).
__global__ void cv_table_point_kernel(const float* tab, TableSpec t, float S0, float v0, float* out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = table_phi(tab, t, 0, S0, v0);
}

template <int D>
__global__ void cv_phi0_kernel(CvKernelArgs c, float S0, float v0, float* out)
{
    __shared__ NetShared sh;
    load_shared<D>(sh, c.params, c.nc);
    __syncthreads();
    const float phi = phi_eval<D>(sh, c.afwd, 0.0f, S0, v0);
    if (threadIdx.x == 0) *out = phi;
}

// One sample per lane; every lane runs every network evaluation (samples
// past the range are simulated and dropped), so waves stay converged.  Two
// blocks per compute unit (two waves per SIMD): with the network constants
// and W2 operands read from LDS per evaluation the kernel fits 256 registers
// per lane without spilling, and the second wave hides the matrix-core and
// transcendental latencies of the first.
template <int MODEL, int PAYOFF, int M>
__global__ __launch_bounds__(256, 2) void cv_level_kernel(LevelArgs<float> a, CvKernelArgs c)
{
    constexpr int D = (MODEL == kGBM) ? 2 : 3;
    __shared__ NetShared sh;
    __shared__ bf16x8 s_afwd[8 * 64];   // W2 operands, read at every evaluation
    load_shared<D>(sh, c.params, c.nc);
    for (int i = threadIdx.x; i < 8 * 64; i += blockDim.x) s_afwd[i] = c.afwd[i];
    __syncthreads();
    const StepParams<float>& P = a.P;
    const bool coupled = a.coupled && a.l > 0;
    double sums[kNumSums] = {0, 0, 0, 0, 0, 0};
    unsigned nonfinite = 0;
    const uint64_t nchunks = (a.N + blockDim.x - 1) / blockDim.x;
    for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const uint64_t idx = ch * blockDim.x + threadIdx.x;
        const uint64_t s = a.offset + idx;
        PathPair<float> q;
        init_pair<float, MODEL, PAYOFF>(q, P);
        float phic = 0.0f;
        for (uint32_t g = 0; g < a.ngroups; ++g) {
            float dw1[4], dwp[4], e[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            fetch_group<MODEL, PAYOFF>(a, s, g, dw1, dwp, e);
            // not unrolled: one copy of each network evaluation in the code
#pragma unroll 1
            for (int k = 0; k < 4; ++k) {
                const int n = 4 * (int)g + k;
                if (n >= a.nf) break;                       // wave-uniform
                const float d1 = k == 0 ? dw1[0] : k == 1 ? dw1[1] : k == 2 ? dw1[2] : dw1[3];
                const float dp = k == 0 ? dwp[0] : k == 1 ? dwp[1] : k == 2 ? dwp[2] : dwp[3];
                const float ek = k == 0 ? e[0] : k == 1 ? e[1] : k == 2 ? e[2] : e[3];
                const float x0 = (float)n * P.h * sh.inv_T;
                const float phif = phi_eval<D>(sh, s_afwd, x0, q.S, q.v);
                q.cvf = __builtin_fmaf(phif, d1, q.cvf);
                if (coupled && (n & (M - 1)) == 0) phic = phi_eval<D>(sh, s_afwd, x0, q.Sc, q.vc);
                fine_step<float, MODEL, PAYOFF>(q, P, d1, dp, ek, n & (M - 1), coupled);
                if (coupled && ((n + 1) & (M - 1)) == 0) {
                    q.cvc = __builtin_fmaf(phic, q.dw1c, q.cvc);
                    coarse_step<float, MODEL, PAYOFF>(q, P);
                }
            }
        }
        const float pf = payoff_value<float, PAYOFF>(P, q.S, q.asum, q.acomp, q.mn, P.h) - q.cvf;
        const float pc = coupled
                             ? payoff_value<float, PAYOFF>(P, q.Sc, q.csum, q.ccomp, q.mnc, P.H) - q.cvc
                             : 0.0f;
        if (idx < a.N) accumulate(a, idx, pf, pc, sums, nonfinite);
    }
    block_reduce_add(sums, nonfinite, a.acc + (blockIdx.x & a.spread_mask));
}

// Levels with n_f >= 4: PPT samples per lane, blocks walk the chunks.
template <int MODEL, int PAYOFF, int M, int PPT>
__global__ __launch_bounds__(256) void cv_tab_level_kernel(LevelArgs<float> a, const float* table,
                                                           TableSpec t)
{
    extern __shared__ __attribute__((aligned(16))) float s_tab[];
    const TabView tv = load_level_table(s_tab, table, t, a.nf);
    double sums[kNumSums] = {0, 0, 0, 0, 0, 0};
    unsigned nonfinite = 0;
    const uint64_t chunk = (uint64_t)blockDim.x * PPT;
    const uint64_t nchunks = (a.N + chunk - 1) / chunk;
    for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x)
        process_chunk_tab<MODEL, PAYOFF, M, PPT>(a, ch * chunk, tv, sums, nonfinite);
    block_reduce_add(sums, nonfinite, a.acc + (blockIdx.x & a.spread_mask));
}

template <int PAYOFF, int M>
__global__ __launch_bounds__(256) void cv_tab_split_kernel(LevelArgs<float> a, const float* table,
                                                           TableSpec t)
{
    extern __shared__ __attribute__((aligned(16))) float s_tab[];
    const TabView tv = load_level_table(s_tab, table, t, a.nf);
    double sums[kNumSums] = {0, 0, 0, 0, 0, 0};
    unsigned nonfinite = 0;
    const uint64_t per_block = blockDim.x / a.split;
    const uint64_t nchunks = (a.N + per_block - 1) / per_block;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x)
        process_split_tab<PAYOFF, M>(a, c * per_block, tv, sums, nonfinite);
    block_reduce_add(sums, nonfinite, a.acc + (blockIdx.x & a.spread_mask));
}

// Levels with n_f < 4 (level 1 at M = 2): one sample per lane, the level's
// table rows in LDS.
template <int MODEL, int PAYOFF, int M>
__global__ __launch_bounds__(256) void cv_tab_short_kernel(LevelArgs<float> a, const float* table,
                                                           TableSpec t)
{
    extern __shared__ __attribute__((aligned(16))) float s_tab[];
    const TabView tv = load_level_table(s_tab, table, t, a.nf);
    double sums[kNumSums] = {0, 0, 0, 0, 0, 0};
    unsigned nonfinite = 0;
    const uint64_t nchunks = (a.N + blockDim.x - 1) / blockDim.x;
    for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x)
        process_short_tab<MODEL, PAYOFF, M>(a, ch * blockDim.x, tv, sums, nonfinite);
    block_reduce_add(sums, nonfinite, a.acc + (blockIdx.x & a.spread_mask));
}

// Training forward of a deep level in runs (as the backward pass cuts it):
// block (64 samples, run r) advances its paths from the start, evaluates
// the network at the points of its run only, and writes its fp32 sums of
// phi dW1 on the fine and the coarse path to part[2r][i], part[2r+1][i];
// the last run also writes the two payoffs to part[2 segs], part[2 segs + 1].
// cv_train_combine_kernel then forms Y (payoff minus the runs' sums, added
// in run order), the per-sample dumps and the level sums.
template <int MODEL, int PAYOFF, int M>
__global__ __launch_bounds__(64) void cv_train_fwd_kernel(LevelArgs<float> a, CvKernelArgs c, uint32_t segs,
                                                          float* part)
{
    constexpr int D = (MODEL == kGBM) ? 2 : 3;
    __shared__ NetShared sh;
    __shared__ bf16x8 s_afwd[8 * 64];
    load_shared<D>(sh, c.params, c.nc);
    for (int i = threadIdx.x; i < 8 * 64; i += blockDim.x) s_afwd[i] = c.afwd[i];
    __syncthreads();
    const StepParams<float>& P = a.P;
    const uint64_t nchunks = (a.N + 63) / 64;
    const uint32_t per_seg = a.ngroups / segs;      // segs divides ngroups (host)
    for (uint64_t b = blockIdx.x; b < nchunks * segs; b += gridDim.x) {
        const uint64_t ch = b / segs;
        const uint32_t r = (uint32_t)(b % segs), g0 = r * per_seg, g1 = g0 + per_seg;
        const uint64_t idx = ch * 64 + threadIdx.x;
        const uint64_t s = a.offset + idx;
        PathPair<float> q;
        init_pair<float, MODEL, PAYOFF>(q, P);
        float phic = 0.0f;
        for (uint32_t g = 0; g < g1; ++g) {
            float dw1[4], dwp[4], e[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            fetch_group<MODEL, PAYOFF>(a, s, g, dw1, dwp, e);
            const bool eval = g >= g0;                      // block-uniform
#pragma unroll 1
            for (int k = 0; k < 4; ++k) {
                const int n = 4 * (int)g + k;
                if (n >= a.nf) break;                       // wave-uniform
                const float d1 = k == 0 ? dw1[0] : k == 1 ? dw1[1] : k == 2 ? dw1[2] : dw1[3];
                const float dp = k == 0 ? dwp[0] : k == 1 ? dwp[1] : k == 2 ? dwp[2] : dwp[3];
                const float ek = k == 0 ? e[0] : k == 1 ? e[1] : k == 2 ? e[2] : e[3];
                if (eval) {
                    const float x0 = (float)n * P.h * sh.inv_T;
                    const float phif = phi_eval<D>(sh, s_afwd, x0, q.S, q.v);
                    q.cvf = __builtin_fmaf(phif, d1, q.cvf);
                    if ((n & (M - 1)) == 0) phic = phi_eval<D>(sh, s_afwd, x0, q.Sc, q.vc);
                }
                fine_step<float, MODEL, PAYOFF>(q, P, d1, dp, ek, n & (M - 1), true);
                if (((n + 1) & (M - 1)) == 0) {
                    if (eval) q.cvc = __builtin_fmaf(phic, q.dw1c, q.cvc);
                    coarse_step<float, MODEL, PAYOFF>(q, P);
                }
            }
        }
        if (idx < a.N) {
            part[(uint64_t)(2 * r) * a.N + idx] = q.cvf;
            part[(uint64_t)(2 * r + 1) * a.N + idx] = q.cvc;
            if (r + 1 == segs) {
                part[(uint64_t)(2 * segs) * a.N + idx] =
                    payoff_value<float, PAYOFF>(P, q.S, q.asum, q.acomp, q.mn, P.h);
                part[(uint64_t)(2 * segs + 1) * a.N + idx] =
                    payoff_value<float, PAYOFF>(P, q.Sc, q.csum, q.ccomp, q.mnc, P.H);
            }
        }
    }
}

__global__ __launch_bounds__(256) void cv_train_combine_kernel(LevelArgs<float> a, uint32_t segs,
                                                               const float* part)
{
    double sums[kNumSums] = {0, 0, 0, 0, 0, 0};
    unsigned nonfinite = 0;
    for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < a.N;
         idx += (uint64_t)gridDim.x * blockDim.x) {
        float cf = 0.0f, cc = 0.0f;
        for (uint32_t r = 0; r < segs; ++r) {
            cf += part[(uint64_t)(2 * r) * a.N + idx];
            cc += part[(uint64_t)(2 * r + 1) * a.N + idx];
        }
        const float pf = part[(uint64_t)(2 * segs) * a.N + idx] - cf;
        const float pc = part[(uint64_t)(2 * segs + 1) * a.N + idx] - cc;
        accumulate(a, idx, pf, pc, sums, nonfinite);
    }
    block_reduce_add(sums, nonfinite, a.acc);
}

// ------------------------------------------------------------ training
// Loss over levels 0..lmax (the MLMC cost functional; total cost scales as
// (sum_l sqrt(V_l C_l))^2):  loss = sum_l sqrt(C_l Var_batch(Y_l)),
// dLoss/dY_i = sqrt(C_l / V_l) (Y_i - mean_l) / (B - 1).
// One block per level: weights of every sample, the level's variance, and
// its loss term (added into loss[0]).
__global__ void cv_weights_kernel(const LevelAcc* rec, const double* ydump, uint64_t B, int M,
                                  float* w, double* loss)
{
    const int l = blockIdx.x;
    const double n = (double)B;
    const double mean = rec[l].sum[0] / n;
    double var = (rec[l].sum[1] - n * mean * mean) / (n - 1.0);
    if (var < 0) var = 0;
    double C = 1.0;
    if (l > 0) {
        double a = 1.0;
        for (int i = 0; i < l - 1; ++i) a *= M;
        C = a * M + a;
    }
    const double scale = var > 0 ? sqrt(C / var) / (n - 1.0) : 0.0;
    const double* pf = ydump + 2 * (uint64_t)l * B;
    const double* pc = pf + B;
    for (uint64_t i = threadIdx.x; i < B; i += blockDim.x)
        w[(uint64_t)l * B + i] = (float)(scale * ((pf[i] - pc[i]) - mean));
    if (threadIdx.x == 0) {
        loss[1 + l] = var;
        atomicAdd(&loss[0], sqrt(C * var));
    }
}

// Backward pass over the samples of one level (one wave per block): the
// same paths as the forward pass, regenerated from their counters; every
// evaluation point contributes with g = -w dW1 (fine) or +w dW1c (coarse).
// A path's generator groups are cut into `segs` runs of whole groups, one
// block per (64 samples, run): a block advances its paths from the start
// (a plain step costs ~20 instructions, an evaluation point with its
// backward pass thousands) and evaluates only the points of its run, so a
// deep level's few samples still fill the device.
template <int MODEL, int PAYOFF, int M>
__global__ __launch_bounds__(64) void cv_backward_kernel(LevelArgs<float> a, CvKernelArgs c,
                                                          const bf16x8* abwd, const float* w,
                                                          float* gpart, uint32_t segs)
{
    constexpr int D = (MODEL == kGBM) ? 2 : 3;
    __shared__ NetShared sh;
    __shared__ bf16x8 afw[8 * 64], abw[8 * 64];
    __shared__ Stage st;
    load_shared<D>(sh, c.params, c.nc);
    for (int i = threadIdx.x; i < 8 * 64; i += blockDim.x) {
        afw[i] = c.afwd[i];
        abw[i] = abwd[i];
    }
    __syncthreads();
    GradAcc acc;
    zero_acc(acc);
    const StepParams<float>& P = a.P;
    const bool coupled = a.l > 0;
    const int lane = threadIdx.x & 63;
    const uint64_t nchunks = (a.N + 63) / 64;
    const uint32_t per_seg = a.ngroups / segs;      // segs divides ngroups (host)
    for (uint64_t b = blockIdx.x; b < nchunks * segs; b += gridDim.x) {
        const uint64_t ch = b / segs;
        const uint32_t g0 = (uint32_t)(b % segs) * per_seg, g1 = g0 + per_seg;
        const uint64_t idx = ch * 64 + lane;
        const uint64_t s = a.offset + idx;
        const float wp = idx < a.N ? w[idx] : 0.0f;
        PathPair<float> q;
        init_pair<float, MODEL, PAYOFF>(q, P);
        for (uint32_t g = 0; g < g1; ++g) {
            float dw1[4], dwp[4], e[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            fetch_group<MODEL, PAYOFF>(a, s, g, dw1, dwp, e);
            const bool eval = g >= g0;                      // block-uniform
#pragma unroll 1
            for (int k = 0; k < 4; ++k) {
                const int n = 4 * (int)g + k;
                if (n >= a.nf) break;
                const float d1 = k == 0 ? dw1[0] : k == 1 ? dw1[1] : k == 2 ? dw1[2] : dw1[3];
                const float dp = k == 0 ? dwp[0] : k == 1 ? dwp[1] : k == 2 ? dwp[2] : dwp[3];
                const float ek = k == 0 ? e[0] : k == 1 ? e[1] : k == 2 ? e[2] : e[3];
                if (eval) {
                    const float x0 = (float)n * P.h * sh.inv_T;
                    eval_backward<D>(sh, afw, abw, st, x0, q.S, q.v, -wp * d1, acc);
                    if (coupled && (n & (M - 1)) == 0) {
                        // the coarse step starting here sums the next M fine increments
                        const float dwc = (M == 4) ? dw1[0] + dw1[1] + dw1[2] + dw1[3]
                                                   : (k == 0 ? dw1[0] + dw1[1] : dw1[2] + dw1[3]);
                        eval_backward<D>(sh, afw, abw, st, x0, q.Sc, q.vc, wp * dwc, acc);
                    }
                }
                fine_step<float, MODEL, PAYOFF>(q, P, d1, dp, ek, n & (M - 1), coupled);
                if (coupled && ((n + 1) & (M - 1)) == 0) coarse_step<float, MODEL, PAYOFF>(q, P);
            }
        }
    }
    // per-block partial gradient (row blockIdx.x of gpart)
    const int np = nparams(D);
    float* row = gpart + (uint64_t)blockIdx.x * np;
    const int h = lane >> 5;
    float b3 = acc.gb3;
    for (int m = 1; m < 64; m <<= 1) b3 += __shfl_xor(b3, m);
    if (lane == 0) row[off_b3(D)] = b3;
#pragma unroll
    for (int t = 0; t < 32; ++t) {
        float v3 = acc.gw3[t], v2 = acc.gb2[t], v1 = acc.gb1[t];
        float u0 = acc.gW1[0][t], u1 = acc.gW1[1][t], u2 = acc.gW1[2][t];
        for (int m = 1; m < 32; m <<= 1) {     // sum over the lane's half
            v3 += __shfl_xor(v3, m);
            v2 += __shfl_xor(v2, m);
            v1 += __shfl_xor(v1, m);
            u0 += __shfl_xor(u0, m);
            u1 += __shfl_xor(u1, m);
            if (D == 3) u2 += __shfl_xor(u2, m);
        }
        if ((lane & 31) == 0) {
            const int j = row_d(h, t / 16, t % 16);
            row[off_w3(D) + j] = v3;
            row[off_b2(D) + j] = v2 * sh.w3[j];
            const int u = unit_b(h, t);
            row[off_b1(D) + u] = v1;
            row[u * D + 0] = u0;
            row[u * D + 1] = u1;
            if (D == 3) row[u * D + 2] = u2;
        }
    }
#pragma unroll
    for (int ut = 0; ut < 2; ++ut)
#pragma unroll
        for (int jt = 0; jt < 2; ++jt)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int u = row_d(h, ut, r);             // rows of G are units
                const int j = 32 * jt + (lane & 31);       // columns are layer-2 units
                row[off_W2(D) + j * H + u] = acc.G[ut][jt][r];
            }
}

// grad[i] = sum over the partial rows (fixed order): rows [r0, r1) of the
// partials into one row, with the loads of a thread issued ahead of its adds.
__global__ void cv_reduce_kernel(const float* gpart, int rows, int np, float* grad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    float s = 0.0f;
#pragma unroll 8
    for (int r = 0; r < rows; ++r) s += gpart[(uint64_t)r * np + i];
    grad[i] = s;
}

// First pass of the reduction: chunk blockIdx.y of kReduceRows rows into row
// blockIdx.y of `partial` (the second pass, cv_reduce_kernel, adds those rows
// in order; the whole sum keeps one fixed order).
constexpr int kReduceRows = 32;
__global__ void cv_reduce_rows_kernel(const float* gpart, int rows, int np, float* partial)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const int r0 = blockIdx.y * kReduceRows;
    const int r1 = r0 + kReduceRows < rows ? r0 + kReduceRows : rows;
    float s = 0.0f;
#pragma unroll 8
    for (int r = r0; r < r1; ++r) s += gpart[(uint64_t)r * np + i];
    partial[(uint64_t)blockIdx.y * np + i] = s;
}

// Adam (Kingma and Ba 2015) on the fp32 master parameters.
__global__ void cv_adam_kernel(float* params, float* m1, float* m2, const float* grad, int np,
                               float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float g = grad[i];
    const float a = b1 * m1[i] + (1.0f - b1) * g;
    const float v = b2 * m2[i] + (1.0f - b2) * g * g;
    m1[i] = a;
    m2[i] = v;
    params[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// ----------------------------------------------------------- dispatch
using CvFn = void (*)(LevelArgs<float>, CvKernelArgs);
using CvBwdFn = void (*)(LevelArgs<float>, CvKernelArgs, const bf16x8*, const float*, float*, uint32_t);
using CvTrainFwdFn = void (*)(LevelArgs<float>, CvKernelArgs, uint32_t, float*);

template <int MODEL>
static CvTrainFwdFn pick_train_fwd(int payoff, int M)
{
    switch (payoff) {
    case kCall: return M == 2 ? cv_train_fwd_kernel<MODEL, kCall, 2> : cv_train_fwd_kernel<MODEL, kCall, 4>;
    case kAsian: return M == 2 ? cv_train_fwd_kernel<MODEL, kAsian, 2> : cv_train_fwd_kernel<MODEL, kAsian, 4>;
    case kLookback:
        return M == 2 ? cv_train_fwd_kernel<MODEL, kLookback, 2> : cv_train_fwd_kernel<MODEL, kLookback, 4>;
    default: return M == 2 ? cv_train_fwd_kernel<MODEL, kDigital, 2> : cv_train_fwd_kernel<MODEL, kDigital, 4>;
    }
}

template <int MODEL, int PAYOFF>
static CvBwdFn pick_bwd_m(int M)
{
    return M == 2 ? cv_backward_kernel<MODEL, PAYOFF, 2> : cv_backward_kernel<MODEL, PAYOFF, 4>;
}

template <int MODEL>
static CvBwdFn pick_bwd_payoff(int payoff, int M)
{
    switch (payoff) {
    case kCall: return pick_bwd_m<MODEL, kCall>(M);
    case kAsian: return pick_bwd_m<MODEL, kAsian>(M);
    case kLookback: return pick_bwd_m<MODEL, kLookback>(M);
    default: return pick_bwd_m<MODEL, kDigital>(M);
    }
}

template <int MODEL, int PAYOFF>
static CvFn pick_cv_m(int M)
{
    return M == 2 ? cv_level_kernel<MODEL, PAYOFF, 2> : cv_level_kernel<MODEL, PAYOFF, 4>;
}

template <int MODEL>
static CvFn pick_cv_payoff(int payoff, int M)
{
    switch (payoff) {
    case kCall: return pick_cv_m<MODEL, kCall>(M);
    case kAsian: return pick_cv_m<MODEL, kAsian>(M);
    case kLookback: return pick_cv_m<MODEL, kLookback>(M);
    default: return pick_cv_m<MODEL, kDigital>(M);
    }
}

using CvTabFn = void (*)(LevelArgs<float>, const float*, TableSpec);

// Tabulated sampler for one payoff: the short-level kernel (n_f < 4), the
// split kernel (GBM, split > 1) or the per-lane kernel with ppt samples.
template <int MODEL, int PAYOFF, int M>
static CvTabFn pick_tab_m(int nf, int split, int ppt)
{
    if (nf < 4) return cv_tab_short_kernel<MODEL, PAYOFF, M>;
    if constexpr (MODEL == kGBM)
        if (split > 1) return cv_tab_split_kernel<PAYOFF, M>;
    return ppt == 2 ? cv_tab_level_kernel<MODEL, PAYOFF, M, 2> : cv_tab_level_kernel<MODEL, PAYOFF, M, 1>;
}

template <int MODEL>
static CvTabFn pick_tab_payoff(int payoff, int M, int nf, int split, int ppt)
{
    switch (payoff) {
    case kCall: return M == 2 ? pick_tab_m<MODEL, kCall, 2>(nf, split, ppt) : pick_tab_m<MODEL, kCall, 4>(nf, split, ppt);
    case kAsian: return M == 2 ? pick_tab_m<MODEL, kAsian, 2>(nf, split, ppt) : pick_tab_m<MODEL, kAsian, 4>(nf, split, ppt);
    case kLookback:
        return M == 2 ? pick_tab_m<MODEL, kLookback, 2>(nf, split, ppt) : pick_tab_m<MODEL, kLookback, 4>(nf, split, ppt);
    default: return M == 2 ? pick_tab_m<MODEL, kDigital, 2>(nf, split, ppt) : pick_tab_m<MODEL, kDigital, 4>(nf, split, ppt);
    }
}

NetConsts net_consts(const mlmc_model& m)
{
    NetConsts c;
    const double sref = m.kind == MLMC_GBM ? m.sigma : std::sqrt(m.theta);
    c.scale = (float)(sref * m.S0);
    const double a = std::log(2.0) / (sref * std::sqrt(m.T));
    c.x1a = (float)a;
    c.x1b = (float)(std::log2(m.S0) * a);
    c.x2a = m.kind == MLMC_HESTON ? (float)(1.0 / m.theta) : 0.0f;
    c.x2b = m.kind == MLMC_HESTON ? 1.0f : 0.0f;
    c.inv_T = (float)(1.0 / m.T);
    c.s_floor = (float)(m.S0 * std::ldexp(1.0, -40));
    return c;
}

static bool same_model(const mlmc_model& a, const mlmc_model& b)
{
    return a.kind == b.kind && a.S0 == b.S0 && a.r == b.r && a.sigma == b.sigma && a.T == b.T &&
           a.kappa == b.kappa && a.theta == b.theta && a.xi == b.xi && a.rho == b.rho && a.v0 == b.v0;
}

// The table of the current parameters for model m in cv->d_table, rebuilt
// when the parameters, the model or the stream changed (the same caching rule
// as phi(0, S0)).
static hipError_t cv_ensure_table(mlmc_cv* cv, const mlmc_model& m, hipStream_t st)
{
    if (cv->table_version == cv->version && cv->table_stream == st && same_model(cv->table_model, m))
        return hipSuccess;
    const TableGrid g = table_grid(m);
    const size_t n = table_size(g);
    if (cv->table_cap < n) {
        // the previous table may still be read by queued launches
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        if (cv->d_table) hipFree(cv->d_table);
        cv->d_table = nullptr;
        cv->table_cap = 0;
        e = hipMalloc(&cv->d_table, sizeof(float) * n);
        if (e != hipSuccess) return e;
        cv->table_cap = n;
    }
    CvKernelArgs c{cv->d_params, cv->d_afwd, net_consts(m), cv->D};
    const int blocks = (int)((n + 255) / 256);
    if (cv->D == 2)
        hipLaunchKernelGGL(cv_table_kernel<2>, dim3(blocks), dim3(256), 0, st, c, g, cv->d_table);
    else
        hipLaunchKernelGGL(cv_table_kernel<3>, dim3(blocks), dim3(256), 0, st, c, g, cv->d_table);
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        cv->table_version = cv->version;
        cv->table_stream = st;
        cv->table_model = m;
    }
    return e;
}

// phi(0, S0) for level 0 in cv->d_phi0[0] (from the network) or, for the
// tabulated form, cv->d_phi0[1] (from the table).  The value depends only on
// the parameters and the model, so it is computed once per parameter change,
// model and stream (a launch on another stream would not be ordered after
// the write) and level-0 launches reuse it.
hipError_t cv_ensure_phi0(const mlmc_cv* ccv, const mlmc_model& m, hipStream_t st, bool tab)
{
    mlmc_cv* cv = const_cast<mlmc_cv*>(ccv);
    const int w = tab ? 1 : 0;
    if (cv->phi0_version[w] == cv->version && cv->phi0_stream[w] == st &&
        same_model(cv->phi0_model[w], m))
        return hipSuccess;
    if (tab) {
        hipError_t e = cv_ensure_table(cv, m, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(cv_table_point_kernel, dim3(1), dim3(64), 0, st, (const float*)cv->d_table,
                           table_spec(table_grid(m)), (float)m.S0, (float)m.v0, cv->d_phi0 + 1);
    } else {
        CvKernelArgs c{cv->d_params, cv->d_afwd, net_consts(m), cv->D};
        if (cv->D == 2)
            hipLaunchKernelGGL(cv_phi0_kernel<2>, dim3(1), dim3(64), 0, st, c, (float)m.S0,
                               (float)m.v0, cv->d_phi0);
        else
            hipLaunchKernelGGL(cv_phi0_kernel<3>, dim3(1), dim3(64), 0, st, c, (float)m.S0,
                               (float)m.v0, cv->d_phi0);
    }
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        cv->phi0_version[w] = cv->version;
        cv->phi0_stream[w] = st;
        cv->phi0_model[w] = m;
    }
    return e;
}

bool cv_tabulated(const mlmc_cv* cv) { return cv->tabulated != 0; }

hipError_t cv_table_view(const mlmc_cv* ccv, const mlmc_model& m, hipStream_t st, int max_nf,
                         const float** table, TableSpec* spec, const float** phi0, size_t* lds_bytes)
{
    const hipError_t e = cv_ensure_phi0(ccv, m, st, true);   // builds the table first
    if (e != hipSuccess) return e;
    const TableGrid g = table_grid(m);
    const int lr = max_nf < g.rows ? max_nf : g.rows;
    *table = ccv->d_table;
    *spec = table_spec(g);
    *phi0 = ccv->d_phi0 + 1;
    *lds_bytes = sizeof(float) * (size_t)lr * g.ns * g.nv;
    return hipSuccess;
}

hipError_t cv_launch_level(const mlmc_cv* ccv, const mlmc_model& m, const mlmc_payoff& p, int M,
                           const LevelArgs<float>& a, int grid, hipStream_t st, bool tab, int ppt)
{
    mlmc_cv* cv = const_cast<mlmc_cv*>(ccv);
    if (tab) {
        hipError_t e = cv_ensure_table(cv, m, st);
        if (e != hipSuccess) return e;
        const TableGrid g = table_grid(m);
        const int lr = a.nf < g.rows ? a.nf : g.rows;    // rows the level reads
        const size_t lds = sizeof(float) * (size_t)lr * g.ns * g.nv;
        CvTabFn fn = m.kind == MLMC_GBM ? pick_tab_payoff<kGBM>(p.kind, M, a.nf, (int)a.split, ppt)
                                        : pick_tab_payoff<kHeston>(p.kind, M, a.nf, 1, ppt);
        hipLaunchKernelGGL(fn, dim3(grid), dim3(256), lds, st, a, (const float*)cv->d_table,
                           table_spec(g));
        return hipGetLastError();
    }
    CvKernelArgs c{cv->d_params, cv->d_afwd, net_consts(m), cv->D};
    CvFn fn = m.kind == MLMC_GBM ? pick_cv_payoff<kGBM>(p.kind, M) : pick_cv_payoff<kHeston>(p.kind, M);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, st, a, c);
    return hipGetLastError();
}

// The backward launch of level l for a batch of B: segments per path (a
// power of two dividing the level's generator groups, so that the level
// has about kBwdBlocks blocks of 64 samples x segment) and its grid.
constexpr uint64_t kBwdBlocks = 2048;
struct BwdShape {
    uint32_t segs;
    int grid;
};
static BwdShape bwd_shape(uint64_t B, int l, int M)
{
    uint64_t nf = 1;
    for (int i = 0; i < l; ++i) nf *= (uint64_t)M;
    const uint64_t groups = (nf + 3) / 4, nchunks = (B + 63) / 64;
    uint32_t segs = 1;
    while ((uint64_t)segs * 2 <= groups && groups % ((uint64_t)segs * 2) == 0 &&
           nchunks * segs * 2 <= kBwdBlocks)
        segs *= 2;
    const uint64_t units = nchunks * segs;
    return BwdShape{segs, (int)(units < kBwdBlocks ? units : kBwdBlocks)};
}

// Rows of per-block gradient partials of one training step, and the
// reduction's first-pass rows after them (the gradient is the row after).
static int bwd_rows(uint64_t B, int lmax, int M)
{
    int rows = 0;
    for (int l = 0; l <= lmax; ++l) rows += bwd_shape(B, l, M).grid;
    return rows;
}

// Scratch for a training batch of B samples per level, levels 0..lmax.
static mlmc_status ensure_train(mlmc_cv* cv, uint64_t B, int lmax, int M)
{
    mlmc_ctx* ctx = cv->ctx;
    const uint64_t need = B * (uint64_t)(lmax + 1);
    const int brows = bwd_rows(B, lmax, M);
    const int rows = brows + (brows + kReduceRows - 1) / kReduceRows;
    if (cv->batch_cap < need) {
        if (cv->d_y) hipFree(cv->d_y);
        if (cv->d_w) hipFree(cv->d_w);
        cv->d_y = nullptr;
        cv->d_w = nullptr;
        MLMC_HIP(ctx, hipMalloc(&cv->d_y, sizeof(double) * 2 * need));
        MLMC_HIP(ctx, hipMalloc(&cv->d_w, sizeof(float) * need));
        cv->batch_cap = need;
    }
    // the forward runs' partials of the level with the most runs
    uint64_t fneed = 0;
    for (int l = 0; l <= lmax; ++l) {
        const uint64_t segs = bwd_shape(B, l, M).segs;
        if (segs > 1 && (2 * segs + 2) * B > fneed) fneed = (2 * segs + 2) * B;
    }
    if (cv->fpart_cap < fneed) {
        if (cv->d_fpart) hipFree(cv->d_fpart);
        cv->d_fpart = nullptr;
        cv->fpart_cap = 0;
        MLMC_HIP(ctx, hipMalloc(&cv->d_fpart, sizeof(float) * fneed));
        cv->fpart_cap = fneed;
    }
    if (cv->gpart_blocks < rows + 1) {
        if (cv->d_gpart) hipFree(cv->d_gpart);
        cv->d_gpart = nullptr;
        MLMC_HIP(ctx, hipMalloc(&cv->d_gpart, sizeof(float) * (uint64_t)(rows + 1) * cv->np));
        cv->gpart_blocks = rows + 1;
    }
    return MLMC_OK;
}

// Kernel arguments of level l of a training batch (the training streams;
// fetch_group forms every counter from the sample index, so no counter words
// are set).
static LevelArgs<float> train_args(const mlmc_model& m, const mlmc_payoff& p, int l, int M, uint64_t B,
                                   uint64_t seed, uint64_t offset)
{
    LevelArgs<float> a;
    a.P = make_step_params<float>(m, p, l, M);
    a.seed = seed;
    a.offset = offset;
    a.N = B;
    a.l = l;
    int nf = 1;
    for (int i = 0; i < l; ++i) nf *= M;
    a.nf = nf;
    a.ngroups = (uint32_t)((nf + 3) / 4);
    a.stream = kStreamTrainNormal;
    a.acc = nullptr;
    a.pf_out = a.pc_out = nullptr;
    a.coupled = 1;
    a.phi0 = nullptr;
    return a;
}

// One loss/gradient evaluation: forward pass with per-sample dumps, weights,
// backward pass into per-block partials, reduction into the last row of
// d_gpart.  Everything is enqueued on the context's stream.
static mlmc_status enqueue_loss_grad(mlmc_cv* cv, const mlmc_model& m, const mlmc_payoff& p, int M,
                                     int lmax, uint64_t B, uint64_t seed, uint64_t step,
                                     LevelAcc* rec, float** grad_out)
{
    mlmc_ctx* ctx = cv->ctx;
    mlmc_status st = ensure_train(cv, B, lmax, M);
    if (st) return st;
    MLMC_HIP(ctx, zero_records(rec, lmax + 1, ctx->stream));
    MLMC_HIP(ctx, hipMemsetAsync(cv->d_loss, 0, sizeof(double) * 64, ctx->stream));
    const uint64_t offset = step * B;
    CvKernelArgs c{cv->d_params, cv->d_afwd, net_consts(m), cv->D};
    for (int l = 0; l <= lmax; ++l) {
        double* pf = cv->d_y + 2 * (uint64_t)l * B;
        const BwdShape bs = bwd_shape(B, l, M);
        if (bs.segs == 1) {
            // one sample per lane (the sampler's own launch)
            st = enqueue_level(ctx, m, p, l, M, B, seed, offset, 32, kStreamTrainNormal, 1, &rec[l],
                               pf, pf + B, cv);
            if (st) return st;
            continue;
        }
        // a deep level in runs of generator groups, as the backward pass
        LevelArgs<float> a = train_args(m, p, l, M, B, seed, offset);
        a.acc = &rec[l];
        a.pf_out = pf;
        a.pc_out = pf + B;
        a.coupled = 1;
        const CvTrainFwdFn fwd = m.kind == MLMC_GBM ? pick_train_fwd<kGBM>(p.kind, M)
                                                    : pick_train_fwd<kHeston>(p.kind, M);
        hipLaunchKernelGGL(fwd, dim3(bs.grid), dim3(64), 0, ctx->stream, a, c, bs.segs, cv->d_fpart);
        MLMC_HIP(ctx, hipGetLastError());
        const int cgrid = (int)((B + 255) / 256 < 256 ? (B + 255) / 256 : 256);
        hipLaunchKernelGGL(cv_train_combine_kernel, dim3(cgrid), dim3(256), 0, ctx->stream, a, bs.segs,
                           (const float*)cv->d_fpart);
        MLMC_HIP(ctx, hipGetLastError());
    }
    hipLaunchKernelGGL(cv_weights_kernel, dim3(lmax + 1), dim3(256), 0, ctx->stream,
                       (const LevelAcc*)rec, (const double*)cv->d_y, B, M, cv->d_w, cv->d_loss);
    MLMC_HIP(ctx, hipGetLastError());
    int row0 = 0;
    const int tix = timed_begin(ctx, 18, 0.0, 0.0);
    for (int l = 0; l <= lmax; ++l) {
        const LevelArgs<float> a = train_args(m, p, l, M, B, seed, offset);
        CvBwdFn fn = m.kind == MLMC_GBM ? pick_bwd_payoff<kGBM>(p.kind, M)
                                        : pick_bwd_payoff<kHeston>(p.kind, M);
        const BwdShape bs = bwd_shape(B, l, M);
        hipLaunchKernelGGL(fn, dim3(bs.grid), dim3(64), 0, ctx->stream, a, c,
                           (const bf16x8*)cv->d_abwd, (const float*)(cv->d_w + (uint64_t)l * B),
                           cv->d_gpart + (uint64_t)row0 * cv->np, bs.segs);
        MLMC_HIP(ctx, hipGetLastError());
        row0 += bs.grid;
    }
    // two passes in a fixed order: chunks of kReduceRows rows, then the chunks
    const int nchunk = (row0 + kReduceRows - 1) / kReduceRows;
    float* partial = cv->d_gpart + (uint64_t)row0 * cv->np;
    float* grad = partial + (uint64_t)nchunk * cv->np;
    hipLaunchKernelGGL(cv_reduce_rows_kernel, dim3((cv->np + 255) / 256, nchunk), dim3(256), 0,
                       ctx->stream, (const float*)cv->d_gpart, row0, cv->np, partial);
    MLMC_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(cv_reduce_kernel, dim3((cv->np + 255) / 256), dim3(256), 0, ctx->stream,
                       (const float*)partial, nchunk, cv->np, grad);
    MLMC_HIP(ctx, hipGetLastError());
    timed_end(ctx, tix);
    *grad_out = grad;
    return MLMC_OK;
}

static mlmc_status check_train_args(mlmc_cv* cv, const mlmc_model* m, const mlmc_payoff* p, int M,
                                    int lmax, uint64_t B)
{
    mlmc_ctx* ctx = cv->ctx;
    mlmc_status st = check_level_args(ctx, m, p, lmax < 0 ? 0 : lmax, M, 32);
    if (st) return st;
    if (lmax < 0 || lmax > 6) return fail(ctx, MLMC_EINVAL, "lmax must be in 0..6");
    if (B < 2 || B > (1ull << 24)) return fail(ctx, MLMC_EINVAL, "batch must be in 2..2^24 per level");
    if (cv->D != (m->kind == MLMC_HESTON ? 3 : 2))
        return fail(ctx, MLMC_EINVAL, "network inputs do not match the model (2: GBM, 3: Heston)");
    if (m->scheme != MLMC_EULER || m->antithetic || p->kind == MLMC_DIGITAL_COND)
        return fail(ctx, MLMC_EINVAL, "the control variate trains on plain Euler paths and payoffs");
    return MLMC_OK;
}

const float* cv_phi0_ptr(const mlmc_cv* cv, bool tab) { return cv->d_phi0 + (tab ? 1 : 0); }
int cv_in_dim(const mlmc_cv* cv) { return cv->D; }

static hipError_t cv_prepare(mlmc_cv* cv, hipStream_t st)
{
    ++cv->version;
    hipLaunchKernelGGL(cv_prepare_kernel, dim3(1), dim3(256), 0, st, (const float*)cv->d_params,
                       cv->D, cv->d_afwd, cv->d_abwd);
    return hipGetLastError();
}

}  // namespace mlmc

using namespace mlmc;

namespace {
const mlmc_payoff kAnyPayoff{MLMC_CALL, 100.0, 1.0};
}

extern "C" {

mlmc_status mlmc_cv_destroy(mlmc_cv* cv)
{
    if (!cv) return MLMC_OK;
    if (cv->ctx) hipSetDevice(cv->ctx->device);
    for (void* p : {(void*)cv->d_params, (void*)cv->d_m1, (void*)cv->d_m2, (void*)cv->d_afwd,
                    (void*)cv->d_abwd, (void*)cv->d_phi0, (void*)cv->d_gpart, (void*)cv->d_y,
                    (void*)cv->d_w, (void*)cv->d_loss, (void*)cv->d_table, (void*)cv->d_fpart})
        if (p) hipFree(p);
    delete cv;
    return MLMC_OK;
}

mlmc_status mlmc_cv_create(mlmc_ctx* ctx, int in_dim, int hidden, uint64_t init_seed, mlmc_cv** out)
{
    if (!ctx) return MLMC_EINVAL;
    if (!out) return fail(ctx, MLMC_EINVAL, "out must not be NULL");
    *out = nullptr;
    if ((in_dim != 2 && in_dim != 3) || hidden != H)
        return fail(ctx, MLMC_EINVAL, "in_dim must be 2 (GBM) or 3 (Heston) and hidden 64");
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    mlmc_cv* cv = new (std::nothrow) mlmc_cv();
    if (!cv) return fail(ctx, MLMC_ENOMEM, "host allocation failed");
    cv->ctx = ctx;
    cv->D = in_dim;
    cv->np = nparams(in_dim);
    hipError_t e = hipMalloc(&cv->d_params, sizeof(float) * cv->np);
    if (e == hipSuccess) e = hipMalloc(&cv->d_m1, sizeof(float) * cv->np);
    if (e == hipSuccess) e = hipMalloc(&cv->d_m2, sizeof(float) * cv->np);
    if (e == hipSuccess) e = hipMalloc(&cv->d_afwd, sizeof(bf16x8) * 8 * 64);
    if (e == hipSuccess) e = hipMalloc(&cv->d_abwd, sizeof(bf16x8) * 8 * 64);
    if (e == hipSuccess) e = hipMalloc(&cv->d_phi0, sizeof(float) * 4);
    if (e == hipSuccess) e = hipMalloc(&cv->d_loss, sizeof(double) * 64);
    if (e == hipSuccess) e = hipMemsetAsync(cv->d_m1, 0, sizeof(float) * cv->np, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(cv->d_m2, 0, sizeof(float) * cv->np, ctx->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(cv_init_kernel, dim3((cv->np + 255) / 256), dim3(256), 0, ctx->stream,
                           cv->d_params, in_dim, init_seed);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = cv_prepare(cv, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        mlmc_cv_destroy(cv);
        return hip_fail(ctx, e, "control variate allocation/initialisation");
    }
    *out = cv;
    return MLMC_OK;
}

mlmc_status mlmc_cv_get_params(const mlmc_cv* cv, float* host, size_t n)
{
    if (!cv) return MLMC_EINVAL;
    mlmc_ctx* ctx = cv->ctx;
    if (!host || n != (size_t)cv->np) return fail(ctx, MLMC_EINVAL, "need a host array of nparams floats");
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    MLMC_HIP(ctx, hipMemcpyAsync(host, cv->d_params, sizeof(float) * n, hipMemcpyDeviceToHost,
                                 ctx->stream));
    MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return MLMC_OK;
}

mlmc_status mlmc_cv_set_params(mlmc_cv* cv, const float* host, size_t n)
{
    if (!cv) return MLMC_EINVAL;
    mlmc_ctx* ctx = cv->ctx;
    if (!host || n != (size_t)cv->np) return fail(ctx, MLMC_EINVAL, "need a host array of nparams floats");
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) return fail(ctx, MLMC_EINVAL, "parameters must be finite");
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    MLMC_HIP(ctx, hipMemcpyAsync(cv->d_params, host, sizeof(float) * n, hipMemcpyHostToDevice,
                                 ctx->stream));
    MLMC_HIP(ctx, cv_prepare(cv, ctx->stream));
    MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return MLMC_OK;
}

size_t mlmc_cv_nparams(const mlmc_cv* cv) { return cv ? (size_t)cv->np : 0; }

mlmc_status mlmc_cv_set_tabulated(mlmc_cv* cv, int on)
{
    if (!cv) return MLMC_EINVAL;
    if (on != 0 && on != 1) return fail(cv->ctx, MLMC_EINVAL, "on must be 0 or 1");
    cv->tabulated = on;
    return MLMC_OK;
}

mlmc_status mlmc_cv_get_table(mlmc_cv* cv, const mlmc_model* model, float* host, size_t n,
                              int* dims)
{
    if (!cv) return MLMC_EINVAL;
    mlmc_ctx* ctx = cv->ctx;
    mlmc_status st = check_level_args(ctx, model, &kAnyPayoff, 0, 2, 32);
    if (st) return st;
    if (cv->D != (model->kind == MLMC_HESTON ? 3 : 2))
        return fail(ctx, MLMC_EINVAL, "network inputs do not match the model (2: GBM, 3: Heston)");
    const TableGrid g = table_grid(*model);
    if (dims) {
        dims[0] = g.rows;
        dims[1] = g.nv;
        dims[2] = g.ns;
    }
    if (!host) return MLMC_OK;
    if (n != table_size(g)) return fail(ctx, MLMC_EINVAL, "need a host array of rows * nv * ns floats");
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    MLMC_HIP(ctx, cv_ensure_table(cv, *model, ctx->stream));
    MLMC_HIP(ctx, hipMemcpyAsync(host, cv->d_table, sizeof(float) * n, hipMemcpyDeviceToHost,
                                 ctx->stream));
    MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return MLMC_OK;
}

mlmc_status mlmc_cv_loss_grad(mlmc_cv* cv, const mlmc_model* model, const mlmc_payoff* payoff,
                              int M, int lmax, uint64_t batch, uint64_t seed, uint64_t step,
                              float* grad, double* var, double* loss)
{
    if (!cv) return MLMC_EINVAL;
    mlmc_ctx* ctx = cv->ctx;
    mlmc_status st = check_train_args(cv, model, payoff, M, lmax, batch);
    if (st) return st;
    ctx->err.clear();
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    float* d_grad = nullptr;
    st = enqueue_loss_grad(cv, *model, *payoff, M, lmax, batch, seed, step, ctx->d_acc, &d_grad);
    if (st) return st;
    if (grad)
        MLMC_HIP(ctx, hipMemcpyAsync(grad, d_grad, sizeof(float) * cv->np, hipMemcpyDeviceToHost,
                                     ctx->stream));
    double hl[64];
    MLMC_HIP(ctx, hipMemcpyAsync(hl, cv->d_loss, sizeof(hl), hipMemcpyDeviceToHost, ctx->stream));
    MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    harvest_timing(ctx);
    if (loss) *loss = hl[0];
    if (var)
        for (int l = 0; l <= lmax; ++l) var[l] = hl[1 + l];
    return MLMC_OK;
}

mlmc_status mlmc_cv_train(mlmc_cv* cv, const mlmc_model* model, const mlmc_payoff* payoff, int M,
                          int lmax, int steps, uint64_t batch, double lr, uint64_t seed,
                          float* loss_hist)
{
    if (!cv) return MLMC_EINVAL;
    mlmc_ctx* ctx = cv->ctx;
    mlmc_status st = check_train_args(cv, model, payoff, M, lmax, batch);
    if (st) return st;
    if (steps < 0 || !(lr > 0)) return fail(ctx, MLMC_EINVAL, "need steps >= 0 and lr > 0");
    ctx->err.clear();
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    double* d_hist = nullptr;
    if (loss_hist && steps > 0) MLMC_HIP(ctx, hipMalloc(&d_hist, sizeof(double) * steps));
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int k = 0; k < steps; ++k) {
        const TraceRange step_range("mlmc_cv_train step");
        float* d_grad = nullptr;
        // each step draws fresh training samples: indices t * batch .. (t+1) * batch - 1
        st = enqueue_loss_grad(cv, *model, *payoff, M, lmax, batch, seed, (uint64_t)cv->adam_t, ctx->d_acc,
                               &d_grad);
        if (st) break;
        cv->adam_t += 1;
        const float c1 = 1.0f - std::pow(b1, (float)cv->adam_t);
        const float c2 = 1.0f - std::pow(b2, (float)cv->adam_t);
        hipLaunchKernelGGL(cv_adam_kernel, dim3((cv->np + 255) / 256), dim3(256), 0, ctx->stream,
                           cv->d_params, cv->d_m1, cv->d_m2, (const float*)d_grad, cv->np, (float)lr,
                           b1, b2, eps, c1, c2);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = cv_prepare(cv, ctx->stream);
        if (e == hipSuccess && d_hist)
            e = hipMemcpyAsync(d_hist + k, cv->d_loss, sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream);
        if (e != hipSuccess) {
            st = hip_fail(ctx, e, "training step");
            break;
        }
    }
    if (!st && d_hist) {
        std::vector<double> h(steps);
        hipError_t e = hipMemcpyAsync(h.data(), d_hist, sizeof(double) * steps,
                                      hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = hip_fail(ctx, e, "loss history copy");
        for (int k = 0; k < steps; ++k) loss_hist[k] = (float)h[k];
    }
    if (!st) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = hip_fail(ctx, e, "training");
        harvest_timing(ctx);
    }
    if (d_hist) hipFree(d_hist);
    return st;
}

}  // extern "C"
