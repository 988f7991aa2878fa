// Learned martingale control variate: the MLP phi(t, X) evaluated for the 64
// samples of a wavefront at once, layer 2 on the bf16 matrix cores.
//
// The control variate is the discrete martingale sum_n phi(t_n, X_n) dW_n
// (left-point evaluation, so every term has conditional mean zero and the
// level estimators of eqs. (eq:mlmc:Yzero), (eq:Yldef) keep their means; the
// control-variate idea is Sec. 5, "Exploiting Structure").  Network:
//   x = (t/T, ln(max(S, S0 2^-40)/S0)/(sref sqrt T) [, (v - theta)/theta])
//   h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), phi = sref S0 (w3.h2 + b3)
// with H = 64 hidden units.  Layer 1 and 3 run in fp32 on the vector ALUs;
// layer 2 is a 64x64x64 product per evaluation (units x units x samples) on
// v_mfma_f32_32x32x16_bf16: W2 and h1 in bf16, fp32 accumulation.
//
// Lane layouts (wave of 64 lanes, lane l, half h = l / 32):
//   bf16 B operand (K = 16 units x N = 32 samples): lane l holds column
//     n = l % 32, rows 8h + i (i < 8) of the K block;
//   A operand (M = 32 rows x K = 16): lane l holds row l % 32, columns
//     8h + i;
//   fp32 accumulator (32 x 32): register r of lane l is row
//     8 (r / 4) + 4h + r % 4, column l % 32.
// Sample p of the wave lives in lane p.  Lane l computes layer 1 for samples
// l % 32 and 32 + l % 32 (its own and lane l ^ 32's), at the 32 units
// unit_b(h, s) of its B-operand slots s = 8 kb + i, so no data moves between
// layer 1 and the matrix product; layer 3 sums each half-column of h2 and one
// exchange with lane l ^ 32 completes phi.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlmc {
namespace cvnet {

constexpr int H = 64;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Unit at B-operand slot s (0..31) of lane half h (k block s / 8, element s % 8).
__host__ __device__ constexpr int unit_b(int h, int s) { return 16 * (s / 8) + 8 * h + s % 8; }
// Row of accumulator register r (0..15) of row tile t for lane half h.
__host__ __device__ constexpr int row_d(int h, int t, int r) { return 32 * t + 8 * (r / 4) + 4 * h + r % 4; }

// Parameter offsets in the flat vector (same order as the CPU reference):
// W1[H][D], b1[H], W2[H][H] (row = output unit), b2[H], w3[H], b3.
__host__ __device__ constexpr int off_b1(int D) { return H * D; }
__host__ __device__ constexpr int off_W2(int D) { return H * D + H; }
__host__ __device__ constexpr int off_b2(int D) { return H * D + H + H * H; }
__host__ __device__ constexpr int off_w3(int D) { return H * D + 2 * H + H * H; }
__host__ __device__ constexpr int off_b3(int D) { return H * D + 3 * H + H * H; }
__host__ __device__ constexpr int nparams(int D) { return H * D + 3 * H + H * H + 1; }

// Network constants shared by a block (loaded into LDS once).
struct NetShared {
    float w1[H][4];       // W1 row u: (t, log S [, v]) weights, then b1[u]
    float b2[H], w3[H];
    float b3, scale;      // scale = sref * S0
    float x1a, x1b;       // x1 = log2(max(S, floor)) * x1a - x1b
    float x2a, x2b;       // x2 = v * x2a - x2b
    float inv_T, s_floor;
};

// Host-side description of the network inputs and output scale.
struct NetConsts {
    float scale, x1a, x1b, x2a, x2b, inv_T, s_floor;
};

__device__ __forceinline__ float tanh_fast(float x)
{
    // 1 - 2 / (e^{2x} + 1); e^{2x} = 2^{2x log2 e}.  Exact limits +-1.
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);
    return __builtin_fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}

template <int D>
__device__ __forceinline__ void load_shared(NetShared& sh, const float* params, const NetConsts& c)
{
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
        for (int d = 0; d < D; ++d) sh.w1[i][d] = params[i * D + d];
        for (int d = D; d < 3; ++d) sh.w1[i][d] = 0.0f;
        sh.w1[i][3] = params[off_b1(D) + i];
        sh.b2[i] = params[off_b2(D) + i];
        sh.w3[i] = params[off_w3(D) + i];
    }
    if (threadIdx.x == 0) {
        sh.b3 = params[off_b3(D)];
        sh.scale = c.scale;
        sh.x1a = c.x1a;
        sh.x1b = c.x1b;
        sh.x2a = c.x2a;
        sh.x2b = c.x2b;
        sh.inv_T = c.inv_T;
        sh.s_floor = c.s_floor;
    }
}

// Forward-pass A operands of W2 (bf16), prepared by the host-side kernel in
// lane order: afwd[(jt * 4 + kb) * 64 + lane] = W2[32 jt + l%32][16 kb + 8h + i].
__device__ __forceinline__ void load_afwd(const bf16x8* afwd, bf16x8 (&a)[2][4])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) a[jt][kb] = afwd[(jt * 4 + kb) * 64 + lane];
}

// Network inputs x1 (and x2) of one sample; x0 = t/T is wave-uniform.
__device__ __forceinline__ float input_x1(const NetShared& sh, float S)
{
    const float s = S > sh.s_floor ? S : sh.s_floor;
    return __builtin_fmaf(__builtin_amdgcn_logf(s), sh.x1a, -sh.x1b);
}

// Layer-1 activations of the lane's two samples, packed as B operands.
// h1f (optional, 64 floats) receives the fp32 values: h1f[nt * 32 + s].
// x0 is the time input of both samples (wave-uniform in the samplers); with
// X0LANE the two samples have their own, x0p[nt].
template <int D, bool KEEP, bool X0LANE = false>
__device__ __forceinline__ void layer1(const NetShared& sh, float x0, const float (&x1)[2],
                                       const float (&x2)[2], bf16x8 (&b)[2][4], float* h1f,
                                       const float* x0p = nullptr)
{
    const int h = (threadIdx.x & 63) >> 5;
#pragma unroll
    for (int s = 0; s < 32; ++s) {
        const int u = unit_b(h, s);
        const float c = __builtin_fmaf(sh.w1[u][0], x0, sh.w1[u][3]);
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const float cn = X0LANE ? __builtin_fmaf(sh.w1[u][0], x0p[nt], sh.w1[u][3]) : c;
            float a = __builtin_fmaf(sh.w1[u][1], x1[nt], cn);
            if (D == 3) a = __builtin_fmaf(sh.w1[u][2], x2[nt], a);
            const float v = tanh_fast(a);
            if (KEEP) h1f[nt * 32 + s] = v;
            b[nt][s / 8][s % 8] = (__bf16)v;
        }
    }
}

// Layer 2 on the matrix cores: acc[jt][nt] = b2 + W2[jt rows] h1[nt samples].
__device__ __forceinline__ void layer2(const NetShared& sh, const bf16x8 (&a)[2][4],
                                       const bf16x8 (&b)[2][4], f32x16 (&acc)[2][2])
{
    const int h = (threadIdx.x & 63) >> 5;
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[jt][nt][r] = sh.b2[row_d(h, jt, r)];
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
                acc[jt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[jt][kb], b[nt][kb],
                                                                      acc[jt][nt], 0, 0, 0);
        }
}

// Samples handled by this lane's two B columns: nt = h is its own sample,
// nt = 1 - h the sample of lane l ^ 32.
template <int D>
__device__ __forceinline__ void pair_inputs(const NetShared& sh, float S, float v, float (&x1)[2],
                                            float (&x2)[2])
{
    const int h = (threadIdx.x & 63) >> 5;
    const float own1 = input_x1(sh, S);
    const float oth1 = __shfl_xor(own1, 32);
    x1[0] = h == 0 ? own1 : oth1;
    x1[1] = h == 0 ? oth1 : own1;
    if (D == 3) {
        const float own2 = __builtin_fmaf(v, sh.x2a, -sh.x2b);
        const float oth2 = __shfl_xor(own2, 32);
        x2[0] = h == 0 ? own2 : oth2;
        x2[1] = h == 0 ? oth2 : own2;
    } else {
        x2[0] = x2[1] = 0.0f;
    }
}

// phi(t, X) of this lane's sample; every lane of the wave must call it.
// afwd: the bf16 W2 operands in lane order (in LDS in the sampler).  Layer 2
// and layer 3 run one 32-row tile at a time, so only half of the matrix
// accumulators are live.
template <int D, bool X0LANE = false>
__device__ __forceinline__ float phi_eval(const NetShared& sh, const bf16x8* afwd, float x0,
                                          float S, float v)
{
    // The network constants are read from LDS at every evaluation: kept in
    // registers across the path loop they would take ~190 VGPRs and leave a
    // single wave per SIMD.  The empty asm (a compiler-only memory clobber,
    // no instruction) stops the loads from being hoisted out of the loop.
    __asm__ volatile("" ::: "memory");
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5;
    float x1[2], x2[2];
    pair_inputs<D>(sh, S, v, x1, x2);
    bf16x8 b[2][4];
    float x0p[2] = {x0, x0};
    if (X0LANE) {
        // this lane's sample and lane l ^ 32's, in B-column order
        const float oth = __shfl_xor(x0, 32);
        x0p[0] = h == 0 ? x0 : oth;
        x0p[1] = h == 0 ? oth : x0;
    }
    layer1<D, false, X0LANE>(sh, x0, x1, x2, b, nullptr, x0p);
    float part[2] = {0.0f, 0.0f};
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
        bf16x8 a[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) a[kb] = afwd[(jt * 4 + kb) * 64 + lane];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            f32x16 acc;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = sh.b2[row_d(h, jt, r)];
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[kb], b[nt][kb], acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 16; ++r)
                part[nt] = __builtin_fmaf(sh.w3[row_d(h, jt, r)], tanh_fast(acc[r]), part[nt]);
        }
    }
    const float send = h == 0 ? part[1] : part[0];
    const float recv = __shfl_xor(send, 32);
    const float mine = h == 0 ? part[0] : part[1];
    return sh.scale * (mine + recv + sh.b3);
}

// ------------------------------------------------------------ tabulated
// The sampler may read phi from a table instead of evaluating the network at
// every point: phi on a grid of `rows` times t_j = j T / rows, ns stock values
// S_i = s_lo + i dS (and nv variances v_k = v_lo + k dv for Heston), filled by
// the network itself (cv_table_kernel), and interpolated linearly in S (and v)
// within the row of the last grid time at or before the evaluation time.  Any
// function of (t_n, X_n) keeps the control variate's mean at zero, so the
// table changes only how much variance it removes, not the level means.
struct TableSpec {
    int rows, ns, nv;
    float s_lo, s_inv;    // u = (S - s_lo) s_inv, grid index in S
    float v_lo, v_inv;    // w = (v - v_lo) v_inv (nv > 1)
};

// Row of step n of a path with nf fine steps: floor(n rows / nf).
__device__ __forceinline__ int table_row(int n, int nf, int rows)
{
    return (int)(((unsigned)n * (unsigned)rows) / (unsigned)nf);
}

// Linear (bilinear for nv > 1) interpolation in one row; points outside the
// grid take the nearest edge of it (a non-finite S or v reads the low edge:
// fmin/fmax return the other operand of a NaN, so the index stays in range).
__device__ __forceinline__ float table_phi(const float* tab, const TableSpec& t, int row, float S,
                                           float v)
{
    const float u = __builtin_fminf(__builtin_fmaxf((S - t.s_lo) * t.s_inv, 0.0f), (float)(t.ns - 1));
    const int i = min((int)u, t.ns - 2);
    const float f = u - (float)i;
    if (t.nv == 1) {
        const float* r = tab + row * t.ns + i;
        return __builtin_fmaf(f, r[1] - r[0], r[0]);
    }
    const float w = __builtin_fminf(__builtin_fmaxf((v - t.v_lo) * t.v_inv, 0.0f), (float)(t.nv - 1));
    const int k = min((int)w, t.nv - 2);
    const float g = w - (float)k;
    const float* r = tab + (row * t.nv + k) * t.ns + i;
    const float a = __builtin_fmaf(f, r[1] - r[0], r[0]);
    const float b = __builtin_fmaf(f, r[t.ns + 1] - r[t.ns], r[t.ns]);
    return __builtin_fmaf(g, b - a, a);
}

// ------------------------------------------------------------- backward
// Gradient of sum_samples w_p * Y_p with respect to the parameters, one
// evaluation point at a time.  With g_p = dLoss/dphi at the point (-w_p dW1
// on the fine path, +w_p dW1c on the coarse path) and dy = scale * g:
//   gb3 += dy,  gw3 += dy h2,  d2 = dy w3 (1 - h2^2),  gb2 += d2,
//   gW2 += d2 h1^T,  d1 = (W2^T d2) (1 - h1^2),  gb1 += d1,  gW1 += d1 x^T.
// d2 is rounded to bf16 where the matrix cores read it (gW2 and W2^T d2),
// and so is h1 in gW2; the derivative 1 - h1^2 uses the fp32 h1.
//
// Lane-local accumulators cover the lane's fixed unit sets (its 32 layer-2
// rows and 32 layer-1 slots, for its two samples); gW2 accumulates in MFMA
// registers: G = sum_p h1[u][p] d2[j][p], i.e. G[u][j] = gW2[j][u], with the
// sample index p as the contraction, staged through LDS (the per-sample
// vectors arrive with p fixed per lane and must be read with p varying).
constexpr int kStageRow = 68;          // bf16 per staged row (64 + pad)

struct GradAcc {
    f32x16 G[2][2];                    // [u tile][j tile]
    float gw3[32], gb2[32];            // rows row_d(h, t / 16, t % 16), t < 32
    float gb1[32], gW1[3][32];         // slots s: units unit_b(h, s)
    float gb3;
};

__device__ __forceinline__ void zero_acc(GradAcc& g)
{
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) g.G[a][b][r] = 0.0f;
#pragma unroll
    for (int t = 0; t < 32; ++t) {
        g.gw3[t] = g.gb2[t] = g.gb1[t] = 0.0f;
        g.gW1[0][t] = g.gW1[1][t] = g.gW1[2][t] = 0.0f;
    }
    g.gb3 = 0.0f;
}

// Staging buffers of one wave: h1 and d2 in bf16, row = sample, column =
// unit (padded rows keep the two lane halves on different banks).
struct Stage {
    __bf16 h1[64 * kStageRow];
    __bf16 d2[64 * kStageRow];
};

// A operand of the backward product e1 = W2^T d2 (permuted), in LDS.
template <int D>
__device__ __forceinline__ void eval_backward(const NetShared& sh, const bf16x8* afwd_lds,
                                              const bf16x8* abwd_lds, Stage& st, float x0, float S,
                                              float v, float g_own, GradAcc& acc)
{
    const int lane = threadIdx.x & 63, h = lane >> 5;
    float x1[2], x2[2];
    pair_inputs<D>(sh, S, v, x1, x2);
    bf16x8 b[2][4];
    float h1f[64];
    layer1<D, true>(sh, x0, x1, x2, b, h1f);
    bf16x8 A[2][4];
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) A[jt][kb] = afwd_lds[(jt * 4 + kb) * 64 + lane];
    f32x16 z[2][2];
    layer2(sh, A, b, z);
    const float g_oth = __shfl_xor(g_own, 32);
    const float dy[2] = {sh.scale * (h == 0 ? g_own : g_oth), sh.scale * (h == 0 ? g_oth : g_own)};
    acc.gb3 += sh.scale * g_own;
    // layer 3 and 2 backward, in place: z becomes d2
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int t = 16 * jt + r;
            const float w3 = sh.w3[row_d(h, jt, r)];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const float hv = tanh_fast(z[jt][nt][r]);
                const float dd = 1.0f - hv * hv;
                acc.gw3[t] = __builtin_fmaf(dy[nt], hv, acc.gw3[t]);
                acc.gb2[t] = __builtin_fmaf(dy[nt], dd, acc.gb2[t]);
                z[jt][nt][r] = dy[nt] * w3 * dd;
            }
        }
    // d2 in bf16, in the register order of the backward product's B operand
    bf16x8 d2b[2][4];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int t = 0; t < 32; ++t) d2b[nt][t / 8][t % 8] = (__bf16)z[t / 16][nt][t % 16];
    // stage h1 (rows: sample, columns: unit) and d2 (rows: sample, columns: j)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const int p = 32 * nt + (lane & 31);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            bf16x8 hv = b[nt][kb];
#pragma unroll
            for (int i = 0; i < 8; ++i) st.h1[p * kStageRow + 16 * kb + 8 * h + i] = hv[i];
        }
#pragma unroll
        for (int t = 0; t < 32; ++t)
            st.d2[p * kStageRow + row_d(h, t / 16, t % 16)] = d2b[nt][t / 8][t % 8];
    }
    // e1 = W2^T d2 on the matrix cores; rows line up with the layer-1 slots
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) A[mt][kb] = abwd_lds[(mt * 4 + kb) * 64 + lane];
    f32x16 e1[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
#pragma unroll
            for (int r = 0; r < 16; ++r) e1[mt][nt][r] = 0.0f;
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
                e1[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[mt][kb], d2b[nt][kb],
                                                                     e1[mt][nt], 0, 0, 0);
        }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int s = 16 * mt + r;
            const float d10 = e1[mt][0][r] * (1.0f - h1f[s] * h1f[s]);
            const float d11 = e1[mt][1][r] * (1.0f - h1f[32 + s] * h1f[32 + s]);
            const float sum = d10 + d11;
            acc.gb1[s] += sum;
            acc.gW1[0][s] = __builtin_fmaf(x0, sum, acc.gW1[0][s]);
            acc.gW1[1][s] = __builtin_fmaf(d10, x1[0], __builtin_fmaf(d11, x1[1], acc.gW1[1][s]));
            if (D == 3)
                acc.gW1[2][s] = __builtin_fmaf(d10, x2[0], __builtin_fmaf(d11, x2[1], acc.gW1[2][s]));
        }
    __syncthreads();
    // gW2 (as G[u][j]) += sum over the 64 samples of h1[u][p] d2[j][p]
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        bf16x8 ah[2], bd[2];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int p = 16 * kb + 8 * h + i;
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                ah[tt][i] = st.h1[p * kStageRow + 32 * tt + (lane & 31)];
                bd[tt][i] = st.d2[p * kStageRow + 32 * tt + (lane & 31)];
            }
        }
#pragma unroll
        for (int ut = 0; ut < 2; ++ut)
#pragma unroll
            for (int jt = 0; jt < 2; ++jt)
                acc.G[ut][jt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ut], bd[jt], acc.G[ut][jt],
                                                                        0, 0, 0);
    }
    __syncthreads();
}

}  // namespace cvnet
}  // namespace mlmc
