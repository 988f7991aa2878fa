// Wavefront -> LDS -> FP64 atomic reduction of per-lane level sums.
//
// The level estimator needs sum Y and sum Y^2 (eq. (eq:Yldef)); fine-level
// differences cancel, so they are kept in fp64 from the lane up.  A wave of 64
// lanes reduces with DPP row operations (quad permutes, row rotates) on the
// two 32-bit halves of each double, then a cross-row exchange; the block's
// waves combine through LDS, and one lane per quantity issues a hardware
// global_atomic_add_f64 into the (payoff, level) record.
//
// Adds from thousands of blocks to one cache line serialise at a few ns each,
// which costs more than the sampling itself for launches of up to a few
// million samples.  A level launch therefore writes into a spread group of
// kSpread records: block b adds into record b mod kSpread, and the group's
// value is the sum of its records (fold_records; the driver folds on the
// device).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlmc {

constexpr int kNumSums = 6;   // Y, Y^2, Pf, Pf^2, Pc, Pc^2

// Record layout in device memory (one per (payoff, level)).
struct LevelAcc {
    double sum[kNumSums];
    unsigned long long n_nonfinite;
    unsigned long long pad;
};

constexpr int kSpread = 64;   // records per spread group (one 64-byte line each)

// Sum of n records, in index order.
__host__ __device__ inline LevelAcc fold_records(const LevelAcc* g, int n)
{
    LevelAcc r = {};
    for (int j = 0; j < n; ++j) {
        for (int k = 0; k < kNumSums; ++k) r.sum[k] += g[j].sum[k];
        r.n_nonfinite += g[j].n_nonfinite;
    }
    return r;
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t bits = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)bits, CTRL, 0xF, 0xF, false);
    const uint32_t hi = __builtin_amdgcn_update_dpp(0u, (uint32_t)(bits >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// DPP control codes (GCN/CDNA encoding).
constexpr int kQuadPerm1032 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kQuadPerm2301 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kRowRor4 = 0x124;       // row_ror:4
constexpr int kRowRor8 = 0x128;       // row_ror:8

__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<kQuadPerm1032>(v);
    v += dpp_f64<kQuadPerm2301>(v);
    v += dpp_f64<kRowRor4>(v);
    v += dpp_f64<kRowRor8>(v);        // every lane holds its 16-lane row sum
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

__device__ __forceinline__ unsigned wave_sum_u32(unsigned v)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// Block-wide reduction of kNumSums doubles and a count; adds into acc.
// Every thread of the block must call it.  LDS: (blockDim/64) * 7 doubles.
__device__ __forceinline__ void block_reduce_add(const double (&s)[kNumSums], unsigned nonfinite,
                                                 LevelAcc* acc)
{
    __shared__ double red[16][kNumSums + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < kNumSums; ++i) {
        const double w = wave_sum(s[i]);
        if (lane == 0) red[wave][i] = w;
    }
    const unsigned c = wave_sum_u32(nonfinite);
    if (lane == 0) red[wave][kNumSums] = (double)c;
    __syncthreads();
    if (threadIdx.x <= kNumSums) {
        double t = 0.0;
        for (int w = 0; w < nwaves; ++w) t += red[w][threadIdx.x];
        if (threadIdx.x < kNumSums) {
            if (t != 0.0) atomicAdd(&acc->sum[threadIdx.x], t);
        } else if (t != 0.0) {
            atomicAdd(&acc->n_nonfinite, (unsigned long long)t);
        }
    }
    __syncthreads();
}

}  // namespace mlmc
