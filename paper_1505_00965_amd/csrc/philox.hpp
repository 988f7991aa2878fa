// Counter-based Philox4x32-10 generator, uniforms and Box--Muller normals for
// gfx950.
//
// The method needs fresh independent normals per level, with the coarse path
// reusing the fine path's increments (Sec. 5, after eq. (eq:Yldef)).  Philox
// (Salmon, Moraes, Dror, Shaw, SC'11) makes every number a pure function of
// (key, counter), so a path is regenerated anywhere, by any thread, from its
// index alone: nothing is stored, and results do not depend on the launch
// shape.  Written from the publication: ten rounds of two 32x32->64 products
// of counter words 0 and 2 by the round multipliers, the high halves xored
// with the other two counter words and the key, the key bumped by the Weyl
// constants between rounds.
//
// Counter layout: word 0 = block j along the path (4 outputs per block),
// word 1 = path index mod 2^32, word 2 = level + 256 * (path index >> 32),
// word 3 = stream.  Key = (seed mod 2^32, seed >> 32).  Words 0, 2, 3 and
// the key are uniform across a wavefront, so the first round's products run
// on the scalar unit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlmc {

enum Stream : uint32_t {
    kStreamNormal = 0,
    kStreamBridge = 1,
    kStreamTrainNormal = 2,
    kStreamTrainBridge = 3,
    kStreamStdMC = 4,
    kStreamStdMCBridge = 5,
    kStreamInit = 6,
    kStreamLevelDraw = 7,   // levels drawn by the randomised estimator
};

struct u32x4 {
    uint32_t x, y, z, w;
};

// Three-input xor in one VALU instruction (gfx950 v_bitop3_b32, truth
// table 0x96 = a ^ b ^ c): halves the xor count of a round.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)kMulA * c.x;
        const uint64_t pb = (uint64_t)kMulB * c.z;
        u32x4 n;
        n.x = xor3((uint32_t)(pb >> 32), c.y, k0);
        n.y = (uint32_t)pb;
        n.z = xor3((uint32_t)(pa >> 32), c.w, k1);
        n.w = (uint32_t)pa;
        c = n;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return c;
}

struct PathKey {
    uint32_t k0, k1;      // key from the seed
    uint32_t s_lo;        // path index low word (counter word 1)
    uint32_t c2;          // level + 256 * path-index high bits
    uint32_t stream;      // counter word 3
};

__host__ __device__ __forceinline__ PathKey make_path_key(uint64_t seed, int level, uint64_t s,
                                                          uint32_t stream)
{
    PathKey p;
    p.k0 = (uint32_t)seed;
    p.k1 = (uint32_t)(seed >> 32);
    p.s_lo = (uint32_t)s;
    p.c2 = (uint32_t)level + 256u * (uint32_t)(s >> 32);
    p.stream = stream;
    return p;
}

__device__ __forceinline__ u32x4 path_block(const PathKey& p, uint32_t j)
{
    return philox4x32_10(u32x4{j, p.s_lo, p.c2, p.stream}, p.k0, p.k1);
}

// ((x >> 8) + 1/2) * 2^-24: exact in fp32 and fp64, strictly inside (0, 1).
__device__ __forceinline__ float u01f(uint32_t x)
{
    return __builtin_fmaf((float)(x >> 8), 0x1p-24f, 0x1p-25f);
}
__device__ __forceinline__ double u01d(uint32_t x)
{
    return __builtin_fma((double)(x >> 8), 0x1p-24, 0x1p-25);
}

// Box--Muller in fp32 on the hardware transcendental units: v_log_f32 is
// log2, v_sin_f32 / v_cos_f32 take their argument in turns, so
// sin(2 pi u) is one instruction.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& z0, float& z1)
{
    const float u1 = u01f(a), u2 = u01f(b);
    // -2 ln u1 = -2 ln2 * log2(u1)
    const float rho = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
    z0 = rho * __builtin_amdgcn_cosf(u2);
    z1 = rho * __builtin_amdgcn_sinf(u2);
}

__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1)
{
    const double u1 = u01d(a), u2 = u01d(b);
    const double rho = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z0 = rho * c;
    z1 = rho * s;
}

}  // namespace mlmc
