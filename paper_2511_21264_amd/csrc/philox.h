// Counter-based Gaussian noise for the sampling step of Alg. 1.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 32x32->64 multiplies with Weyl-sequence key bumps between rounds.
// Counter (sample j, control step k, quad q, iteration m), key = 64-bit
// seed.  Each word w becomes a uniform ((w >> 8) + 1) * 2^-24 in (0, 1],
// exact in FP32; pairs of uniforms become normals by Box-Muller.  Quads
// q = 0..3 give 16 normals, the first 14 drive the 14 joints.  Nothing is
// stored: the rollout and the update regenerate the same values.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mppi {

struct U4 {
    uint32_t x, y, z, w;
};

__host__ __device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
    constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kM0 * c.x;
        const uint64_t p1 = (uint64_t)kM1 * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += kW0;
        k1 += kW1;
    }
    return c;
}

__device__ __forceinline__ float u24(uint32_t w) { return (float)((w >> 8) + 1u) * 5.9604644775390625e-8f; }

__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float &z0, float &z1)
{
    const float rad = sqrtf(-2.0f * logf(u24(a)));
    float s, c;
    sincospif(2.0f * u24(b), &s, &c);
    z0 = rad * c;
    z1 = rad * s;
}

// The 14 standard normals of (j, k, m).
__device__ __forceinline__ void normals14(uint32_t key0, uint32_t key1, uint32_t j, uint32_t k, uint32_t m,
                                          float z[14])
{
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
        const U4 w = philox4x32_10(U4{j, k, q, m}, key0, key1);
        box_muller(w.x, w.y, z[4 * q], z[4 * q + 1]);
        if (q < 3) box_muller(w.z, w.w, z[4 * q + 2], z[4 * q + 3]);
    }
}

}  // namespace mppi
