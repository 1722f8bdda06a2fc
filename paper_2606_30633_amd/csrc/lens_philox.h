// Counter-based random numbers on the device: Philox4x32-10 (Salmon, Moraes,
// Dror & Shaw 2011, "Parallel random numbers: as easy as 1, 2, 3"), the one
// generator of every kernel that draws (HMC momenta and accept uniforms, SVI
// surrogate draws, network initialisation, image noise, proposals).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace lens {

// Ten rounds of two 32x32-bit multiplications whose high and low halves are
// mixed into the four counter words, with a Weyl-sequence key schedule.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k.x += W0; k.y += W1; }
        const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
        const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    }
    return c;
}

__device__ __forceinline__ uint2 philox_key(uint64_t seed) {
    return make_uint2((uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
}

// Uniform on (0, 1) from the top 24 bits of a word (never 0 or 1).
__device__ __forceinline__ double philox_uniform01(uint32_t w) {
    return ((double)(w >> 8) + 0.5) * (1.0 / 16777216.0);
}

// Box-Muller: two words -> two standard normals (float64).
__device__ __forceinline__ void philox_box_muller(uint32_t a, uint32_t b, double& z0, double& z1) {
    const double r = sqrt(-2.0 * log(philox_uniform01(a)));
    const double ang = 6.283185307179586476925 * philox_uniform01(b);
    z0 = r * cos(ang);
    z1 = r * sin(ang);
}

}  // namespace lens
