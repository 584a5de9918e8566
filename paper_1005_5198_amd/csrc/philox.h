// Counter-based random ray positions (the GPU code's random sampling, Section 3.1).
//
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds, each multiplying two of the four
// 64-bit counter words by the published constants into 128-bit products and
// mixing the halves with the other words and the key; the key is bumped by
// the published Weyl constants between rounds.
//
// Ray (i, j) of a map with seed s uses the block at counter (j nx + i, 0, 0, 0)
// and key (s, 0); its uniforms are U = ((word >> 12) + 1/2) 2^-52 of words 0
// and 1, strictly inside (0, 1) and exact in FP64, and it sits at
// x1 = sx0 + U1 sw, x2 = sy0 + U2 sh (two FP64 operations each, no contraction).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace rs {

struct PhiloxOut {
    uint64_t w0, w1;
};

__device__ __forceinline__ PhiloxOut philox4x64_10_w01(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                        uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return PhiloxOut{c0, c1};
}

__device__ __forceinline__ void random_ray_xy(double sx0, double sy0, double sw, double sh, int64_t nx,
                                              uint64_t seed, int64_t i, int64_t j, double &x1, double &x2) {
    const uint64_t k = (uint64_t)j * (uint64_t)nx + (uint64_t)i;
    const PhiloxOut o = philox4x64_10_w01(k, 0ull, 0ull, 0ull, seed, 0ull);
    const double u1 = ((double)(o.w0 >> 12) + 0.5) * 0x1p-52;
    const double u2 = ((double)(o.w1 >> 12) + 0.5) * 0x1p-52;
    x1 = sx0 + u1 * sw;
    x2 = sy0 + u2 * sh;
}

}  // namespace rs
