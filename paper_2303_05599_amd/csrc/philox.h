// philox.h -- Philox4x64-10 counter-based generator (Salmon, Moraes, Dror,
// Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), device side.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace cpic {

struct u64x4 {
    uint64_t v[4];
};

__device__ __forceinline__ u64x4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                            uint64_t k1)
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    return {{c0, c1, c2, c3}};
}

// uniform in [0, 1) and (0, 1] from the top 53 bits
__device__ __forceinline__ double u01_co(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }
__device__ __forceinline__ double u01_oc(uint64_t r) { return (double)((r >> 11) + 1) * 0x1.0p-53; }

// Box-Muller pair from two words: radius from the first, angle from the second
__device__ __forceinline__ void box_muller(uint64_t ra, uint64_t rb, double& z0, double& z1)
{
    const double rad = sqrt(-2.0 * log(u01_oc(ra)));
    const double ang = 2.0 * M_PI * u01_co(rb);
    z0 = rad * cos(ang);
    z1 = rad * sin(ang);
}

}  // namespace cpic
