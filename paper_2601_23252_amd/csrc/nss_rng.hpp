// Counter-based random numbers for the chains: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), implemented from that definition.
//
// Every draw is addressed by (purpose, index, iteration, step, draw): counter
// (purpose<<24 | index, iteration, step, draw), key (seed_lo, seed_hi ^ run_id).  Results
// therefore do not depend on how chains are scheduled onto workgroups.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nss {

enum Purpose : uint32_t {
    PUR_INIT = 1,      // prior draws of the initial live set (index = particle)
    PUR_RESAMPLE = 2,  // parent choice (index = chain)
    PUR_DIR = 3,       // direction normals (index = chain, draw = pair of coordinates)
    PUR_STEP = 4,      // initial bracket offset and slice height (index = chain)
    PUR_SHRINK = 5     // shrinkage proposals (index = chain, draw = proposal number)
};

__device__ __forceinline__ void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2,
                                              uint32_t &c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
}

// Uniform in (0,1) from a 64-bit word: (2*(x>>12)+1) * 2^-53, exact in FP64.
__device__ __forceinline__ double u53(uint32_t lo, uint32_t hi)
{
    const uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
    return (double)(2ull * (x >> 12) + 1ull) * 0x1p-53;
}

__device__ __forceinline__ void draw2(uint32_t k0, uint32_t k1, uint32_t purpose, uint32_t index,
                                      uint32_t c1, uint32_t c2, uint32_t c3, double &ua,
                                      double &ub)
{
    uint32_t a = (purpose << 24) | (index & 0xFFFFFFu), b = c1, c = c2, d = c3;
    philox4x32_10(a, b, c, d, k0, k1);
    ua = u53(a, b);
    ub = u53(c, d);
}

// Box-Muller: z0 = sqrt(-2 ln ua) cos(2 pi ub), z1 = sqrt(-2 ln ua) sin(2 pi ub).
__device__ __forceinline__ void box_muller(double ua, double ub, double &z0, double &z1)
{
    const double rad = sqrt(-2.0 * log(ua));
    double s, c;
    sincospi(2.0 * ub, &s, &c);  // sin / cos of 2 pi ub without an argument reduction
    z0 = rad * c;
    z1 = rad * s;
}

}  // namespace nss
