// Wave-level helpers shared by the gfx950 kernels: reductions over a wave or over the 16 lanes
// of a DPP row, lane broadcasts, and the wave-local LDS ordering fence.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace nss {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

#define LOG_2PI 1.8378770664093454836

// ------------------------------------------------------------------------------------------
// wave helpers
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_sumf(float v)
{
#pragma unroll
    for (int o = 32; o; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_maxf(float v)
{
#pragma unroll
    for (int o = 32; o; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
// Make this wave's LDS writes visible to its own other lanes.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// Reductions over the 16 lanes of a DPP row with VALU data movement (quad swaps, half-row and
// row mirrors); every lane of the row ends with the same result.
template <int CTRL>
__device__ __forceinline__ float dppf(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dppd(double v)
{
    int2 p = __builtin_bit_cast(int2, v);
    p.x = __builtin_amdgcn_update_dpp(0, p.x, CTRL, 0xF, 0xF, false);
    p.y = __builtin_amdgcn_update_dpp(0, p.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, p);
}
#define DPP_XOR1 0xB1   /* quad_perm [1,0,3,2] */
#define DPP_XOR2 0x4E   /* quad_perm [2,3,0,1] */
#define DPP_HMIR 0x141  /* row_half_mirror */
#define DPP_RMIR 0x140  /* row_mirror */
__device__ __forceinline__ float row_sum16(float v)
{
    v += dppf<DPP_XOR1>(v); v += dppf<DPP_XOR2>(v); v += dppf<DPP_HMIR>(v); v += dppf<DPP_RMIR>(v);
    return v;
}
__device__ __forceinline__ float row_max16(float v)
{
    v = fmaxf(v, dppf<DPP_XOR1>(v)); v = fmaxf(v, dppf<DPP_XOR2>(v));
    v = fmaxf(v, dppf<DPP_HMIR>(v)); v = fmaxf(v, dppf<DPP_RMIR>(v));
    return v;
}
__device__ __forceinline__ double row_sum16(double v)
{
    v += dppd<DPP_XOR1>(v); v += dppd<DPP_XOR2>(v); v += dppd<DPP_HMIR>(v); v += dppd<DPP_RMIR>(v);
    return v;
}
__device__ __forceinline__ double row_max16(double v)
{
    v = fmax(v, dppd<DPP_XOR1>(v)); v = fmax(v, dppd<DPP_XOR2>(v));
    v = fmax(v, dppd<DPP_HMIR>(v)); v = fmax(v, dppd<DPP_RMIR>(v));
    return v;
}
__device__ __forceinline__ double readlane_d(double v, int lane)
{
    int2 p = __builtin_bit_cast(int2, v);
    p.x = __builtin_amdgcn_readlane(p.x, lane);
    p.y = __builtin_amdgcn_readlane(p.y, lane);
    return __builtin_bit_cast(double, p);
}
__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uniform_d(double v) { return readlane_d(v, 0); }

// Sum over the wave: row sums, then the four row results combined as (r0 + r1) + (r2 + r3)
// in every lane.  The result stays in vector registers: lane broadcasts into scalar registers
// (readlane) that then feed floating-point compares have been compiled into selects that read
// the scalar condition code instead of the compare's result, so decision data never goes
// through them.
__device__ __forceinline__ double wave_sum_fast(double v)
{
    v = row_sum16(v);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

__device__ __forceinline__ double sanitize(double L, unsigned long long &nonfinite)
{
    if (L != L || L == INFINITY) { ++nonfinite; return -INFINITY; }
    return L;
}

}  // namespace nss
