// rng.h -- per-step building blocks shared by the walk kernels: Philox
// counters, uniforms, Box-Muller normals, the update and the exit test
// (Sec. 2.2: Euler-Maruyama with pseudo-random normals and an exit test at
// the end of every step).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace sdd {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// Philox4x32-10 (Salmon et al., SC'11).  The key schedule is wave-uniform;
// each three-input XOR is one v_bitop3_b32 (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Uniform from the low 23 bits of a word: u = ((r & 0x7fffff) + 1/2) 2^-23,
// exact in float and double.  In float it is built as the bit pattern
// 1 + m 2^-23 (one v_and_or_b32) minus (1 - 2^-24), an exact subtraction.
__device__ __forceinline__ float uniform_f32(uint32_t r)
{
    return __uint_as_float((r & 0x007fffffu) | 0x3f800000u) - 0x1.fffffep-1f;
}

// Box-Muller pair (z0, z1) = sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b).
// The float version returns the pair scaled by 1/sqrt(2 ln 2),
// sqrt(-log2 u_a) (cos, sin), and the caller folds sqrt(2 ln 2) into the
// step's noise factor; v_sin/v_cos take their argument in turns.
__device__ __forceinline__ void normals(uint32_t ra, uint32_t rb, float& z0, float& z1)
{
    const float ua = uniform_f32(ra);
    const float ub = uniform_f32(rb);
    const float radius = __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(ua));
    z0 = radius * __builtin_amdgcn_cosf(ub);
    z1 = radius * __builtin_amdgcn_sinf(ub);
}

__device__ __forceinline__ void normals(uint32_t ra, uint32_t rb, double& z0, double& z1)
{
    const double ua = ((double)(ra & 0x007fffffu) + 0.5) * 0x1p-23;
    const double ub = ((double)(rb & 0x007fffffu) + 0.5) * 0x1p-23;
    const double radius = sqrt(-2.0 * log(ua));
    double sn, cs;
    sincos(kTwoPi * ub, &sn, &cs);
    z0 = radius * cs;
    z1 = radius * sn;
}

__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Outside the open square: x <= 0, x >= 1 (or NaN) for either coordinate.
// For a float, 0 < x < 1 exactly when its bit pattern minus one is below
// that of 1.0f minus one (unsigned), which costs no NaN canonicalisation.
__device__ __forceinline__ bool outside(float x, float y)
{
    const uint32_t bx = __float_as_uint(x) - 1u, by = __float_as_uint(y) - 1u;
    return (bx > by ? bx : by) >= 0x3f7fffffu;
}
__device__ __forceinline__ bool outside(double x, double y) { return x <= 0.0 || x >= 1.0 || y <= 0.0 || y >= 1.0; }


}  // namespace sdd
