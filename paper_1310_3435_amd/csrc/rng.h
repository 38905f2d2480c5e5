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

// The uniforms of one Philox block (Sec. 2.2 asks only for parallel
// pseudo-random numbers; reading): the block of counter (m, p, g, 0) serves
// steps 3m, 3m+1, 3m+2 with two 21-bit fields each, u = (b + 1/2) 2^-21,
// exact in float and double:
//   step 3m:   hi(w0), hi(w1)      hi(w) = w >> 11
//   step 3m+1: hi(w2), hi(w3)
//   step 3m+2: lo(w0, w1), lo(w2, w3)   lo(w, v) = (w & 0x7ff) | (v & 0x3ff) << 11
// In float the field becomes the mantissa of 1 + b 2^-21, and subtracting
// 1 - 2^-22 is exact.
__device__ __forceinline__ float field_hi(uint32_t w, float)
{
    return __uint_as_float(((w >> 9) & 0x007ffffcu) | 0x3f800000u) - 0x1.fffff8p-1f;
}
__device__ __forceinline__ float field_lo(uint32_t w, uint32_t v, float)
{
    return __uint_as_float(((w & 0x7ffu) << 2) | ((v & 0x3ffu) << 13) | 0x3f800000u) - 0x1.fffff8p-1f;
}
__device__ __forceinline__ double field_hi(uint32_t w, double) { return ((double)(w >> 11) + 0.5) * 0x1p-21; }
__device__ __forceinline__ double field_lo(uint32_t w, uint32_t v, double)
{
    return ((double)((w & 0x7ffu) | ((v & 0x3ffu) << 11)) + 0.5) * 0x1p-21;
}

// Uniform of the bridge test from a word of the block with counter word 3
// = 1: u = ((q & 0x7fffff) + 1/2) 2^-23, exact in float and double; in
// float one v_and_or_b32 and an exact subtraction.
__device__ __forceinline__ float uniform23(uint32_t q, float)
{
    return __uint_as_float((q & 0x007fffffu) | 0x3f800000u) - 0x1.fffffep-1f;
}
__device__ __forceinline__ double uniform23(uint32_t q, double) { return ((double)(q & 0x007fffffu) + 0.5) * 0x1p-23; }

// Exponential time stepping (Sec. 2.2): the length of step 3m + j is an
// exponential variate with mean dt (rate 1/dt), tau = -ln(u) dt, u from
// word j of the block of counter (m, p, g, 2) as uniform23 forms it.
// Float: c = dt ln 2, so that tau = -log2(u) c on the transcendental unit.
__device__ __forceinline__ float expo_step(uint32_t q, float c) { return -__builtin_amdgcn_logf(uniform23(q, 0.0f)) * c; }
__device__ __forceinline__ double expo_step(uint32_t q, double dt) { return -log(uniform23(q, 0.0)) * dt; }

// Box-Muller pair (z0, z1) = sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b).
// The float version returns the pair scaled by 1/sqrt(2 ln 2),
// sqrt(-log2 u_a) (cos, sin), and the caller folds sqrt(2 ln 2) into the
// step's noise factor; v_sin/v_cos take their argument in turns.
__device__ __forceinline__ void normals(float ua, float ub, float& z0, float& z1)
{
    const float radius = __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(ua));
    z0 = radius * __builtin_amdgcn_cosf(ub);
    z1 = radius * __builtin_amdgcn_sinf(ub);
}

__device__ __forceinline__ void normals(double ua, double ub, double& z0, double& z1)
{
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

// Brownian-bridge exit probability of one step P -> Q with both ends
// inside (the conditional exit probability of Sec. 2.2).  Each coordinate of
// the bridge is an independent one-dimensional bridge with diffusion
// coefficient 2, and one that starts a and ends b away from a wall hits it
// within dt with probability exp(-a b / dt); per axis the nearer wall
// counts, and the step exits with probability p_xi + p_eta - p_xi p_eta.
// The step exits when its bridge uniform u (uniform23 above) is below it.
//
// Float: c = -log2(e) / dt.
__device__ __forceinline__ float bridge_prob(float px, float py, float qx, float qy, float c)
{
    const float mx = __builtin_fminf(px * qx, (1.0f - px) * (1.0f - qx));
    const float my = __builtin_fminf(py * qy, (1.0f - py) * (1.0f - qy));
    const float pxi = __builtin_amdgcn_exp2f(mx * c), peta = __builtin_amdgcn_exp2f(my * c);
    return __builtin_fmaf(-pxi, peta, pxi + peta);
}

// Double: c = dt.
__device__ __forceinline__ double bridge_prob(double px, double py, double qx, double qy, double c)
{
    const double m0 = px * qx, m1 = (1.0 - px) * (1.0 - qx);
    const double m2 = py * qy, m3 = (1.0 - py) * (1.0 - qy);
    const double pxi = exp(-(m0 <= m1 ? m0 : m1) / c), peta = exp(-(m2 <= m3 ? m2 : m3) / c);
    return __builtin_fma(-pxi, peta, pxi + peta);
}

// No bridge uniform is below 2^-24 (q = 0 gives (0 + 1/2) 2^-23), so a step
// whose exit probability is at most 2^-24 never exits by the bridge, and
// its uniform need not be drawn: a wave skips the bridge block when none of
// its lanes has a larger probability.  The decisions are unchanged.
template <typename R>
__device__ __forceinline__ bool bridge_may_exit(R prob) { return prob > R(0x1p-24); }

// Side a bridged exit leaves through: the nearer wall of the axis with the
// larger probability, xi on ties (the walk's own precision decides).
template <typename R>
__device__ __forceinline__ uint32_t bridge_side(R px, R py, R qx, R qy)
{
    const R m0 = px * qx, m1 = (R(1) - px) * (R(1) - qx);
    const R m2 = py * qy, m3 = (R(1) - py) * (R(1) - qy);
    const R mx = m0 <= m1 ? m0 : m1, my = m2 <= m3 ? m2 : m3;
    return mx <= my ? (m0 <= m1 ? 0u : 1u) : (m2 <= m3 ? 2u : 3u);
}

}  // namespace sdd
