// common.h -- device-side building blocks of the HIP library (gfx950).
//
// Density of the linear Winslow generator (eq. (5): w > 0) and the drift
// grad w / w of its diffusion (eq. (6)/(7b)), the boundary map (Dirichlet
// data of eq. (5)) and the exit point of a finished Euler-Maruyama step
// (Sec. 2.2).  Float versions use the CDNA transcendental unit directly
// (v_exp_f32 is 2^x, v_log_f32 is log2, v_sin/v_cos take turns); double
// versions use the device math library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sdd.h"

namespace sdd {

constexpr int kWave = 64;
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kInvTwoPi = 0.15915494309189535f;

// Density in the layout the kernels read: per-term parameters as arrays so
// that a wave-uniform term loop indexes kernel arguments (SGPRs).
struct Density {
    int32_t n_terms;
    int32_t kind[SDD_MAX_TERMS];
    double base;
    double amp[SDD_MAX_TERMS], coef[SDD_MAX_TERMS], cx[SDD_MAX_TERMS], cy[SDD_MAX_TERMS];
    double r0[SDD_MAX_TERMS], nx[SDD_MAX_TERMS], ny[SDD_MAX_TERMS];
    // float copies for the float walk; k2 = -coef * log2(e) so that
    // exp(-coef t) = 2^(k2 t)
    float fbase;
    float famp[SDD_MAX_TERMS], fcoef[SDD_MAX_TERMS], fk2[SDD_MAX_TERMS], fcx[SDD_MAX_TERMS];
    float fcy[SDD_MAX_TERMS], fr0[SDD_MAX_TERMS], fnx[SDD_MAX_TERMS], fny[SDD_MAX_TERMS];
    // la = log2(amp) (amp e^{-c t} = 2^(k2 t + la)), m2c = -2 coef
    float fla[SDD_MAX_TERMS], fm2c[SDD_MAX_TERMS];
    // single-term sech^2 and sin^2 walks: the argument as a plane
    // pa xi + pb eta + pc in the unit of its transcendental (sech^2:
    // 2 log2(e) s, so that e^{-2|s|} = 2^-|.|; sin^2: s / (2 pi) turns), the
    // Horner constant sd = 2 base + 4 amp (sech^2) and the gradient factors
    // gx, gy that multiply the term's scalar factor
    float fpa[SDD_MAX_TERMS], fpb[SDD_MAX_TERMS], fpc[SDD_MAX_TERMS], fsd[SDD_MAX_TERMS];
    float fgx[SDD_MAX_TERMS], fgy[SDD_MAX_TERMS];
};

struct Bmap {
    int32_t kind;
    int32_t n;
    double p[8];
    const double* table;
};

// ------------------------------------------------------------------ density

// One density term's value and gradient added into (W, Gx, Gy), double.
template <int KIND>
__device__ inline void term_f64(const Density& D, int t, double xi, double eta, double& W, double& Gx, double& Gy)
{
    const double dx = xi - D.cx[t], dy = eta - D.cy[t];
    const double a = D.amp[t], c = D.coef[t];
    if (KIND == SDD_TERM_GAUSS) {
        const double e = a * exp(-c * (dx * dx + dy * dy));
        W += e;
        const double g = -2.0 * c * e;
        Gx += g * dx;
        Gy += g * dy;
    } else if (KIND == SDD_TERM_RING) {
        const double r = sqrt(dx * dx + dy * dy);
        const double d = r - D.r0[t];
        const double e = a * exp(-c * d * d);
        W += e;
        if (r > 0.0) {
            const double g = -2.0 * c * d * e / r;
            Gx += g * dx;
            Gy += g * dy;
        }
    } else if (KIND == SDD_TERM_SECH2) {
        // sech^2 s = 4q/(1+q)^2, tanh s = sign(s)(1-q)/(1+q), q = e^{-2|s|}
        const double s = c * (D.nx[t] * dx + D.ny[t] * dy);
        const double q = exp(-2.0 * fabs(s));
        const double inv = 1.0 / (1.0 + q);
        const double f = a * 4.0 * q * inv * inv;
        const double th = copysign((1.0 - q) * inv, s);
        W += f;
        const double g = -2.0 * f * th * c;
        Gx += g * D.nx[t];
        Gy += g * D.ny[t];
    } else if (KIND == SDD_TERM_SIN2) {
        const double s = c * (D.nx[t] * dx + D.ny[t] * dy);
        double sn, cs;
        sincos(s, &sn, &cs);
        W += a * sn * sn;
        const double g = 2.0 * a * sn * cs * c;
        Gx += g * D.nx[t];
        Gy += g * D.ny[t];
    }
}

// w and grad w in double.  KIND >= 0: a single term of that kind (known at
// compile time); KIND = kAnyTerms: the general sum over D.n_terms terms.
// kGaussSum (float walks only): a sum of Gaussian bumps, gauss_sum_drift.
constexpr int kAnyTerms = -1;
constexpr int kGaussSum = -2;

template <int KIND = kAnyTerms>
__device__ inline void density_grad(const Density& D, double xi, double eta, double& w, double& gx, double& gy)
{
    double W = D.base, Gx = 0.0, Gy = 0.0;
    if (KIND >= 0) {
        term_f64<KIND>(D, 0, xi, eta, W, Gx, Gy);
    } else {
        for (int t = 0; t < D.n_terms; ++t) {
            switch (D.kind[t]) {
            case SDD_TERM_GAUSS: term_f64<SDD_TERM_GAUSS>(D, t, xi, eta, W, Gx, Gy); break;
            case SDD_TERM_RING: term_f64<SDD_TERM_RING>(D, t, xi, eta, W, Gx, Gy); break;
            case SDD_TERM_SECH2: term_f64<SDD_TERM_SECH2>(D, t, xi, eta, W, Gx, Gy); break;
            case SDD_TERM_SIN2: term_f64<SDD_TERM_SIN2>(D, t, xi, eta, W, Gx, Gy); break;
            default: break;
            }
        }
    }
    w = W;
    gx = Gx;
    gy = Gy;
}

__device__ inline double density_value(const Density& D, double xi, double eta)
{
    double w, gx, gy;
    density_grad(D, xi, eta, w, gx, gy);
    return w;
}

// One term in float, on the transcendental unit.
template <int KIND>
__device__ inline void term_f32(const Density& D, int t, float xi, float eta, float& W, float& Gx, float& Gy)
{
    const float dx = xi - D.fcx[t], dy = eta - D.fcy[t];
    const float a = D.famp[t], c = D.fcoef[t];
    if (KIND == SDD_TERM_GAUSS) {
        const float e = a * __builtin_amdgcn_exp2f(D.fk2[t] * (dx * dx + dy * dy));
        W += e;
        const float g = -2.0f * c * e;
        Gx += g * dx;
        Gy += g * dy;
    } else if (KIND == SDD_TERM_RING) {
        const float r2 = dx * dx + dy * dy;
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float r = (r2 > 0.0f) ? r2 * rinv : 0.0f;  // rsq(0) = inf
        const float d = r - D.fr0[t];
        const float e = a * __builtin_amdgcn_exp2f(D.fk2[t] * d * d);
        W += e;
        const float g = (r2 > 0.0f) ? (-2.0f * c * d * e * rinv) : 0.0f;
        Gx += g * dx;
        Gy += g * dy;
    } else if (KIND == SDD_TERM_SECH2) {
        const float s = c * (D.fnx[t] * dx + D.fny[t] * dy);
        const float q = __builtin_amdgcn_exp2f(-2.0f * kLog2e * fabsf(s));
        const float inv = __builtin_amdgcn_rcpf(1.0f + q);
        const float f = a * 4.0f * q * inv * inv;
        const float th = copysignf((1.0f - q) * inv, s);
        W += f;
        const float g = -2.0f * f * th * c;
        Gx += g * D.fnx[t];
        Gy += g * D.fny[t];
    } else if (KIND == SDD_TERM_SIN2) {
        const float s = c * (D.fnx[t] * dx + D.fny[t] * dy);
        float turns = s * kInvTwoPi;
        turns = turns - floorf(turns);
        const float sn = __builtin_amdgcn_sinf(turns);
        const float cs = __builtin_amdgcn_cosf(turns);
        W += a * sn * sn;
        const float g = 2.0f * a * sn * cs * c;
        Gx += g * D.fnx[t];
        Gy += g * D.fny[t];
    }
}

// Float parameters of a sum of up to SDD_MAX_TERMS Gaussian bumps in the
// form gauss_sum_drift reads: amp e^{-c r^2} = 2^(k2 r^2 + la), m2c = -2c.
struct GaussParams {
    int32_t n_terms;
    float base;
    float cx[SDD_MAX_TERMS], cy[SDD_MAX_TERMS], k2[SDD_MAX_TERMS], la[SDD_MAX_TERMS], m2c[SDD_MAX_TERMS];
};

// drift b = grad w / w in float of w = base + sum of Gaussian bumps, the
// terms taken in order; with m2c times the step length (fixed steps) it is
// b dt.  The walk of an estimate call (parameters in scalar registers) and
// the request server's walk (parameters per lane) both evaluate exactly
// this sequence of operations, so a request walks bit for bit the paths an
// estimate call walks.
__device__ __forceinline__ void gauss_sum_drift(int n, float base, const float* cx, const float* cy, const float* k2,
                                                const float* la, const float* m2c, float x, float y, float& bx,
                                                float& by)
{
    float W = base, Gx = 0.0f, Gy = 0.0f;
#pragma unroll
    for (int q = 0; q < SDD_MAX_TERMS; ++q) {
        if (q < n) {
            const float dx = x - cx[q], dy = y - cy[q];
            const float e = __builtin_amdgcn_exp2f(__builtin_fmaf(k2[q], __builtin_fmaf(dx, dx, dy * dy), la[q]));
            W += e;
            const float h = m2c[q] * e;
            Gx = __builtin_fmaf(h, dx, Gx);
            Gy = __builtin_fmaf(h, dy, Gy);
        }
    }
    const float iw = __builtin_amdgcn_rcpf(W);
    bx = Gx * iw;
    by = Gy * iw;
}

// drift b = grad w / w in float for a single ring, sech^2 or sin^2 term,
// times `scale` (the step length for fixed steps, so that the update's
// X + b dt is one FMA per coordinate; 1 otherwise), written so that 1/w
// goes into one common factor h: b = h (d_xi, d_eta) for the ring (its
// amplitude folded into the exponent), b = h (gx, gy) for sech^2 and
// sin^2, whose argument is one plane in (xi, eta).  The constants times
// scale are loop invariants of the walk.
template <int KIND>
__device__ inline void drift1_f32(const Density& D, float scale, float xi, float eta, float& bx, float& by)
{
    const float dx = xi - D.fcx[0], dy = eta - D.fcy[0];
    if (KIND == SDD_TERM_RING) {
        // r^2 clamped away from 0: at the centre d_xi = d_eta = 0 and b = 0
        const float r2 = fmaxf(__builtin_fmaf(dx, dx, dy * dy), 1e-30f);
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float d = __builtin_fmaf(r2, rinv, -D.fr0[0]);
        const float e = __builtin_amdgcn_exp2f(__builtin_fmaf(D.fk2[0] * d, d, D.fla[0]));
        const float h = (D.fm2c[0] * scale) * d * e * rinv * __builtin_amdgcn_rcpf(D.fbase + e);
        bx = h * dx;
        by = h * dy;
    } else if (KIND == SDD_TERM_SECH2) {
        // with q = e^{-2|s|}: sech^2 s = 4q/(1+q)^2 and tanh|s| = (1-q)/(1+q),
        // so f tanh s / (base + f), f = amp sech^2 s, is
        //   sign(s) 4 amp q (1-q) / ((1+q) (base (1+q)^2 + 4 amp q)),
        // with base (1+q)^2 + 4 amp q = base + q (2 base + 4 amp + base q):
        // one reciprocal, and 4 amp m2c n in the gradient factors
        const float s2 = __builtin_fmaf(D.fpa[0], xi, __builtin_fmaf(D.fpb[0], eta, D.fpc[0]));
        const float q = __builtin_amdgcn_exp2f(-fabsf(s2));
        const float dq = __builtin_fmaf(q, __builtin_fmaf(D.fbase, q, D.fsd[0]), D.fbase);
        const float den = __builtin_fmaf(q, dq, dq);
        const float h = copysignf(__builtin_fmaf(-q, q, q) * __builtin_amdgcn_rcpf(den), s2);
        bx = h * (D.fgx[0] * scale);
        by = h * (D.fgy[0] * scale);
    } else {  // SIN2
        float turns = __builtin_fmaf(D.fpa[0], xi, __builtin_fmaf(D.fpb[0], eta, D.fpc[0]));
        turns = turns - floorf(turns);
        const float sn = __builtin_amdgcn_sinf(turns);
        const float cs = __builtin_amdgcn_cosf(turns);
        const float h = sn * cs * __builtin_amdgcn_rcpf(__builtin_fmaf(D.famp[0] * sn, sn, D.fbase));
        bx = h * (D.fgx[0] * scale);
        by = h * (D.fgy[0] * scale);
    }
}

// drift b = grad w / w in float, times scale (see drift1_f32).
template <int KIND = kAnyTerms>
__device__ inline void drift_f32(const Density& D, float scale, float xi, float eta, float& bx, float& by)
{
    if (KIND >= 0) {
        drift1_f32<KIND>(D, scale, xi, eta, bx, by);
        return;
    }
    float W = D.fbase, Gx = 0.0f, Gy = 0.0f;
    {
        for (int t = 0; t < D.n_terms; ++t) {
            switch (D.kind[t]) {
            case SDD_TERM_GAUSS: term_f32<SDD_TERM_GAUSS>(D, t, xi, eta, W, Gx, Gy); break;
            case SDD_TERM_RING: term_f32<SDD_TERM_RING>(D, t, xi, eta, W, Gx, Gy); break;
            case SDD_TERM_SECH2: term_f32<SDD_TERM_SECH2>(D, t, xi, eta, W, Gx, Gy); break;
            case SDD_TERM_SIN2: term_f32<SDD_TERM_SIN2>(D, t, xi, eta, W, Gx, Gy); break;
            default: break;
            }
        }
    }
    const float iw = __builtin_amdgcn_rcpf(W) * scale;
    bx = Gx * iw;
    by = Gy * iw;
}

template <int KIND = kAnyTerms>
__device__ inline void drift_f64(const Density& D, double xi, double eta, double& bx, double& by)
{
    double w, gx, gy;
    density_grad<KIND>(D, xi, eta, w, gx, gy);
    bx = gx / w;
    by = gy / w;
}

// ------------------------------------------------------------ boundary map

// (x_b, y_b) at boundary point (xi, eta) of side `side` (0: xi=0, 1: xi=1,
// 2: eta=0, 3: eta=1).
__device__ inline void bmap_eval(const Bmap& B, int side, double xi, double eta, double& x, double& y)
{
    switch (B.kind) {
    case SDD_BMAP_AFFINE:
        x = B.p[0] + B.p[1] * xi + B.p[2] * eta;
        y = B.p[3] + B.p[4] * xi + B.p[5] * eta;
        return;
    case SDD_BMAP_ANNULUS: {
        const double rho = B.p[0] + (B.p[1] - B.p[0]) * xi;
        const double th = B.p[2] + (B.p[3] - B.p[2]) * eta;
        double sn, cs;
        sincos(th, &sn, &cs);
        x = rho * cs;
        y = rho * sn;
        return;
    }
    case SDD_BMAP_TABLE: {
        const double s = (side < 2) ? eta : xi;
        const double pos = s * (double)(B.n - 1);
        int q = (int)floor(pos);
        q = q < 0 ? 0 : (q > B.n - 2 ? B.n - 2 : q);
        const double f = pos - (double)q;
        const double* v = B.table + ((size_t)side * B.n + q) * 2;
        x = v[0] + f * (v[2] - v[0]);
        y = v[1] + f * (v[3] - v[1]);
        return;
    }
    default:
        x = xi;
        y = eta;
        return;
    }
}

// Boundary side of a point known to lie on the boundary, first match in the
// order xi=0, xi=1, eta=0, eta=1.
__device__ inline int boundary_side(double xi, double eta)
{
    if (xi == 0.0) return 0;
    if (xi == 1.0) return 1;
    if (eta == 0.0) return 2;
    return 3;
}

// ------------------------------------------------------------ exit point

// First crossing of segment P -> Q with the square boundary (P inside, Q on
// or outside), in double.  Ties keep the earlier side of xi=0, xi=1, eta=0,
// eta=1.  E gets the side's coordinate exactly, the other one clamped.
__device__ inline int exit_point(double px, double py, double qx, double qy, double& ex, double& ey)
{
    double tb = 2.0;
    int side = 0;
    if (qx <= 0.0) { const double t = (0.0 - px) / (qx - px); if (t < tb) { tb = t; side = 0; } }
    if (qx >= 1.0) { const double t = (1.0 - px) / (qx - px); if (t < tb) { tb = t; side = 1; } }
    if (qy <= 0.0) { const double t = (0.0 - py) / (qy - py); if (t < tb) { tb = t; side = 2; } }
    if (qy >= 1.0) { const double t = (1.0 - py) / (qy - py); if (t < tb) { tb = t; side = 3; } }
    double x = px + tb * (qx - px);
    double y = py + tb * (qy - py);
    x = fmin(fmax(x, 0.0), 1.0);
    y = fmin(fmax(y, 0.0), 1.0);
    if (side == 0) x = 0.0;
    if (side == 1) x = 1.0;
    if (side == 2) y = 0.0;
    if (side == 3) y = 1.0;
    ex = x;
    ey = y;
    return side;
}

// Nearest boundary point of an interior point (step-capped paths); ties in
// the same side order.
__device__ inline int nearest_side(double px, double py, double& ex, double& ey)
{
    int side = 0;
    double best = px;
    if (1.0 - px < best) { best = 1.0 - px; side = 1; }
    if (py < best) { best = py; side = 2; }
    if (1.0 - py < best) { side = 3; }
    ex = (side == 0) ? 0.0 : (side == 1 ? 1.0 : px);
    ey = (side == 2) ? 0.0 : (side == 3 ? 1.0 : py);
    return side;
}

}  // namespace sdd
