// host.h -- host-side validation and conversion shared by the C ABI layer
// and the request server.
#pragma once

#include <math.h>
#include <string.h>

#include "common.h"
#include "sdd.h"
#include "walk.h"

struct sdd_ctx {
    int device;
    int cu_count;
    int wall_rate_khz;  // rate of the device wall clock (wall_clock64)
    void* scratch;      // this device's copy of the library's static scratch array
};

namespace sdd {


inline bool is_finite(double v) { return isfinite(v) != 0; }

inline sdd_status check_density(const sdd_density* w)
{
    if (!w) return SDD_EINVAL;
    if (!(w->base > 0.0) || !is_finite(w->base)) return SDD_EINVAL;
    if (w->n_terms < 0 || w->n_terms > SDD_MAX_TERMS) return SDD_EINVAL;
    for (int t = 0; t < w->n_terms; ++t) {
        const sdd_density_term& T = w->term[t];
        if (T.kind < SDD_TERM_GAUSS || T.kind > SDD_TERM_SIN2) return SDD_EINVAL;
        if (!(T.amp >= 0.0) || !is_finite(T.amp) || !is_finite(T.coef) || !is_finite(T.cx) || !is_finite(T.cy) ||
            !is_finite(T.r0) || !is_finite(T.nx) || !is_finite(T.ny))
            return SDD_EINVAL;
        if ((T.kind == SDD_TERM_GAUSS || T.kind == SDD_TERM_RING) && !(T.coef >= 0.0)) return SDD_EINVAL;
    }
    return SDD_OK;
}

inline sdd_status check_bmap(const sdd_bmap* b)
{
    if (!b) return SDD_EINVAL;
    if (b->kind < SDD_BMAP_IDENTITY || b->kind > SDD_BMAP_TABLE) return SDD_EINVAL;
    if (b->kind == SDD_BMAP_TABLE && (!b->table || b->n_per_edge < 2)) return SDD_EINVAL;
    for (int i = 0; i < 8; ++i)
        if (!is_finite(b->p[i])) return SDD_EINVAL;
    return SDD_OK;
}

inline sdd_status check_layout(const sdd_layout* L)
{
    if (!L) return SDD_EINVAL;
    if (L->sx < 1 || L->sy < 1 || L->nx < 3 || L->ny < 3) return SDD_EINVAL;
    if ((L->nx - 1) % L->sx || (L->ny - 1) % L->sy) return SDD_EINVAL;
    if ((L->nx - 1) / L->sx < 2 || (L->ny - 1) / L->sy < 2) return SDD_EINVAL;
    if ((int64_t)L->nx * L->ny > (int64_t)1 << 31) return SDD_EINVAL;
    return SDD_OK;
}

inline Density to_device(const sdd_density* w)
{
    Density D;
    memset(&D, 0, sizeof(D));
    D.n_terms = w->n_terms;
    D.base = w->base;
    D.fbase = (float)w->base;
    for (int t = 0; t < w->n_terms; ++t) {
        const sdd_density_term& T = w->term[t];
        D.kind[t] = T.kind;
        D.amp[t] = T.amp;
        D.coef[t] = T.coef;
        D.cx[t] = T.cx;
        D.cy[t] = T.cy;
        D.r0[t] = T.r0;
        D.nx[t] = T.nx;
        D.ny[t] = T.ny;
        D.famp[t] = (float)T.amp;
        D.fcoef[t] = (float)T.coef;
        D.fk2[t] = (float)(-T.coef * 1.4426950408889634073599246810019);
        D.fla[t] = (float)log2(T.amp);  // -inf for a zero amplitude: the term vanishes
        D.fm2c[t] = (float)(-2.0 * T.coef);
        D.fcx[t] = (float)T.cx;
        D.fcy[t] = (float)T.cy;
        D.fr0[t] = (float)T.r0;
        D.fnx[t] = (float)T.nx;
        D.fny[t] = (float)T.ny;
        // the argument's plane and the gradient factors (common.h, drift1_f32)
        const double off = -(T.nx * T.cx + T.ny * T.cy);
        if (T.kind == SDD_TERM_SECH2) {
            const double k = 2.0 * 1.4426950408889634073599246810019 * T.coef;  // 2 log2(e) coef
            D.fpa[t] = (float)(k * T.nx);
            D.fpb[t] = (float)(k * T.ny);
            D.fpc[t] = (float)(k * off);
            D.fsd[t] = (float)(2.0 * w->base + 4.0 * T.amp);
            D.fgx[t] = (float)(-8.0 * T.amp * T.coef * T.nx);  // 4 amp m2c n
            D.fgy[t] = (float)(-8.0 * T.amp * T.coef * T.ny);
        } else if (T.kind == SDD_TERM_SIN2) {
            const double k = T.coef / 6.283185307179586476925286766559;  // turns
            D.fpa[t] = (float)(k * T.nx);
            D.fpb[t] = (float)(k * T.ny);
            D.fpc[t] = (float)(k * off);
            D.fgx[t] = (float)(2.0 * T.amp * T.coef * T.nx);  // -m2c amp n
            D.fgy[t] = (float)(2.0 * T.amp * T.coef * T.ny);
        }
    }
    return D;
}

inline Bmap to_device(const sdd_bmap* b)
{
    Bmap B;
    B.kind = b->kind;
    B.n = b->n_per_edge;
    for (int i = 0; i < 8; ++i) B.p[i] = b->p[i];
    B.table = b->table;
    return B;
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline sdd_status from_hip(hipError_t e) { return e == hipSuccess ? SDD_OK : SDD_EDEVICE; }

// Nodes and paths per node are counter words of 32 bits; the node sums are
// exact for up to 2^32 paths per node.
constexpr int64_t kMaxNodes = ((int64_t)1 << 32) - 1;
constexpr int64_t kMaxPathsPerNode = ((int64_t)1 << 32) - 1;

// Noise factor of a float step: sqrt(2 dt) sqrt(2 ln 2) (the float normals
// come scaled by 1/sqrt(2 ln 2)).
inline double noise_f32(double dt) { return sqrt(2.0 * dt) * sqrt(2.0 * 0.69314718055994530942); }

// Step cap ceil(t_max/dt) rounded up to whole three-step Philox blocks; -1
// when it does not fit the 28-bit step count.
inline int32_t step_cap(double t_max, double dt)
{
    double kd = ceil(t_max / dt);
    if (!(kd >= 1.0) || kd >= (double)(((int64_t)1 << 28) - 3)) return -1;
    kd += fmod(3.0 - fmod(kd, 3.0), 3.0);
    return (int32_t)kd;
}

// Paths per pool of a walk launch: 64, or up to 256 when the launch has at
// least 8 pools of that size for every wave a device of cu_count CUs keeps
// (16 per CU).  Results do not depend on it.
inline uint32_t pool_paths_for(int64_t total_paths, int cu_count)
{
    const int64_t waves = (int64_t)(cu_count > 0 ? cu_count : 256) * 16;
    int64_t k = total_paths / (waves * kPoolPaths * 8);
    if (k < 1) k = 1;
    if (k > (int64_t)(kMaxPoolPaths / kPoolPaths)) k = kMaxPoolPaths / kPoolPaths;
    return (uint32_t)(k * kPoolPaths);
}

// Float Gaussian-sum parameters of a density whose terms are all GAUSS.
inline GaussParams gauss_params(const Density& D)
{
    GaussParams G;
    memset(&G, 0, sizeof(G));
    G.n_terms = D.n_terms;
    G.base = D.fbase;
    for (int t = 0; t < D.n_terms; ++t) {
        G.cx[t] = D.fcx[t];
        G.cy[t] = D.fcy[t];
        G.k2[t] = D.fk2[t];
        G.la[t] = D.fla[t];
        G.m2c[t] = D.fm2c[t];
    }
    return G;
}


}  // namespace sdd
