// host.h -- host-side validation and conversion shared by the C ABI layer
// and the request server.
#pragma once

#include <math.h>
#include <string.h>

#include "common.h"
#include "sdd.h"

struct sdd_ctx {
    int device;
    int cu_count;
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

// tickets (node, path) are 32-bit; keep clear of the top for the batch fetches
constexpr int64_t kMaxTickets = ((int64_t)1 << 32) - ((int64_t)1 << 24);


}  // namespace sdd
