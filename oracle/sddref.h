/*
 * sddref.h -- declarations of the plain CPU oracle (test infrastructure).
 *
 * This header belongs to the oracle alone.  It is not included by, and does
 * not include, anything of the HIP library; the structures below are the
 * oracle's own and are filled from plain Python dictionaries by
 * oracle/__init__.py.  Only tests, the smoke check and the CPU-baseline leg
 * of the benchmark load the oracle.
 *
 * Method: Bihlo & Haynes, "Parallel stochastic methods for PDE based grid
 * generation", Sec. 2.1 eq. (5)-(7) (linear Winslow generator and its
 * stochastic representation) and Sec. 2.2 (Euler-Maruyama, exit test,
 * arithmetic mean over pseudo-random paths).
 */
#ifndef SDDREF_H
#define SDDREF_H

#include <stdint.h>

#define REF_MAX_TERMS 8

enum { REF_GAUSS = 0, REF_RING = 1, REF_SECH2 = 2, REF_SIN2 = 3 };
enum { REF_BMAP_IDENTITY = 0, REF_BMAP_AFFINE = 1, REF_BMAP_ANNULUS = 2, REF_BMAP_TABLE = 3 };
enum { REF_FP64 = 0, REF_FP32 = 1 };

typedef struct {
    int32_t kind;
    int32_t pad;
    double amp, coef, cx, cy, r0, nx, ny;
} ref_term;

typedef struct {
    double base;
    int32_t n_terms;
    int32_t pad;
    ref_term term[REF_MAX_TERMS];
} ref_density;

/* TABLE: values[4][n][2] on the sides xi=0, xi=1, eta=0, eta=1, each sampled
 * at parameter q/(n-1), q = 0..n-1 (the parameter is eta on the first two
 * sides and xi on the last two). */
typedef struct {
    int32_t kind;
    int32_t n_per_edge;
    double p[8];
    const double* table;
} ref_bmap;

typedef struct {
    double exit_xi, exit_eta;
    int64_t steps;
    int32_t side;
    int32_t capped;
} ref_path_record;

#endif
