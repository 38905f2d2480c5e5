/*
 * walk_ref.c -- plain CPU oracle of the interface Monte Carlo estimate.
 *
 * TEST INFRASTRUCTURE.  Only tests/, the smoke check and the CPU-baseline
 * leg of the benchmark may load this code.  It shares no source with the
 * HIP library.  It is deliberately plain: scalar loops, one path at a time,
 * in the order the method states them, built with -ffp-contract=off so that
 * the only fused multiply-adds are the explicit fma() calls of the
 * Euler-Maruyama update.
 *
 * What is computed (Bihlo & Haynes, Sec. 2.1-2.2):
 *   The mesh map solves div(w grad x) = 0 on the unit square with Dirichlet
 *   data x = x_b on the boundary (eq. (5), written for the map from the
 *   computational square).  Its expanded form (eq. (6)) is
 *   Laplace(x) + (grad w / w) . grad x = 0, whose Ito diffusion has drift
 *   grad w / w and diffusion coefficient sqrt(2) (the generator of
 *   dX = b dt + sigma dW is b.grad + sigma^2/2 Laplace).  The solution is the
 *   expected boundary value at the first exit (eq. (7a)); each path is
 *   stepped with Euler-Maruyama and tested for exit at the end of every step
 *   (Sec. 2.2), and the estimate is the arithmetic mean over N pseudo-random
 *   paths with standard error O(N^-1/2) (Sec. 2.2).
 *
 * Readings where the paper is silent (the same readings bind the HIP path):
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed,
 *     counter = (block m, path p, node g, 0); block m serves steps 3m, 3m+1
 *     and 3m+2 with two 21-bit fields each (block_fields below);
 *   - uniforms u = (b + 1/2) * 2^-21 for a field b, exactly representable in
 *     both float and double; normals by Box-Muller,
 *     (z_xi, z_eta) = sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b);
 *   - exit point: first crossing of the last step's segment with the square
 *     boundary, in double precision; ties go to xi=0, xi=1, eta=0, eta=1;
 *   - step cap ceil(t_max / dt) rounded up to a multiple of three (whole
 *     Philox blocks); a capped path takes the boundary value at the nearest
 *     boundary point and is counted;
 *   - the Brownian-bridge test of step 3m+j draws word j of the block with
 *     counter (m, p, g, 1);
 *   - exponential time stepping (Sec. 2.2): step 3m+j has the length
 *     tau = -ln(u) dt, u formed from word j of the block with counter
 *     (m, p, g, 2) as for the bridge, so that tau is exponential with mean
 *     dt; the step is Euler-Maruyama with that length and the exit test is
 *     the end-of-step check plus the bridge test with tau in place of dt.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "sddref.h"

/* ---------------------------------------------------------------- Philox */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 4):
 * each round multiplies two counter words by the round multipliers and mixes
 * the 64-bit products with the other two words and the round key; the key is
 * advanced by the Weyl constants between rounds. */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void sddref_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void sddref_philox_many(int64_t n, const uint32_t* ctr, const uint32_t key[2], uint32_t* out)
{
    for (int64_t i = 0; i < n; ++i) sddref_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* ---------------------------------------------------------------- normals */

/* The uniform fields of one Philox block (the paper asks only for parallel
 * pseudo-random numbers, Sec. 2.2; reading): a block serves three steps
 * with two 21-bit fields each.  Steps 3m and 3m+1 take the high 21 bits of
 * words (0, 1) and (2, 3); step 3m+2 takes the low 11 bits of word 0 with
 * the low 10 bits of word 1 above them, and likewise words 2 and 3.  Every
 * bit of the block but bit 10 of words 1 and 3 is used once. */
static void block_fields(const uint32_t r[4], int j, uint32_t* ba, uint32_t* bb)
{
    if (j < 2) {
        *ba = r[2 * j] >> 11;
        *bb = r[2 * j + 1] >> 11;
    } else {
        *ba = (r[0] & 0x7FFu) | ((r[1] & 0x3FFu) << 11);
        *bb = (r[2] & 0x7FFu) | ((r[3] & 0x3FFu) << 11);
    }
}

/* u = (b + 1/2) 2^-21 for a 21-bit field b: in (0, 1), exact in float. */
static double uniform21(uint32_t b) { return ((double)b + 0.5) * 0x1p-21; }

static void box_muller64(uint32_t ra, uint32_t rb, double* z0, double* z1)
{
    const double two_pi = 6.283185307179586476925286766559;
    double ua = uniform21(ra), ub = uniform21(rb);
    double radius = sqrt(-2.0 * log(ua));
    double angle = two_pi * ub;
    *z0 = radius * cos(angle);
    *z1 = radius * sin(angle);
}

static void box_muller32(uint32_t ra, uint32_t rb, float* z0, float* z1)
{
    const float two_pi = 6.28318530717958647692f;
    float ua = ((float)ra + 0.5f) * 0x1p-21f;
    float ub = ((float)rb + 0.5f) * 0x1p-21f;
    float radius = sqrtf(-2.0f * logf(ua));
    float angle = two_pi * ub;
    *z0 = radius * cosf(angle);
    *z1 = radius * sinf(angle);
}

/* 21-bit field pairs [n][2] -> z[n][2] (double precision transform) */
void sddref_normals64(int64_t n, const uint32_t* fields, double* z)
{
    for (int64_t i = 0; i < n; ++i) box_muller64(fields[2 * i], fields[2 * i + 1], z + 2 * i, z + 2 * i + 1);
}

/* blocks [n][4] -> u[n][6]: (u_a, u_b) of steps 3m, 3m+1, 3m+2 */
void sddref_block_uniforms(int64_t n, const uint32_t* blocks, double* u)
{
    for (int64_t i = 0; i < n; ++i)
        for (int j = 0; j < 3; ++j) {
            uint32_t a, b;
            block_fields(blocks + 4 * i, j, &a, &b);
            u[6 * i + 2 * j] = uniform21(a);
            u[6 * i + 2 * j + 1] = uniform21(b);
        }
}

/* ---------------------------------------------------------------- density */

/* w = base + sum_t amp_t f_t and its gradient (Sec. 2.1: w > 0 is the
 * diffusion coefficient of eq. (5); the drift of eq. (7b) is grad w / w). */
static void density64(const ref_density* d, double xi, double eta, double* w, double* gx, double* gy)
{
    double W = d->base, Gx = 0.0, Gy = 0.0;
    for (int t = 0; t < d->n_terms; ++t) {
        const ref_term* T = &d->term[t];
        double dx = xi - T->cx, dy = eta - T->cy;
        switch (T->kind) {
        case REF_GAUSS: {
            double e = T->amp * exp(-T->coef * (dx * dx + dy * dy));
            W += e;
            Gx += -2.0 * T->coef * dx * e;
            Gy += -2.0 * T->coef * dy * e;
        } break;
        case REF_RING: {
            double r = sqrt(dx * dx + dy * dy);
            double e = T->amp * exp(-T->coef * (r - T->r0) * (r - T->r0));
            W += e;
            if (r > 0.0) {
                double g = -2.0 * T->coef * (r - T->r0) * e / r;
                Gx += g * dx;
                Gy += g * dy;
            }
        } break;
        case REF_SECH2: {
            double s = T->coef * (T->nx * dx + T->ny * dy);
            double sech = 1.0 / cosh(s);
            double f = T->amp * sech * sech;
            double dfds = -2.0 * f * tanh(s);
            W += f;
            Gx += dfds * T->coef * T->nx;
            Gy += dfds * T->coef * T->ny;
        } break;
        case REF_SIN2: {
            double s = T->coef * (T->nx * dx + T->ny * dy);
            double sn = sin(s), cs = cos(s);
            double dfds = 2.0 * T->amp * sn * cs;
            W += T->amp * sn * sn;
            Gx += dfds * T->coef * T->nx;
            Gy += dfds * T->coef * T->ny;
        } break;
        default: break;
        }
    }
    *w = W; *gx = Gx; *gy = Gy;
}

static void density32(const ref_density* d, float xi, float eta, float* w, float* gx, float* gy)
{
    float W = (float)d->base, Gx = 0.0f, Gy = 0.0f;
    for (int t = 0; t < d->n_terms; ++t) {
        const ref_term* T = &d->term[t];
        float amp = (float)T->amp, coef = (float)T->coef;
        float dx = xi - (float)T->cx, dy = eta - (float)T->cy;
        switch (T->kind) {
        case REF_GAUSS: {
            float e = amp * expf(-coef * (dx * dx + dy * dy));
            W += e;
            Gx += -2.0f * coef * dx * e;
            Gy += -2.0f * coef * dy * e;
        } break;
        case REF_RING: {
            float r = sqrtf(dx * dx + dy * dy);
            float r0 = (float)T->r0;
            float e = amp * expf(-coef * (r - r0) * (r - r0));
            W += e;
            if (r > 0.0f) {
                float g = -2.0f * coef * (r - r0) * e / r;
                Gx += g * dx;
                Gy += g * dy;
            }
        } break;
        case REF_SECH2: {
            float nx = (float)T->nx, ny = (float)T->ny;
            float s = coef * (nx * dx + ny * dy);
            float sech = 1.0f / coshf(s);
            float f = amp * sech * sech;
            float dfds = -2.0f * f * tanhf(s);
            W += f;
            Gx += dfds * coef * nx;
            Gy += dfds * coef * ny;
        } break;
        case REF_SIN2: {
            float nx = (float)T->nx, ny = (float)T->ny;
            float s = coef * (nx * dx + ny * dy);
            float sn = sinf(s), cs = cosf(s);
            float dfds = 2.0f * amp * sn * cs;
            W += amp * sn * sn;
            Gx += dfds * coef * nx;
            Gy += dfds * coef * ny;
        } break;
        default: break;
        }
    }
    *w = W; *gx = Gx; *gy = Gy;
}

/* pts[n][2] -> w[n], grad[n][2] */
void sddref_density_eval(const ref_density* d, int64_t n, const double* pts, double* w, double* grad)
{
    for (int64_t i = 0; i < n; ++i) {
        double gx, gy;
        density64(d, pts[2 * i], pts[2 * i + 1], &w[i], &gx, &gy);
        if (grad) { grad[2 * i] = gx; grad[2 * i + 1] = gy; }
    }
}

/* ------------------------------------------------------------ boundary map */

/* Dirichlet data on the square boundary (eq. (5)): (x_b, y_b) at a boundary
 * point E on side `side` (0: xi=0, 1: xi=1, 2: eta=0, 3: eta=1). */
static void bmap_eval(const ref_bmap* b, int side, double xi, double eta, double* x, double* y)
{
    switch (b->kind) {
    case REF_BMAP_IDENTITY:
        *x = xi; *y = eta;
        return;
    case REF_BMAP_AFFINE:
        *x = b->p[0] + b->p[1] * xi + b->p[2] * eta;
        *y = b->p[3] + b->p[4] * xi + b->p[5] * eta;
        return;
    case REF_BMAP_ANNULUS: {
        double rho = b->p[0] + (b->p[1] - b->p[0]) * xi;
        double th = b->p[2] + (b->p[3] - b->p[2]) * eta;
        *x = rho * cos(th);
        *y = rho * sin(th);
        return;
    }
    case REF_BMAP_TABLE: {
        int n = b->n_per_edge;
        double s = (side < 2) ? eta : xi;
        double pos = s * (double)(n - 1);
        int64_t q = (int64_t)floor(pos);
        if (q < 0) q = 0;
        if (q > n - 2) q = n - 2;
        double frac = pos - (double)q;
        const double* v = b->table + ((int64_t)side * n + q) * 2;
        *x = v[0] + frac * (v[2] - v[0]);
        *y = v[1] + frac * (v[3] - v[1]);
        return;
    }
    default:
        *x = NAN; *y = NAN;
    }
}

void sddref_bmap_eval(const ref_bmap* b, int64_t n, const int32_t* side, const double* pts, double* out)
{
    for (int64_t i = 0; i < n; ++i)
        bmap_eval(b, side[i], pts[2 * i], pts[2 * i + 1], &out[2 * i], &out[2 * i + 1]);
}

/* ------------------------------------------------------------ exit point */

/* First crossing of the segment P -> Q with the boundary of the unit square,
 * P strictly inside and Q on or outside (the exit test of Sec. 2.2 has just
 * fired).  Returns the side; E has that side's coordinate set exactly. */
int sddref_exit_point(double px, double py, double qx, double qy, double* ex, double* ey)
{
    double tbest = INFINITY;
    int side = -1;
    if (qx <= 0.0) { double t = (0.0 - px) / (qx - px); if (t < tbest) { tbest = t; side = 0; } }
    if (qx >= 1.0) { double t = (1.0 - px) / (qx - px); if (t < tbest) { tbest = t; side = 1; } }
    if (qy <= 0.0) { double t = (0.0 - py) / (qy - py); if (t < tbest) { tbest = t; side = 2; } }
    if (qy >= 1.0) { double t = (1.0 - py) / (qy - py); if (t < tbest) { tbest = t; side = 3; } }
    double x = px + tbest * (qx - px);
    double y = py + tbest * (qy - py);
    if (x < 0.0) x = 0.0;
    if (x > 1.0) x = 1.0;
    if (y < 0.0) y = 0.0;
    if (y > 1.0) y = 1.0;
    if (side == 0) x = 0.0;
    if (side == 1) x = 1.0;
    if (side == 2) y = 0.0;
    if (side == 3) y = 1.0;
    *ex = x; *ey = y;
    return side;
}

/* Nearest boundary point of an interior point (capped paths). */
static int nearest_boundary(double px, double py, double* ex, double* ey)
{
    double d[4] = { px, 1.0 - px, py, 1.0 - py };
    int side = 0;
    for (int s = 1; s < 4; ++s) if (d[s] < d[side]) side = s;
    *ex = px; *ey = py;
    if (side == 0) *ex = 0.0;
    if (side == 1) *ex = 1.0;
    if (side == 2) *ey = 0.0;
    if (side == 3) *ey = 1.0;
    return side;
}

/* ------------------------------------------------------- bridge exit test */

/* The bridge test of step 3m+j draws word j of the Philox block with
 * counter word 3 = 1 (the normals' blocks have 0 there), as the uniform
 * u = ((q mod 2^23) + 1/2) 2^-23, exact in float and double. */
static double bridge_uniform(uint32_t q) { return ((double)(q & 0x7FFFFFu) + 0.5) * 0x1p-23; }

/* Bridge uniforms of n words (test access). */
void sddref_bridge_uniforms(int64_t n, const uint32_t* words, double* u)
{
    for (int64_t i = 0; i < n; ++i) u[i] = bridge_uniform(words[i]);
}

/* Brownian-bridge exit test (the conditional exit probability within a step
 * of Sec. 2.2).  Given the step P -> Q with both ends inside, each
 * coordinate of the Brownian bridge between them is an independent
 * one-dimensional bridge with diffusion coefficient 2 over time dt, and such
 * a bridge from distance a to distance b off a wall hits it with probability
 * exp(-a b / dt).  Per axis the nearer wall is taken (the far one is at
 * distance ~1 and contributes nothing at the time steps used); the path
 * exits with probability 1 - (1 - p_xi)(1 - p_eta), through the side of the
 * axis with the larger probability (xi on ties).
 * Returns the probability; *side receives that side. */
double sddref_bridge_exit_prob(double px, double py, double qx, double qy, double dt, int* side)
{
    double m0 = px * qx, m1 = (1.0 - px) * (1.0 - qx);
    double m2 = py * qy, m3 = (1.0 - py) * (1.0 - qy);
    double mx = (m0 <= m1) ? m0 : m1, my = (m2 <= m3) ? m2 : m3;
    double pxi = exp(-mx / dt), peta = exp(-my / dt);
    *side = (mx <= my) ? ((m0 <= m1) ? 0 : 1) : ((m2 <= m3) ? 2 : 3);
    return fma(-pxi, peta, pxi + peta);
}

static float bridge_exit_prob32(float px, float py, float qx, float qy, float dt, int* side)
{
    float m0 = px * qx, m1 = (1.0f - px) * (1.0f - qx);
    float m2 = py * qy, m3 = (1.0f - py) * (1.0f - qy);
    float mx = (m0 <= m1) ? m0 : m1, my = (m2 <= m3) ? m2 : m3;
    float pxi = expf(-mx / dt), peta = expf(-my / dt);
    *side = (mx <= my) ? ((m0 <= m1) ? 0 : 1) : ((m2 <= m3) ? 2 : 3);
    return fmaf(-pxi, peta, pxi + peta);
}

static int bridge_exit64(double px, double py, double qx, double qy, double dt, double u)
{
    int s;
    return (u < sddref_bridge_exit_prob(px, py, qx, qy, dt, &s)) ? s : -1;
}

static int bridge_exit32(float px, float py, float qx, float qy, float dt, float u)
{
    int s;
    return (u < bridge_exit_prob32(px, py, qx, qy, dt, &s)) ? s : -1;
}

/* Q projected onto side s. */
static void onto_side(int s, double qx, double qy, double* ex, double* ey)
{
    *ex = (s == 0) ? 0.0 : (s == 1) ? 1.0 : qx;
    *ey = (s == 2) ? 0.0 : (s == 3) ? 1.0 : qy;
}

/* Exponential time stepping: the length of a step from its uniform word,
 * tau = -ln(u) dt (an exponential variate with mean dt, rate 1/dt). */
static double expo_tau(uint32_t q, double dt) { return -log(bridge_uniform(q)) * dt; }

/* Exponential step lengths of n words (test access). */
void sddref_expo_steps(int64_t n, const uint32_t* words, double dt, double* tau)
{
    for (int64_t i = 0; i < n; ++i) tau[i] = expo_tau(words[i], dt);
}

/* ------------------------------------------------------------ one path */

typedef struct {
    double x, y;        /* boundary value at the exit point */
    double exi, eeta;   /* exit point */
    int64_t steps;
    int side;
    int capped;
} path_out;

/* proj_mode 0: value at the projected exit point (the method).
 * proj_mode 1: test mode, the map evaluated at the unprojected overshoot
 *              point X_{k+1} (only meaningful for identity/affine maps).
 * exit_test 1: also apply the Brownian-bridge exit test after each step.
 * exit_test 2: exponential time stepping (steps of random length tau, the
 *              bridge test with tau). */
static void walk_path64(const ref_density* d, const ref_bmap* b, double xi0, double eta0,
                        uint64_t g, uint64_t p, double dt, const uint32_t key[2], int64_t kmax,
                        int proj_mode, int exit_test, path_out* o)
{
    const int bridge = exit_test != 0;
    double X = xi0, Y = eta0;
    uint32_t r[4] = { 0, 0, 0, 0 }, q[4] = { 0, 0, 0, 0 }, e[4] = { 0, 0, 0, 0 };
    int64_t k = 0;
    for (;;) {
        if (k == kmax) {
            o->side = nearest_boundary(X, Y, &o->exi, &o->eeta);
            o->capped = 1;
            break;
        }
        const int j = (int)(k % 3);
        if (j == 0) {
            uint32_t ctr[4] = { (uint32_t)(k / 3), (uint32_t)p, (uint32_t)g, 0u };
            sddref_philox4x32_10(ctr, key, r);
            if (bridge) {
                ctr[3] = 1u;
                sddref_philox4x32_10(ctr, key, q);
            }
            if (exit_test == 2) {
                ctr[3] = 2u;
                sddref_philox4x32_10(ctr, key, e);
            }
        }
        const double h = (exit_test == 2) ? expo_tau(e[j], dt) : dt;  /* this step's length */
        const double s = sqrt(2.0 * h);
        uint32_t ra, rb;
        block_fields(r, j, &ra, &rb);
        double zx, zy, w, gx, gy;
        box_muller64(ra, rb, &zx, &zy);
        density64(d, X, Y, &w, &gx, &gy);
        double bx = gx / w, by = gy / w;
        double Xn = fma(s, zx, fma(bx, h, X));
        double Yn = fma(s, zy, fma(by, h, Y));
        ++k;
        if (Xn <= 0.0 || Xn >= 1.0 || Yn <= 0.0 || Yn >= 1.0) {
            if (proj_mode == 1) {
                o->exi = Xn; o->eeta = Yn; o->side = -1;
            } else {
                o->side = sddref_exit_point(X, Y, Xn, Yn, &o->exi, &o->eeta);
            }
            o->capped = 0;
            break;
        }
        if (bridge) {
            int sb = bridge_exit64(X, Y, Xn, Yn, h, bridge_uniform(q[j]));
            if (sb >= 0) {
                onto_side(sb, Xn, Yn, &o->exi, &o->eeta);
                o->side = sb;
                o->capped = 0;
                break;
            }
        }
        X = Xn; Y = Yn;
    }
    o->steps = k;
    bmap_eval(b, o->side < 0 ? 0 : o->side, o->exi, o->eeta, &o->x, &o->y);
}

static void walk_path32(const ref_density* d, const ref_bmap* b, double xi0, double eta0,
                        uint64_t g, uint64_t p, double dt, const uint32_t key[2], int64_t kmax,
                        int proj_mode, int exit_test, path_out* o)
{
    const int bridge = exit_test != 0;
    float X = (float)xi0, Y = (float)eta0;
    uint32_t r[4] = { 0, 0, 0, 0 }, q[4] = { 0, 0, 0, 0 }, e[4] = { 0, 0, 0, 0 };
    int64_t k = 0;
    for (;;) {
        if (k == kmax) {
            o->side = nearest_boundary((double)X, (double)Y, &o->exi, &o->eeta);
            o->capped = 1;
            break;
        }
        const int j = (int)(k % 3);
        if (j == 0) {
            uint32_t ctr[4] = { (uint32_t)(k / 3), (uint32_t)p, (uint32_t)g, 0u };
            sddref_philox4x32_10(ctr, key, r);
            if (bridge) {
                ctr[3] = 1u;
                sddref_philox4x32_10(ctr, key, q);
            }
            if (exit_test == 2) {
                ctr[3] = 2u;
                sddref_philox4x32_10(ctr, key, e);
            }
        }
        /* this step's length and noise factor, in float */
        const float h = (exit_test == 2) ? -logf((float)bridge_uniform(e[j])) * (float)dt : (float)dt;
        const float s = (exit_test == 2) ? sqrtf(2.0f * h) : (float)sqrt(2.0 * dt);
        uint32_t ra, rb;
        block_fields(r, j, &ra, &rb);
        float zx, zy, w, gx, gy;
        box_muller32(ra, rb, &zx, &zy);
        density32(d, X, Y, &w, &gx, &gy);
        float bx = gx / w, by = gy / w;
        float Xn = fmaf(s, zx, fmaf(bx, h, X));
        float Yn = fmaf(s, zy, fmaf(by, h, Y));
        ++k;
        if (Xn <= 0.0f || Xn >= 1.0f || Yn <= 0.0f || Yn >= 1.0f) {
            if (proj_mode == 1) {
                o->exi = (double)Xn; o->eeta = (double)Yn; o->side = -1;
            } else {
                o->side = sddref_exit_point((double)X, (double)Y, (double)Xn, (double)Yn, &o->exi, &o->eeta);
            }
            o->capped = 0;
            break;
        }
        if (bridge) {
            int sb = bridge_exit32(X, Y, Xn, Yn, h, (float)bridge_uniform(q[j]));
            if (sb >= 0) {
                onto_side(sb, (double)Xn, (double)Yn, &o->exi, &o->eeta);
                o->side = sb;
                o->capped = 0;
                break;
            }
        }
        X = Xn; Y = Yn;
    }
    o->steps = k;
    bmap_eval(b, o->side < 0 ? 0 : o->side, o->exi, o->eeta, &o->x, &o->y);
}

/* ------------------------------------------------------------ estimate */

/* Neumaier's compensated summation. */
typedef struct { double s, c; } nsum;
static void nsum_add(nsum* a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static double nsum_get(const nsum* a) { return a->s + a->c; }

/*
 * Interface estimate (eq. (7a) by the arithmetic mean, Sec. 2.2).
 *
 * nodes[n][2]       start points, strictly inside the unit square
 * node_ids[n]       counter word g of each node (NULL: g = list index)
 * paths, path_begin paths path_begin .. path_begin+paths-1 are walked
 * mean[n][2], se[n][2]  outputs; sums[n][4] (optional) = sum x, sum y,
 *                   sum x^2, sum y^2 before division
 * exit_test         0: end-of-step test only; 1: also the Brownian-bridge test;
 *                   2: exponential time stepping with mean step dt
 * stats[3]          total steps, total paths, capped paths
 * per_path[n][paths] optional records
 * Returns 0, or -1 on invalid arguments.
 */
int sddref_interface_estimate(const ref_density* d, const ref_bmap* b, const double* nodes,
                              const int64_t* node_ids, int64_t n, int64_t paths, int64_t path_begin,
                              double dt, uint64_t seed, int prec, double t_max, int proj_mode,
                              int exit_test, double* mean, double* se, double* sums, int64_t* stats,
                              ref_path_record* per_path, int nthreads)
{
    if (n < 1 || paths < 1 || !(dt > 0.0) || !(dt < 1.0) || path_begin < 0) return -1;
    if (exit_test < 0 || exit_test > 2) return -1;
    for (int64_t i = 0; i < n; ++i) {
        double a = nodes[2 * i], c = nodes[2 * i + 1];
        if (!(a > 0.0 && a < 1.0 && c > 0.0 && c < 1.0)) return -1;
    }
    if (!(t_max > 0.0)) t_max = 8.0;
    int64_t kmax = (int64_t)ceil(t_max / dt);
    kmax += (3 - kmax % 3) % 3;  /* a whole number of Philox blocks (three steps each) */
    const uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    int64_t tot_steps = 0, tot_capped = 0;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(+ : tot_steps, tot_capped)
#endif
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t g = node_ids ? (uint64_t)node_ids[i] : (uint64_t)i;
        nsum sx = { 0, 0 }, sy = { 0, 0 }, sxx = { 0, 0 }, syy = { 0, 0 };
        for (int64_t j = 0; j < paths; ++j) {
            const uint64_t p = (uint64_t)(path_begin + j);
            path_out o;
            if (prec == REF_FP32)
                walk_path32(d, b, nodes[2 * i], nodes[2 * i + 1], g, p, dt, key, kmax, proj_mode, exit_test, &o);
            else
                walk_path64(d, b, nodes[2 * i], nodes[2 * i + 1], g, p, dt, key, kmax, proj_mode, exit_test, &o);
            nsum_add(&sx, o.x);
            nsum_add(&sy, o.y);
            nsum_add(&sxx, o.x * o.x);
            nsum_add(&syy, o.y * o.y);
            tot_steps += o.steps;
            tot_capped += o.capped;
            if (per_path) {
                ref_path_record* R = &per_path[i * paths + j];
                R->exit_xi = o.exi;
                R->exit_eta = o.eeta;
                R->steps = o.steps;
                R->side = o.side;
                R->capped = o.capped;
            }
        }
        const double N = (double)paths;
        const double Sx = nsum_get(&sx), Sy = nsum_get(&sy);
        const double Sxx = nsum_get(&sxx), Syy = nsum_get(&syy);
        const double mx = Sx / N, my = Sy / N;
        mean[2 * i] = mx;
        mean[2 * i + 1] = my;
        if (se) {
            if (paths > 1) {
                double vx = Sxx - N * mx * mx, vy = Syy - N * my * my;
                se[2 * i] = sqrt((vx > 0.0 ? vx : 0.0) / (N * (N - 1.0)));
                se[2 * i + 1] = sqrt((vy > 0.0 ? vy : 0.0) / (N * (N - 1.0)));
            } else {
                se[2 * i] = 0.0;
                se[2 * i + 1] = 0.0;
            }
        }
        if (sums) {
            sums[4 * i] = Sx; sums[4 * i + 1] = Sy; sums[4 * i + 2] = Sxx; sums[4 * i + 3] = Syy;
        }
    }
    if (stats) {
        stats[0] = tot_steps;
        stats[1] = n * paths;
        stats[2] = tot_capped;
    }
    return 0;
}
