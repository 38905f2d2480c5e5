/*
 * sdd.h -- C ABI of the MI355X library for stochastic-deterministic domain
 * decomposition of the linear Winslow mesh generator.
 *
 * Method: A. Bihlo and R. D. Haynes, "Parallel stochastic methods for PDE
 * based grid generation" (arXiv 1310.3435).
 *
 *   Problem (Sec. 2.1, eq. (5)): on the computational unit square find the
 *   mesh map (x, y)(xi, eta) with div(w grad x) = div(w grad y) = 0, w > 0,
 *   and (x, y) = (x_b, y_b) on the boundary.
 *   Stochastic representation (eq. (6), (7a), (7b)): x(p) = E[x_b(X_tau)]
 *   where X starts at p, solves the Ito SDE dX = (grad w / w) dt + sqrt(2) dW
 *   (drift and diffusion read off the expanded form eq. (6); the generator of
 *   dX = b dt + s dW is b.grad + s^2/2 Laplace) and tau is the first exit
 *   time from the square.
 *   Numerics (Sec. 2.2): Euler-Maruyama with step dt, exit test at the end
 *   of each step, arithmetic mean over N pseudo-random paths (error
 *   O(N^-1/2)).
 *   Decomposition (Sec. 2.1, Fig. 1): the estimate is evaluated only at
 *   interface points; the interfaces are completed by interpolation
 *   (Sec. 3.6) and every subdomain is then solved once, independently, by
 *   centred finite differences (Sec. 3.2).
 *
 * Conventions for every entry point:
 *   - Pointers documented "device" must be device memory of the context's
 *     GPU (e.g. a torch tensor's data_ptr()); "host" pointers are read
 *     before the call returns.  The caller owns every buffer; the library
 *     allocates nothing the caller sees.  Scratch memory comes from a
 *     caller-provided workspace whose size the matching *_workspace_bytes
 *     call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue work and return after host-side validation; outputs are
 *     valid once the stream has been synchronised.
 *   - Return values: SDD_OK (0); positive values are warnings (the work was
 *     done); negative values are errors; no exception crosses the ABI.  Argument errors (SDD_EINVAL, SDD_ENOSPC) are found
 *     before anything is enqueued; SDD_EDEVICE reports a failed HIP call,
 *     after which the outputs are undefined.  sdd_status_string() names
 *     them.  A context is not thread-safe; use one per host thread.
 *   - Arrays of points are [n][2] doubles (xi, eta) or (x, y), row-major.
 *   - Environment (tuning only; no result depends on it): SDD_WALK_WAVES_PER_SIMD
 *     and SDD_SERVE_WAVES_PER_SIMD set the waves per SIMD of the walk's and
 *     the server's persistent grids instead of the measured defaults;
 *     SDD_SERVE_RESERVED_CUS (default 0) keeps a server's walk launches off
 *     that many CUs, read when the server is created, so that its subdomain
 *     solves find free CUs (lower p99 latency, lower capacity).
 */
#ifndef SDD_H
#define SDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SDD_OK = 0,
    SDD_WARN_CAPPED = 1,   /* done, but some paths stopped at the step cap (sdd_walk_status, sdd_result) */
    SDD_EINVAL = -1,       /* an argument is out of range or inconsistent */
    SDD_ENOSPC = -2,       /* the workspace is smaller than required */
    SDD_EDEVICE = -3,      /* a HIP runtime call failed */
    SDD_EAGAIN = -4,       /* not finished yet (server poll) */
    SDD_ECANCELED = -5,    /* cancelled, or the server shut down first */
    SDD_EUNSUPPORTED = -6  /* a valid request of a kind the library does not implement */
} sdd_status;

typedef enum { SDD_FP64 = 0, SDD_FP32 = 1 } sdd_precision;

/* Exit test of a walk step (Sec. 2.2).  END_OF_STEP: the path exits when a
 * step ends on or outside the square.  BRIDGE: in addition, a step whose
 * ends are both inside exits with the probability that the Brownian bridge
 * between them left the square (Sec. 2.2 notes that this conditional
 * probability greatly reduces the error of plain stepping near the
 * boundary).  EXPONENTIAL: exponential time stepping (Sec. 2.2): every step
 * has an exponentially distributed length with mean dt (rate lambda =
 * 1/dt), and the boundary test is both the end-of-step check and the
 * conditional crossing probability of the step, as for BRIDGE. */
typedef enum { SDD_EXIT_END_OF_STEP = 0, SDD_EXIT_BRIDGE = 1, SDD_EXIT_EXPONENTIAL = 2 } sdd_exit_test;

/* Density terms; w = base + sum_t amp_t f_t with amp_t >= 0 and base > 0,
 * so w >= base > 0 as eq. (5) requires.  With d = (xi - cx, eta - cy) and
 * s = coef * (nx d_xi + ny d_eta):
 *   GAUSS  f = exp(-coef |d|^2)
 *   RING   f = exp(-coef (|d| - r0)^2)       (gradient of |d| taken as 0 at d = 0)
 *   SECH2  f = sech^2(s)
 *   SIN2   f = sin^2(s)                                                   */
typedef enum { SDD_TERM_GAUSS = 0, SDD_TERM_RING = 1, SDD_TERM_SECH2 = 2, SDD_TERM_SIN2 = 3 } sdd_term_kind;

#define SDD_MAX_TERMS 4

typedef struct {
    int32_t kind; /* sdd_term_kind */
    int32_t pad;
    double amp, coef, cx, cy, r0, nx, ny;
} sdd_density_term;

typedef struct {
    double base;
    int32_t n_terms; /* 0 .. SDD_MAX_TERMS */
    int32_t pad;
    sdd_density_term term[SDD_MAX_TERMS];
} sdd_density;

/* Boundary map (x_b, y_b) on the sides of the square:
 *   IDENTITY  (xi, eta)
 *   AFFINE    x = p0 + p1 xi + p2 eta, y = p3 + p4 xi + p5 eta
 *   ANNULUS   rho = p0 + (p1-p0) xi, theta = p2 + (p3-p2) eta,
 *             (x, y) = rho (cos theta, sin theta)
 *   TABLE     device table[4][n_per_edge][2] for the sides xi=0, xi=1,
 *             eta=0, eta=1, sampled at parameter q/(n_per_edge-1) (eta on
 *             the first two sides, xi on the last two), linear in between.
 *             sdd_bmap_edge1d_table() fills it with the one-dimensional
 *             generator data of Sec. 3.2.                                  */
typedef enum { SDD_BMAP_IDENTITY = 0, SDD_BMAP_AFFINE = 1, SDD_BMAP_ANNULUS = 2, SDD_BMAP_TABLE = 3 } sdd_bmap_kind;

typedef struct {
    int32_t kind; /* sdd_bmap_kind */
    int32_t n_per_edge;
    double p[8];
    const double* table; /* device, TABLE only */
} sdd_bmap;

/* Global (nx x ny)-node grid on [0,1]^2, xi_i = i/(nx-1), eta_j = j/(ny-1),
 * split into sx x sy subdomains of (nx-1)/sx + 1 by (ny-1)/sy + 1 nodes
 * (both divisions exact, at least 2 cells per subdomain side). */
typedef struct {
    int32_t nx, ny, sx, sy;
} sdd_layout;

/* Walk totals: sum of exit step counts (the exiting step included), paths
 * walked, paths stopped by the step cap, and T_stoc (Sec. 5, Tables 5-8):
 * the device time in ms from the start of the call's first kernel to the
 * end of its finalize, read from the device wall clock. */
typedef struct {
    int64_t steps, paths, capped;
    double t_stoc_ms;
} sdd_walk_stats;

/* One path's exit (parity mode): exit point, step count, side (0: xi=0,
 * 1: xi=1, 2: eta=0, 3: eta=1), capped flag. */
typedef struct {
    double exit_xi, exit_eta;
    int64_t steps;
    int32_t side;
    int32_t capped;
} sdd_path_record;

typedef struct sdd_ctx sdd_ctx;

const char* sdd_status_string(int status);

/* Library version, major*10000 + minor*100 + patch. */
int32_t sdd_version(void);

/* Context bound to HIP device `device`; reads its properties once.
 * SDD_EINVAL for a bad device index or NULL out. */
sdd_status sdd_create(int32_t device, sdd_ctx** out);
void sdd_destroy(sdd_ctx* ctx);

/* ---------------------------------------------------------------- walk ---
 * Monte Carlo estimate of the mesh map at interface points (eq. (7a) by the
 * arithmetic mean of Sec. 2.2, paths of eq. (7b) by Euler-Maruyama).
 *
 * Random numbers (the paper asks only for parallel pseudo-random numbers,
 * Sec. 2.2): Philox4x32-10 with key (seed mod 2^32, seed >> 32).  The block
 * of counter (m, p, g, 0) (path p of node g, g = index in `nodes`) serves
 * steps 3m, 3m+1 and 3m+2 with words w0..w3 cut into six 21-bit fields:
 * step 3m takes w0 >> 11 and w1 >> 11, step 3m+1 w2 >> 11 and w3 >> 11,
 * step 3m+2 (w0 & 0x7ff) | (w1 & 0x3ff) << 11 and the same of (w2, w3).
 * Uniforms u = (b + 1/2) 2^-21 (exact in float); normals by Box-Muller,
 * sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b).  Path p is therefore the
 * same wherever and whenever it is walked.
 *
 * Step: X <- X + (grad w / w)(X) dt + sqrt(2 dt) Z in the precision `prec`
 * (SDD_FP32 walks in float, SDD_FP64 in double).  The path exits at the
 * first step that ends on or outside the square; its exit point is the
 * first crossing of that step's segment with the boundary, computed in
 * double in both modes, and its value is the boundary map there.  A path
 * still inside after ceil(t_max/dt) steps, rounded up to a multiple of 3
 * (whole Philox blocks), is capped: it takes the value at the nearest
 * boundary point and is counted in stats->capped.
 *
 * exit_test SDD_EXIT_BRIDGE adds, after a step P -> Q with both ends inside,
 * the bridge test: each coordinate of the Brownian bridge from P to Q is an
 * independent one-dimensional bridge with diffusion coefficient 2, which
 * hits a wall it starts a and ends b away from with probability
 * exp(-a b / dt).  Per axis the nearer wall counts, and the step exits with
 * probability p_xi + p_eta - p_xi p_eta (computed as one fma), compared with
 * a uniform from a block of its own: step 3m + j takes word j of the block
 * of counter (m, p, g, 1), u = ((q mod 2^23) + 1/2) 2^-23.
 * A bridged exit leaves through the nearer wall of the axis with the larger
 * probability (xi on ties), at Q moved onto that wall; these decisions are
 * taken in the walk precision.  Its bias in the exit point is O(dt) where
 * the end-of-step test's is O(sqrt dt).
 *
 * exit_test SDD_EXIT_EXPONENTIAL (exponential time stepping): step 3m + j
 * has length tau = -ln(u) dt, u from word j of the block of counter
 * (m, p, g, 2) formed as for the bridge, so tau is exponential with mean dt;
 * X <- X + (grad w / w)(X) tau + sqrt(2 tau) Z, the exact law of the
 * diffusion with the drift frozen over the step; and the bridge test above
 * with tau in place of dt, which given tau is the exact crossing
 * probability of that process.  The step cap counts steps as above
 * (ceil(t_max/dt), i.e. t_max in expectation).
 *
 * Node sums are exact: each path's x, y, x^2, y^2 is rounded to a multiple
 * of 2^-F (2^-54 times a power of two bounding the boundary map's image,
 * from its parameters or, for a TABLE map, its table: below a double's
 * rounding of such values) and added into 64-bit integer limbs, so the
 * sums are independent of the order in which paths finish and the results
 * are bitwise reproducible.  The workspace
 * holds these sums (96 bytes per node) and a 256-byte header; the walk
 * keeps each finished path only in on-chip memory until its exit is
 * processed.
 *
 *   w, bmap      host structs (bmap->table, if any, is device memory)
 *   nodes        device [n_nodes][2]; 1 <= n_nodes < 2^32
 *   paths_per_node  1 <= N < 2^32; paths path_begin .. path_begin+N-1 are
 *                walked (path_begin + N <= 2^32)
 *   dt           0 < dt < 1 (the mean step for SDD_EXIT_EXPONENTIAL), and
 *                ceil(t_max/dt) < 2^28 - 3
 *   t_max        step cap in time units; <= 0 selects 8
 *   exit_test    sdd_exit_test
 *   mean         device [n][2]   sum / N
 *   se           device [n][2] or NULL: sqrt(max(0, S2 - N mean^2) / (N(N-1))),
 *                0 when N = 1
 *   sums         device [n][4] or NULL: sum x, sum y, sum x^2, sum y^2
 *   stats        device sdd_walk_stats or NULL (overwritten)
 *   per_path     device [n][N] sdd_path_record or NULL
 *   workspace    device, >= sdd_workspace_bytes(n_nodes, N, prec) bytes
 * Errors: SDD_EINVAL (bad argument), SDD_ENOSPC, SDD_EDEVICE.  Node
 * positions live on the device and are not read by the host: a node on or
 * outside the boundary walks no path and gets NaN mean, SE and sums (and
 * per-path records with NaN exit, 0 steps, side -1).  Capped paths are a
 * device-side condition: read stats and pass it to sdd_walk_status. */
size_t sdd_workspace_bytes(int64_t n_nodes, int64_t paths_per_node, int32_t prec);

sdd_status sdd_interface_estimate(sdd_ctx* ctx, const sdd_density* w, const sdd_bmap* bmap,
                                  const double* nodes, int64_t n_nodes, int64_t paths_per_node,
                                  int64_t path_begin, double dt, uint64_t seed, int32_t prec, double t_max,
                                  int32_t exit_test, double* mean, double* se, double* sums,
                                  sdd_walk_stats* stats, sdd_path_record* per_path, void* workspace,
                                  size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * estimate as sdd_interface_estimate, with the same arguments but no
 * workspace.  Its scratch (the node sums and a header) is a static device
 * array of the library, 256 + 96 * sdd_noalloc_max_nodes() bytes (6.3 MB),
 * which each GPU the library runs on holds until the process ends; the
 * call allocates nothing.  n_nodes above sdd_noalloc_max_nodes() (65536)
 * gives SDD_ENOSPC.  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (other streams, other threads, other contexts)
 * race and give wrong results; calls in one stream's order are safe.
 * The first kernel of each call resets the scratch it uses. */
sdd_status sdd_interface_estimate_noalloc(sdd_ctx* ctx, const sdd_density* w, const sdd_bmap* bmap,
                                          const double* nodes, int64_t n_nodes, int64_t paths_per_node,
                                          int64_t path_begin, double dt, uint64_t seed, int32_t prec, double t_max,
                                          int32_t exit_test, double* mean, double* se, double* sums,
                                          sdd_walk_stats* stats, sdd_path_record* per_path, void* stream);

/* Largest n_nodes sdd_interface_estimate_noalloc accepts. */
int64_t sdd_noalloc_max_nodes(void);

/* SDD_WARN_CAPPED if the host copy of a walk's stats counts capped paths,
 * SDD_OK otherwise; SDD_EINVAL for NULL. */
sdd_status sdd_walk_status(const sdd_walk_stats* stats);

/* ----------------------------------------------------------- interfaces ---
 * Interface points of a layout (Sec. 2.1, Fig. 1): the (sx-1)(sy-1)
 * crosspoints row by row, then k points on every segment of every vertical
 * interface line (lines left to right, segments bottom to top, points in
 * increasing eta), then k points on every segment of every horizontal line
 * (lines bottom to top, segments left to right, increasing xi).
 * placement 0 (uniform): s_i = a + (b-a) i/(k+1) on segment [a, b];
 * placement 1 (equidistributed): int_a^{s_i} w ds = i/(k+1) int_a^b w ds,
 * with the integral by Simpson's rule on 4096 panels and linear inversion
 * inside a panel (the paper places points from the density, Sec. 3.6).
 * nodes: device [sdd_layout_node_count(L, k)][2].  w may be NULL for
 * placement 0. */
int64_t sdd_layout_node_count(const sdd_layout* L, int32_t k);

sdd_status sdd_layout_nodes(sdd_ctx* ctx, const sdd_layout* L, int32_t k, int32_t placement, const sdd_density* w,
                            double* nodes, void* stream);

/* Interface points at the extrema of the density's first and second
 * derivatives along every segment (Sec. 3.6 places the Monte Carlo points
 * at the maxima and minima of the first and second derivatives of the
 * monitor function along the dividing lines).  Per segment (open interval):
 * the derivative along the line from the analytic gradient of w at 4097
 * equally spaced samples, the second derivative from its central
 * differences; a strict local extremum of either on the samples is moved to
 * the vertex of the parabola through its three samples; the points are
 * sorted and a point closer than one sample to the previous one is dropped
 * (at most 64 extrema of each derivative are examined).
 *   nodes   device [sdd_layout_node_count(L, cap)][2]: the crosspoints,
 *           then cap slots per segment (segment order of sdd_layout_nodes)
 *           holding its points in increasing parameter, then (-1, -1)
 *           (off the square: sdd_interface_estimate walks nothing there
 *           and gives NaN)
 *   counts  device int32 [number of segments]: points found per segment;
 *           the first min(counts[s], cap) slots are used
 * Pass the same cap and counts to sdd_fill_interfaces_counts. */
sdd_status sdd_layout_nodes_extrema(sdd_ctx* ctx, const sdd_layout* L, const sdd_density* w, int32_t cap,
                                    double* nodes, int32_t* counts, void* stream);

/* One-dimensional edge data (Sec. 3.2: tangential boundary values from the
 * 1D generator): on each side the tangential coordinate is
 * int_0^s 1/w / int_0^1 1/w along that side (cumulative Simpson on the
 * n_per_edge - 1 sample intervals), the normal coordinate the side's value.
 * table: device [4][n_per_edge][2], n_per_edge >= 3.  Use it as a TABLE
 * bmap. */
sdd_status sdd_bmap_edge1d_table(sdd_ctx* ctx, const sdd_density* w, int32_t n_per_edge, double* table,
                                 void* stream);

/* Interface completion (Sec. 3.6: Monte Carlo at a few points plus
 * interpolation).  values: device [node_count][2], the estimates at `nodes`
 * (layout order above).  Every segment is interpolated through (start, its
 * k points, end) in the segment parameter: interp 0 linear, interp 1
 * monotone piecewise cubic (Fritsch-Carlson slopes, three-point
 * shape-preserving end slopes).  Segment ends are crosspoint estimates or,
 * on the outer boundary, the boundary map.
 * vert: device [sx-1][ny][2] (the full line xi = a/sx); horiz: device
 * [sy-1][nx][2] (the full line eta = b/sy).  Either may be NULL when that
 * direction has no line. */
sdd_status sdd_fill_interfaces(sdd_ctx* ctx, const sdd_layout* L, int32_t k, const sdd_bmap* bmap,
                               const double* nodes, const double* values, int32_t interp, double* vert,
                               double* horiz, void* stream);

/* As sdd_fill_interfaces for a node list of cap slots per segment of which
 * segment s uses the first min(counts[s], cap) (device int32 counts, e.g.
 * from sdd_layout_nodes_extrema); a segment with no points is interpolated
 * between its ends. */
sdd_status sdd_fill_interfaces_counts(sdd_ctx* ctx, const sdd_layout* L, int32_t cap, const int32_t* counts,
                                      const sdd_bmap* bmap, const double* nodes, const double* values,
                                      int32_t interp, double* vert, double* horiz, void* stream);

/* ------------------------------------------------------------ subdomains ---
 * Independent Dirichlet solves of every subdomain (Sec. 2.1: solved once, no
 * iteration between subdomains).  Discretisation: conservative centred
 * 5-point stencil (Sec. 3.2 uses centred differences), w at the edge
 * midpoints, x_P = sum a_nb x_nb / sum a_nb with a_E = w(xi+h/2, eta)/h^2
 * etc.  Solved by red-black successive over-relaxation until the largest
 * change of a sweep is <= tol (tol <= 0 selects 1e-13), until that change
 * stops falling (no halving within 512 sweeps: the rounding floor), or
 * after max_sweeps (<= 0 selects 100000) sweeps.
 * mesh: device [ny][nx][2]; on return the boundary ring holds the map, the
 * interface lines hold vert/horiz, every subdomain interior its solution.
 * sweeps (device [sx*sy] int32 or NULL) and resid (device [sx*sy] double or
 * NULL) report, per subdomain b*sx + a, the sweeps taken and the last
 * largest change (the larger of the two components).
 * The solve is double only, on purpose: it is a few percent of a pass
 * (T_sub, Sec. 5), its subdomains stay in LDS in double, and a float
 * iteration would stall near 1e-7 of the map's scale, far above the 1e-13
 * the stopping rule reaches and to which the result is checked. */
size_t sdd_subdomain_workspace_bytes(const sdd_layout* L);

sdd_status sdd_subdomain_solve(sdd_ctx* ctx, const sdd_density* w, const sdd_bmap* bmap, const sdd_layout* L,
                               const double* vert, const double* horiz, double tol, int32_t max_sweeps,
                               double* mesh, int32_t* sweeps, double* resid, void* workspace, size_t ws_bytes,
                               void* stream);

/* ------------------------------------------------------ whole-grid mesh ---
 * The mesh by Monte Carlo at every grid point (Sec. 3.3), for comparison
 * with the decomposition.  sdd_grid_nodes writes the (nx-2)(ny-2) interior
 * nodes (i/(nx-1), j/(ny-1)) row by row (j = 1..ny-2 outer, i = 1..nx-2
 * inner) to device nodes[][2]; estimate them with sdd_interface_estimate;
 * sdd_assemble_mesh then writes device mesh[ny][nx][2]: the boundary map on
 * the ring (as sdd_subdomain_solve writes it) and device values[][2], in
 * the order of sdd_grid_nodes, inside.  nx, ny >= 3. */
sdd_status sdd_grid_nodes(sdd_ctx* ctx, int32_t nx, int32_t ny, double* nodes, void* stream);

sdd_status sdd_assemble_mesh(sdd_ctx* ctx, int32_t nx, int32_t ny, const sdd_bmap* bmap, const double* values,
                             double* mesh, void* stream);

/* ------------------------------------------------- quality and smoothing ---
 * Geometric mesh quality (eq. (11), Sec. 3.1).  For each of the
 * (nx-1)(ny-1) cells, J is the Jacobian of the cell's bilinear map at its
 * centre: x_xi = ((x10 + x11) - (x00 + x01)) / (2 h_xi),
 * x_eta = ((x01 + x11) - (x00 + x10)) / (2 h_eta), y alike, with
 * h_xi = 1/(nx-1), h_eta = 1/(ny-1) and x_ab the node (i+a, j+b); then
 * Q = tr(J^T J) / (2 sqrt(det(J^T J))), computed as |J|_F^2 / (2 |det J|).
 *   mesh  device [ny][nx][2]
 *   q     device [ny-1][nx-1] or NULL: Q of every cell, row-major
 *   out   device double[3]: Q_max, Q_mean (Sec. 3.3), the number of cells
 *         with det J <= 0 (folded or degenerate; a degenerate cell has
 *         Q = +inf)
 * Sums run in a fixed order.  workspace: device,
 * >= sdd_quality_workspace_bytes(nx, ny) (also serves sdd_mesh_compare). */
size_t sdd_quality_workspace_bytes(int32_t nx, int32_t ny);

sdd_status sdd_mesh_quality(sdd_ctx* ctx, int32_t nx, int32_t ny, const double* mesh, double* q, double* out,
                            void* workspace, size_t ws_bytes, void* stream);

/* Two meshes of the same grid (Sec. 3.3): out[0] = l_inf =
 * max over nodes |w(mesh_i) - w(ref_i)|, w evaluated at the nodes' physical
 * positions (meaningful where the physical domain lies in the unit square);
 * out[1] = the largest Euclidean node displacement.  out: device double[2]. */
sdd_status sdd_mesh_compare(sdd_ctx* ctx, int32_t nx, int32_t ny, const sdd_density* w, const double* mesh,
                            const double* ref, double* out, void* workspace, size_t ws_bytes, void* stream);

/* Perona-Malik anisotropic diffusion of the mesh (eq. (12), Sec. 3.4):
 * each component u in {x, y} of the mesh map over the computational grid
 * takes `steps` forward-in-time centred-in-space steps of
 * u_t = div(c grad u), c = exp(-|grad u|^2 / k^2):
 *   u_P += dt (c_E (u_E - u_P) + c_W (u_W - u_P)) / h_xi^2
 *        + dt (c_N (u_N - u_P) + c_S (u_S - u_P)) / h_eta^2,
 * each face coefficient from the one-sided difference across the face,
 * c_E = exp(-((u_E - u_P) / h_xi)^2 / k^2) (Perona and Malik's
 * discretisation).  The boundary ring is fixed; with per_subdomain = 1 the
 * interface lines of L are fixed too, so every subdomain is smoothed on
 * its own (Sec. 3.5); per_subdomain = 2 fixes instead the lines half a
 * subdomain (rounded down) further on, the subdomains of a second cycle
 * whose interiors hold the original interfaces (Sec. 4); per_subdomain = 0
 * smooths the whole grid.
 * Requires dt (2/h_xi^2 + 2/h_eta^2) <= 1 (then each step is a convex
 * combination: no new extrema), else SDD_EINVAL.  k > 0, steps >= 0.
 *   mesh       device [ny][nx][2], smoothed in place
 *   workspace  device, >= sdd_smooth_workspace_bytes(L) */
size_t sdd_smooth_workspace_bytes(const sdd_layout* L);

sdd_status sdd_mesh_smooth(sdd_ctx* ctx, const sdd_layout* L, int32_t per_subdomain, double dt, double k,
                           int32_t steps, double* mesh, void* workspace, size_t ws_bytes, void* stream);

/* Interface pre-smoothing (Sec. 4: interface values smoothed by locally
 * weighted quadratic least squares before the subdomain solves).  Along
 * every full interface line (vert, horiz as for sdd_fill_interfaces), each
 * point except the outer-boundary ends and the crosspoints takes the value
 * at its own parameter of the quadratic fitted to the `span` points nearest
 * in index (the window shifted to stay on the line) with tricube weights
 * (1 - (|t|/d)^3)^3, d the largest |t| in the window (Cleveland's local
 * regression).  span odd, 5 <= span <= the points of a line.  In place;
 * workspace >= sdd_smooth_interfaces_workspace_bytes(L). */
size_t sdd_smooth_interfaces_workspace_bytes(const sdd_layout* L);

sdd_status sdd_smooth_interfaces(sdd_ctx* ctx, const sdd_layout* L, int32_t span, double* vert, double* horiz,
                                 void* workspace, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------- serving ---
 * A request server that batches whole mesh requests (interface estimate,
 * fill and subdomain solves) continuously: requests that arrive while
 * others run are admitted as slots and device memory free up, and every
 * walk launch mixes blocks of paths from all admitted requests.
 *
 * Paths are scheduled in blocks of 1024 per node.  With se_target > 0 the
 * first block is a pilot; the request then runs
 * N = max(1024, ceil((s / se_target)^2)) paths per node, rounded up to a
 * multiple of 1024, where s is the largest sample standard deviation of x
 * or y over its nodes (the paper notes the mean's additivity makes such a
 * stopping rule compatible with the method, Sec. 6).  With se_target <= 0
 * paths_per_node (<= 2^30) is used, rounded up to a multiple of 1024, and
 * there is no pilot: every block may go into the first launch.  The
 * node sums are exact and a path's random numbers depend only on (seed,
 * node, path, step), so a request's result is bitwise the same alone or in
 * any mix.
 *
 * Requests walk in float (exact node sums, double exit projection) with
 * the exit test of sdd_interface_estimate that exit_test names
 * (END_OF_STEP or BRIDGE); the density must be a sum of up to four GAUSS
 * terms; the boundary map IDENTITY, AFFINE or ANNULUS.  A request walks
 * exactly the paths an sdd_interface_estimate call (SDD_FP32, path_begin 0,
 * the request's nodes, N = its paths per node) walks, and its node
 * estimates are bitwise those of that call.  A request's device footprint
 * (nodes, sums, interface lines, mesh, subdomain workspace) comes from an
 * arena of hbm_budget_bytes allocated once at creation; a request is
 * admitted first come, first served when a slot and enough arena are free.
 * The server also holds pinned host staging of
 * max_slots x (max_nodes x 112 + max_points x 16) bytes.  A scheduler thread owns the device work; every call below is
 * thread-safe.  Times are seconds on the server's steady clock. */
typedef struct {
    sdd_density w;
    sdd_bmap bmap;
    sdd_layout layout;
    int32_t k;          /* interface points per segment */
    int32_t placement;  /* 0 uniform, 1 equidistributed */
    int32_t interp;     /* 0 linear, 1 monotone cubic */
    int32_t exit_test;  /* sdd_exit_test */
    double dt;
    double se_target;       /* > 0: paths from a pilot; <= 0: paths_per_node */
    int64_t paths_per_node; /* used when se_target <= 0 */
    uint64_t seed;
    double t_max;           /* step cap in time units; <= 0 selects 8 */
} sdd_request;

typedef struct {
    int32_t status; /* SDD_OK, SDD_WARN_CAPPED (done; some paths capped), SDD_ECANCELED or an error */
    int32_t pad;
    int64_t n_nodes, paths_per_node, steps, capped;
    double max_se;  /* largest node standard error over both components */
    double t_submit, t_admit, t_done; /* t_done: the mesh is in the caller's buffer */
    /* stage times in ms (Sec. 5: T_stoc, T_sub): waiting for admission
     * (host clock); the request's walks, from the start of the first walk
     * launch holding one of its blocks to the end of the last (device
     * events; other requests share those launches); finalize + interface
     * fill; subdomain solves */
    double t_queue_ms, t_stoc_ms, t_fill_ms, t_sub_ms;
} sdd_result;

typedef struct sdd_server sdd_server;

/* max_slots requests in flight at once (1..256); requests of up to max_nodes
 * interface points and max_points mesh nodes (nx * ny); launch_paths paths
 * per walk launch (0 selects 2^25).  SDD_EINVAL on bad limits, SDD_EDEVICE
 * when the device or pinned memory cannot be allocated. */
sdd_status sdd_server_create(sdd_ctx* ctx, size_t hbm_budget_bytes, int32_t max_slots, int64_t max_nodes,
                             int64_t max_points, int64_t launch_paths, sdd_server** out);

/* Queue a request (copied); never blocks on device work.  mesh: host
 * [ny][nx][2], caller-owned, written before the request reports done.
 * SDD_EINVAL for an invalid or oversized request, SDD_EUNSUPPORTED for a
 * density or map kind the server does not walk. */
sdd_status sdd_server_submit(sdd_server* srv, const sdd_request* req, double* mesh, uint64_t* id);

/* SDD_EAGAIN until the request is done; then fills *out and returns its
 * status (the id is released).  SDD_EINVAL for an unknown id. */
sdd_status sdd_server_poll(sdd_server* srv, uint64_t id, sdd_result* out);

/* As poll, but blocks until the request is done. */
sdd_status sdd_server_wait(sdd_server* srv, uint64_t id, sdd_result* out);

/* Cancel a queued or running request: it finishes with SDD_ECANCELED
 * once its in-flight blocks have drained, its mesh untouched. */
sdd_status sdd_server_cancel(sdd_server* srv, uint64_t id);

/* Seconds on the server's clock (the clock of sdd_result). */
double sdd_server_clock(sdd_server* srv);

/* Cancel everything pending, drain the device, free all memory. */
sdd_status sdd_server_destroy(sdd_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* SDD_H */
