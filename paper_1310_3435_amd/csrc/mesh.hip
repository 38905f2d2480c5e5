// mesh.hip -- interface placement, edge data, interface fill and the
// batched finite-difference subdomain solves (gfx950).
//
// Sec. 2.1 (Fig. 1): interface points of a non-overlapping decomposition;
// Sec. 3.6: estimates at a few points plus interpolation along each
// interface, points placed from the density; Sec. 3.2: centred finite
// differences for the single-domain and subdomain solves, with tangential
// boundary values from the one-dimensional generator.
#include "common.h"
#include "kernels.h"

namespace sdd {

// ----------------------------------------------------------- block scans

// Inclusive prefix sum over a block of `nthreads` (multiple of 64, <= 1024)
// per-thread values; returns this thread's inclusive value.
__device__ inline double block_inclusive_scan(double v, double* wave_tot)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) {
        const double u = __shfl_up(v, m, kWave);
        if (lane >= m) v += u;
    }
    if (lane == kWave - 1) wave_tot[w] = v;
    __syncthreads();
    double off = 0.0;
    for (int i = 0; i < w; ++i) off += wave_tot[i];
    __syncthreads();
    return v + off;
}

// Cumulative Simpson integral of f along a line: F[0] = 0,
// F[q+1] = F[q] + h/6 (f(s_q) + 4 f(s_q + h/2) + f(s_{q+1})),
// s_q = a + ((b - a) q) / M.  F has M+1 entries (global or shared memory).
template <typename Fn>
__device__ void cumulative_simpson(Fn f, double a, double b, int M, double* F, double* wave_tot)
{
    const int T = blockDim.x;
    const int per = (M + T - 1) / T;
    const int q0 = threadIdx.x * per;
    const int q1 = min(q0 + per, M);
    const double h = (b - a) / M;
    double local = 0.0;
    for (int q = q0; q < q1; ++q) {
        const double s0 = a + ((b - a) * q) / M;
        const double s1 = a + ((b - a) * (q + 1)) / M;
        local += (h / 6.0) * (f(s0) + 4.0 * f(s0 + 0.5 * h) + f(s1));
    }
    const double incl = block_inclusive_scan(local, wave_tot);
    double run = incl - local;
    for (int q = q0; q < q1; ++q) {
        const double s0 = a + ((b - a) * q) / M;
        const double s1 = a + ((b - a) * (q + 1)) / M;
        run += (h / 6.0) * (f(s0) + 4.0 * f(s0 + 0.5 * h) + f(s1));
        F[q + 1] = run;
    }
    if (threadIdx.x == 0) F[0] = 0.0;
    __syncthreads();
}

// ------------------------------------------------------------ placement

constexpr int kPlacePanels = 4096;

// Block 0: crosspoints.  Blocks 1..: one segment each (vertical segments
// first, then horizontal), k points per segment.
__global__ __launch_bounds__(256) void layout_nodes_kernel(sdd_layout L, int k, int placement, const Density D,
                                                           double* __restrict__ nodes)
{
    __shared__ double F[kPlacePanels + 1];
    __shared__ double wave_tot[256 / kWave];
    const int sx = L.sx, sy = L.sy;
    const int ncross = (sx - 1) * (sy - 1);
    if (blockIdx.x == 0) {
        for (int c = threadIdx.x; c < ncross; c += blockDim.x) {
            const int a = 1 + c % (sx - 1), b = 1 + c / (sx - 1);
            nodes[2 * c] = (double)a / sx;
            nodes[2 * c + 1] = (double)b / sy;
        }
        return;
    }
    const int seg = blockIdx.x - 1;
    const int nvert = (sx - 1) * sy;
    bool vertical;
    double fixed, a0, a1;
    if (seg < nvert) {
        vertical = true;
        const int a = 1 + seg / sy, b = seg % sy;
        fixed = (double)a / sx;
        a0 = (double)b / sy;
        a1 = (double)(b + 1) / sy;
    } else {
        vertical = false;
        const int h = seg - nvert;
        const int b = 1 + h / sx, a = h % sx;
        fixed = (double)b / sy;
        a0 = (double)a / sx;
        a1 = (double)(a + 1) / sx;
    }
    double* out = nodes + 2 * ((int64_t)ncross + (int64_t)seg * k);
    if (placement == 0) {
        for (int i = threadIdx.x; i < k; i += blockDim.x) {
            const double s = a0 + ((a1 - a0) * (i + 1)) / (k + 1);
            out[2 * i] = vertical ? fixed : s;
            out[2 * i + 1] = vertical ? s : fixed;
        }
        return;
    }
    auto w = [&](double s) { return vertical ? density_value(D, fixed, s) : density_value(D, s, fixed); };
    cumulative_simpson(w, a0, a1, kPlacePanels, F, wave_tot);
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const double T = (F[kPlacePanels] * (i + 1)) / (k + 1);
        // largest q with F[q] <= T
        int lo = 0, hi = kPlacePanels;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (F[mid] <= T) lo = mid; else hi = mid;
        }
        const int q = min(lo, kPlacePanels - 1);
        const double s0 = a0 + ((a1 - a0) * q) / kPlacePanels;
        const double s1 = a0 + ((a1 - a0) * (q + 1)) / kPlacePanels;
        const double s = s0 + (s1 - s0) * (T - F[q]) / (F[q + 1] - F[q]);
        out[2 * i] = vertical ? fixed : s;
        out[2 * i + 1] = vertical ? s : fixed;
    }
}

hipError_t launch_layout_nodes(const sdd_layout& L, int k, int placement, const Density& D, double* nodes,
                               hipStream_t stream)
{
    const int nseg = (L.sx - 1) * L.sy + (L.sy - 1) * L.sx;
    hipLaunchKernelGGL(layout_nodes_kernel, dim3(1 + nseg), dim3(256), 0, stream, L, k, placement, D, nodes);
    return hipGetLastError();
}

// Placement at the extrema of the density's first and second derivatives
// along each segment (Sec. 3.6).  One block per segment: the derivative
// along the line from the analytic gradient at 4097 samples and the second
// derivative from its central differences, both in LDS; strict local
// extrema of either on the samples, moved to the vertex of the parabola
// through their three samples; sorted; a point closer than one sample to
// the previous kept one is dropped.  counts[s] = points kept; the segment's
// cap slots hold them in increasing order, then (-1, -1).  At most
// kExtremaMax extrema of each derivative are examined per segment.
constexpr int kExtremaPanels = 4096;
constexpr int kExtremaMax = 64;

__device__ __forceinline__ double parabola_vertex(const double* f, int q, double sq, double h)
{
    const double delta = 0.5 * (f[q - 1] - f[q + 1]) / (f[q - 1] - 2.0 * f[q] + f[q + 1]);
    return sq + delta * h;
}

__global__ __launch_bounds__(256) void layout_extrema_kernel(sdd_layout L, int cap, const Density D,
                                                             double* __restrict__ nodes, int32_t* __restrict__ counts)
{
    __shared__ double f1[kExtremaPanels + 1];
    __shared__ double f2[kExtremaPanels + 1];
    __shared__ double cand[2 * kExtremaMax];
    __shared__ int ncand[2];
    __shared__ int kept;
    const int sx = L.sx, sy = L.sy;
    const int ncross = (sx - 1) * (sy - 1);
    if (blockIdx.x == 0) {
        for (int c = threadIdx.x; c < ncross; c += blockDim.x) {
            const int a = 1 + c % (sx - 1), b = 1 + c / (sx - 1);
            nodes[2 * c] = (double)a / sx;
            nodes[2 * c + 1] = (double)b / sy;
        }
        return;
    }
    const int seg = blockIdx.x - 1;
    const int nvert = (sx - 1) * sy;
    bool vertical;
    double fixed, a0, a1;
    if (seg < nvert) {
        vertical = true;
        const int a = 1 + seg / sy, b = seg % sy;
        fixed = (double)a / sx;
        a0 = (double)b / sy;
        a1 = (double)(b + 1) / sy;
    } else {
        vertical = false;
        const int hs = seg - nvert;
        const int b = 1 + hs / sx, a = hs % sx;
        fixed = (double)b / sy;
        a0 = (double)a / sx;
        a1 = (double)(a + 1) / sx;
    }
    const int M = kExtremaPanels;
    const double h = (a1 - a0) / M;
    auto sample = [&](int q) { return a0 + ((a1 - a0) * q) / M; };
    if (threadIdx.x < 2) ncand[threadIdx.x] = 0;
    for (int q = threadIdx.x; q <= M; q += blockDim.x) {
        const double sq = sample(q);
        double w, gx, gy;
        density_grad(D, vertical ? fixed : sq, vertical ? sq : fixed, w, gx, gy);
        f1[q] = vertical ? gy : gx;
    }
    __syncthreads();
    for (int q = threadIdx.x; q <= M; q += blockDim.x)
        f2[q] = (q >= 1 && q <= M - 1) ? (f1[q + 1] - f1[q - 1]) / (2.0 * h) : 0.0;
    __syncthreads();
    for (int q = threadIdx.x; q <= M; q += blockDim.x) {
        if (q >= 1 && q <= M - 1 && (f1[q] - f1[q - 1]) * (f1[q + 1] - f1[q]) < 0.0) {
            const int slot = atomicAdd(&ncand[0], 1);
            if (slot < kExtremaMax) cand[slot] = parabola_vertex(f1, q, sample(q), h);
        }
        if (q >= 2 && q <= M - 2 && (f2[q] - f2[q - 1]) * (f2[q + 1] - f2[q]) < 0.0) {
            const int slot = atomicAdd(&ncand[1], 1);
            if (slot < kExtremaMax) cand[kExtremaMax + slot] = parabola_vertex(f2, q, sample(q), h);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int n1 = min(ncand[0], kExtremaMax), n2 = min(ncand[1], kExtremaMax);
        // gather both lists at the front, insertion sort, drop near duplicates
        for (int i = 0; i < n2; ++i) cand[n1 + i] = cand[kExtremaMax + i];
        const int n = n1 + n2;
        for (int i = 1; i < n; ++i) {
            const double v = cand[i];
            int j = i - 1;
            while (j >= 0 && cand[j] > v) {
                cand[j + 1] = cand[j];
                --j;
            }
            cand[j + 1] = v;
        }
        int m = 0;
        for (int i = 0; i < n; ++i)
            if (m == 0 || cand[i] - cand[m - 1] >= h) cand[m++] = cand[i];
        kept = m;
        counts[seg] = m;
    }
    __syncthreads();
    double* out = nodes + 2 * ((int64_t)ncross + (int64_t)seg * cap);
    for (int i = threadIdx.x; i < cap; i += blockDim.x) {
        if (i < kept) {
            out[2 * i] = vertical ? fixed : cand[i];
            out[2 * i + 1] = vertical ? cand[i] : fixed;
        } else {
            out[2 * i] = -1.0;
            out[2 * i + 1] = -1.0;
        }
    }
}

hipError_t launch_layout_extrema(const sdd_layout& L, int cap, const Density& D, double* nodes, int32_t* counts,
                                 hipStream_t stream)
{
    const int nseg = (L.sx - 1) * L.sy + (L.sy - 1) * L.sx;
    hipLaunchKernelGGL(layout_extrema_kernel, dim3(1 + nseg), dim3(256), 0, stream, L, cap, D, nodes, counts);
    return hipGetLastError();
}

// ------------------------------------------------------------ edge data

// One block per side; table[side][q] = (normal, tangential) per the side.
__global__ __launch_bounds__(1024) void edge1d_kernel(const Density D, int n, double* __restrict__ table)
{
    __shared__ double wave_tot[1024 / kWave];
    const int side = blockIdx.x;
    const double fixed = (side & 1) ? 1.0 : 0.0;
    double* T = table + (size_t)side * n * 2;
    // cumulative integral of 1/w into the tangential slot, via a scratch
    // pass over the normal slot of the same rows
    double* F = T;  // written with stride 2 below
    auto inv_w = [&](double s) {
        return 1.0 / ((side < 2) ? density_value(D, fixed, s) : density_value(D, s, fixed));
    };
    // the scan helper writes contiguous F; use the table rows as scratch by
    // running it on a strided view
    const int M = n - 1;
    const int Tn = blockDim.x;
    const int per = (M + Tn - 1) / Tn;
    const int q0 = threadIdx.x * per;
    const int q1 = min(q0 + per, M);
    const double h = 1.0 / M;
    double local = 0.0;
    for (int q = q0; q < q1; ++q) {
        const double s0 = (1.0 * q) / M, s1 = (1.0 * (q + 1)) / M;
        local += (h / 6.0) * (inv_w(s0) + 4.0 * inv_w(s0 + 0.5 * h) + inv_w(s1));
    }
    const double incl = block_inclusive_scan(local, wave_tot);
    double run = incl - local;
    for (int q = q0; q < q1; ++q) {
        const double s0 = (1.0 * q) / M, s1 = (1.0 * (q + 1)) / M;
        run += (h / 6.0) * (inv_w(s0) + 4.0 * inv_w(s0 + 0.5 * h) + inv_w(s1));
        F[2 * (q + 1)] = run;
    }
    if (threadIdx.x == 0) F[0] = 0.0;
    __syncthreads();
    __shared__ double total;
    if (threadIdx.x == 0) total = F[2 * M];
    __syncthreads();
    const double tot = total;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const double u = F[2 * q] / tot;
        if (side < 2) {
            T[2 * q] = fixed;
            T[2 * q + 1] = u;
        } else {
            T[2 * q] = u;
            T[2 * q + 1] = fixed;
        }
    }
}

hipError_t launch_edge1d_table(const Density& D, int n, double* table, hipStream_t stream)
{
    hipLaunchKernelGGL(edge1d_kernel, dim3(4), dim3(1024), 0, stream, D, n, table);
    return hipGetLastError();
}

// ------------------------------------------------------------ interface fill

__device__ inline double sgn(double v) { return (v > 0.0) - (v < 0.0); }

// Knot m of a segment: 0 = start, 1..k = nodes, k+1 = end.
struct Segment {
    double t0, t1;            // parameter of start and end
    double v0[2], v1[2];      // values at start and end
    const double* nodes;      // this segment's k nodes [k][2]
    const double* values;     // their estimates [k][2]
    int k;
    int axis;                 // parameter coordinate inside a node (1 for vertical lines)
    __device__ double t(int m) const { return m == 0 ? t0 : (m == k + 1 ? t1 : nodes[2 * (m - 1) + axis]); }
    __device__ double v(int m, int c) const
    {
        return m == 0 ? v0[c] : (m == k + 1 ? v1[c] : values[2 * (m - 1) + c]);
    }
};

// Shape-preserving knot slope (Fritsch-Carlson with the Fritsch-Butland
// harmonic mean inside, three-point end slopes limited as in Moler's pchip).
__device__ double pchip_slope(const Segment& S, int j, int c)
{
    const int n = S.k + 2;
    auto h = [&](int i) { return S.t(i + 1) - S.t(i); };
    auto del = [&](int i) { return (S.v(i + 1, c) - S.v(i, c)) / h(i); };
    if (n == 2) return del(0);
    if (j > 0 && j < n - 1) {
        const double a = del(j - 1), b = del(j);
        if (a == 0.0 || b == 0.0 || ((a > 0.0) != (b > 0.0))) return 0.0;
        const double w1 = 2.0 * h(j) + h(j - 1);
        const double w2 = h(j) + 2.0 * h(j - 1);
        return (w1 + w2) / (w1 / a + w2 / b);
    }
    double h0, h1, d0, d1;
    if (j == 0) {
        h0 = h(0); h1 = h(1); d0 = del(0); d1 = del(1);
    } else {
        h0 = h(n - 2); h1 = h(n - 3); d0 = del(n - 2); d1 = del(n - 3);
    }
    const double e = ((2.0 * h0 + h1) * d0 - h0 * d1) / (h0 + h1);
    if (sgn(e) != sgn(d0)) return 0.0;
    if (sgn(d0) != sgn(d1) && fabs(e) > 3.0 * fabs(d0)) return 3.0 * d0;
    return e;
}

__device__ void interp_at(const Segment& S, double t, int interp, double out[2])
{
    // largest m in [0, k] with t_m <= t
    int lo = 0, hi = S.k + 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (S.t(mid) <= t) lo = mid; else hi = mid;
    }
    const int m = lo;
    const double tm = S.t(m), tn = S.t(m + 1);
    const double h = tn - tm;
    const double tau = (t - tm) / h;
    for (int c = 0; c < 2; ++c) {
        const double a = S.v(m, c), b = S.v(m + 1, c);
        if (interp == 0) {
            out[c] = a + tau * (b - a);
        } else {
            const double dm = pchip_slope(S, m, c), dn = pchip_slope(S, m + 1, c);
            const double t2 = tau * tau, t3 = t2 * tau;
            const double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + tau;
            const double h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
            out[c] = h00 * a + h10 * h * dm + h01 * b + h11 * h * dn;
        }
    }
}

// One thread per point of every interface line.
__global__ __launch_bounds__(256) void fill_kernel(sdd_layout L, int k, const int32_t* __restrict__ counts,
                                                   const Bmap B, const double* __restrict__ nodes,
                                                   const double* __restrict__ values, int interp,
                                                   double* __restrict__ vert, double* __restrict__ horiz)
{
    const int nx = L.nx, ny = L.ny, sx = L.sx, sy = L.sy;
    const int mx = (nx - 1) / sx, my = (ny - 1) / sy;
    const int ncross = (sx - 1) * (sy - 1);
    const int64_t nv = (int64_t)(sx - 1) * ny;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nv + (int64_t)(sy - 1) * nx) return;
    const bool vertical = id < nv;
    int line, j, n_along, m_cells, s_cnt, s_other;
    if (vertical) {
        line = 1 + (int)(id / ny);
        j = (int)(id % ny);
        n_along = ny; m_cells = my; s_cnt = sy; s_other = sx;
    } else {
        const int64_t h = id - nv;
        line = 1 + (int)(h / nx);
        j = (int)(h % nx);
        n_along = nx; m_cells = mx; s_cnt = sx; s_other = sy;
    }
    const double fixed = (double)line / s_other;
    double* out = vertical ? vert + ((int64_t)(line - 1) * ny + j) * 2 : horiz + ((int64_t)(line - 1) * nx + j) * 2;
    auto point = [&](double t, double& xi, double& eta) {
        xi = vertical ? fixed : t;
        eta = vertical ? t : fixed;
    };
    auto cross = [&](int other) -> const double* {
        // crosspoint where this line meets perpendicular line `other`
        const int a = vertical ? line : other, b = vertical ? other : line;
        return values + 2 * ((int64_t)(b - 1) * (sx - 1) + (a - 1));
    };
    auto bval = [&](double t, double v[2]) {
        double xi, eta;
        point(t, xi, eta);
        bmap_eval(B, boundary_side(xi, eta), xi, eta, v[0], v[1]);
    };
    if (j == 0 || j == n_along - 1) {
        double v[2];
        bval(j == 0 ? 0.0 : 1.0, v);
        out[0] = v[0];
        out[1] = v[1];
        return;
    }
    if (j % m_cells == 0) {
        const double* c = cross(j / m_cells);
        out[0] = c[0];
        out[1] = c[1];
        return;
    }
    const int seg = j / m_cells;
    Segment S;
    S.k = k;
    S.axis = vertical ? 1 : 0;
    S.t0 = (double)seg / s_cnt;
    S.t1 = (double)(seg + 1) / s_cnt;
    if (seg == 0) {
        bval(0.0, S.v0);
    } else {
        const double* c = cross(seg);
        S.v0[0] = c[0];
        S.v0[1] = c[1];
    }
    if (seg == s_cnt - 1) {
        bval(1.0, S.v1);
    } else {
        const double* c = cross(seg + 1);
        S.v1[0] = c[0];
        S.v1[1] = c[1];
    }
    const int64_t first = vertical ? (int64_t)(line - 1) * sy + seg
                                   : (int64_t)(sx - 1) * sy + (int64_t)(line - 1) * sx + seg;
    S.nodes = nodes + 2 * (ncross + first * k);
    S.values = values + 2 * (ncross + first * k);
    if (counts) S.k = min(counts[first], k);  // k slots per segment, the first counts[] used
    const double t = (double)j / (n_along - 1);
    double v[2];
    interp_at(S, t, interp, v);
    out[0] = v[0];
    out[1] = v[1];
}

hipError_t launch_fill(const sdd_layout& L, int k, const int32_t* counts, const Bmap& B, const double* nodes,
                       const double* values, int interp, double* vert, double* horiz, hipStream_t stream)
{
    const int64_t total = (int64_t)(L.sx - 1) * L.ny + (int64_t)(L.sy - 1) * L.nx;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, L, k, counts, B,
                       nodes, values, interp, vert, horiz);
    return hipGetLastError();
}

// ------------------------------------------------------------ subdomains

// Boundary ring from the map and interface lines from the fill.
__global__ __launch_bounds__(256) void frame_kernel(sdd_layout L, const Bmap B, const double* __restrict__ vert,
                                                    const double* __restrict__ horiz, double* __restrict__ mesh)
{
    const int nx = L.nx, ny = L.ny;
    const int mx = (nx - 1) / L.sx, my = (ny - 1) / L.sy;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)nx * ny) return;
    const int i = (int)(id % nx), j = (int)(id / nx);
    double* o = mesh + 2 * id;
    if (j % my == 0 && j != 0 && j != ny - 1) {
        const double* h = horiz + ((int64_t)(j / my - 1) * nx + i) * 2;
        o[0] = h[0];
        o[1] = h[1];
        return;
    }
    if (i % mx == 0 && i != 0 && i != nx - 1) {
        const double* v = vert + ((int64_t)(i / mx - 1) * ny + j) * 2;
        o[0] = v[0];
        o[1] = v[1];
        return;
    }
    if (i == 0 || i == nx - 1 || j == 0 || j == ny - 1) {
        const double xi = (double)i / (nx - 1), eta = (double)j / (ny - 1);
        bmap_eval(B, boundary_side(xi, eta), xi, eta, o[0], o[1]);
    }
}

// Every interior node of the grid, row by row (Sec. 3.3: Monte Carlo at
// every grid point).
__global__ __launch_bounds__(256) void grid_nodes_kernel(int nx, int ny, double* __restrict__ nodes)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int w = nx - 2;
    if (id >= (int64_t)w * (ny - 2)) return;
    const int i = 1 + (int)(id % w), j = 1 + (int)(id / w);
    nodes[2 * id] = (double)i / (nx - 1);
    nodes[2 * id + 1] = (double)j / (ny - 1);
}

// Boundary ring from the map, interior from per-node estimates in the
// order of grid_nodes_kernel.
__global__ __launch_bounds__(256) void assemble_kernel(int nx, int ny, const Bmap B, const double* __restrict__ values,
                                                       double* __restrict__ mesh)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)nx * ny) return;
    const int i = (int)(id % nx), j = (int)(id / nx);
    double* o = mesh + 2 * id;
    if (i == 0 || i == nx - 1 || j == 0 || j == ny - 1) {
        const double xi = (double)i / (nx - 1), eta = (double)j / (ny - 1);
        bmap_eval(B, boundary_side(xi, eta), xi, eta, o[0], o[1]);
    } else {
        const double* v = values + 2 * ((int64_t)(j - 1) * (nx - 2) + (i - 1));
        o[0] = v[0];
        o[1] = v[1];
    }
}

hipError_t launch_grid_nodes(int nx, int ny, double* nodes, hipStream_t stream)
{
    const int64_t n = (int64_t)(nx - 2) * (ny - 2);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(grid_nodes_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, nx, ny, nodes);
    return hipGetLastError();
}

hipError_t launch_assemble(int nx, int ny, const Bmap& B, const double* values, double* mesh, hipStream_t stream)
{
    const int64_t n = (int64_t)nx * ny;
    hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, nx, ny, B, values,
                       mesh);
    return hipGetLastError();
}

// Initial guess for every subdomain interior: the transfinite (Coons)
// interpolant of the subdomain's four sides.
__global__ __launch_bounds__(256) void coons_kernel(sdd_layout L, double* __restrict__ mesh)
{
    const int nx = L.nx, ny = L.ny;
    const int mx = (nx - 1) / L.sx, my = (ny - 1) / L.sy;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)nx * ny) return;
    const int i = (int)(id % nx), j = (int)(id / nx);
    if (i % mx == 0 || j % my == 0) return;
    const int i0 = (i / mx) * mx, i1 = i0 + mx, j0 = (j / my) * my, j1 = j0 + my;
    const double u = (double)(i - i0) / mx, v = (double)(j - j0) / my;
    auto at = [&](int a, int b, int c) { return mesh[2 * ((int64_t)b * nx + a) + c]; };
    for (int c = 0; c < 2; ++c) {
        const double side = (1 - u) * at(i0, j, c) + u * at(i1, j, c) + (1 - v) * at(i, j0, c) + v * at(i, j1, c);
        const double corner = (1 - u) * (1 - v) * at(i0, j0, c) + u * (1 - v) * at(i1, j0, c) +
                              (1 - u) * v * at(i0, j1, c) + u * v * at(i1, j1, c);
        mesh[2 * id + c] = side - corner;
    }
}

// Edge coefficients a_E(i,j) = w(xi_{i+1/2}, eta_j)/hx^2 and
// a_N(i,j) = w(xi_i, eta_{j+1/2})/hy^2 of every node.
__global__ __launch_bounds__(256) void coef_kernel(sdd_layout L, const Density D, double* __restrict__ aE,
                                                   double* __restrict__ aN)
{
    const int nx = L.nx, ny = L.ny;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)nx * ny) return;
    const int i = (int)(id % nx), j = (int)(id / nx);
    const double hx = 1.0 / (nx - 1), hy = 1.0 / (ny - 1);
    const double xi = i / (double)(nx - 1), eta = j / (double)(ny - 1);
    aE[id] = density_value(D, (i + 0.5) / (nx - 1), eta) / (hx * hx);
    aN[id] = density_value(D, xi, (j + 0.5) / (ny - 1)) / (hy * hy);
}

constexpr int kSorBlock = 1024;
constexpr int kSorCheck = 8;

// One block per (subdomain, component).  Red-black SOR; the block holds its
// subdomain's component values in LDS when kLds, else works in `mesh`.
template <bool kLds>
__global__ __launch_bounds__(kSorBlock) void sor_kernel(sdd_layout L, const double* __restrict__ aE,
                                                        const double* __restrict__ aN, double omega, double tol,
                                                        int max_sweeps, double* __restrict__ mesh,
                                                        int32_t* __restrict__ sweeps_out,
                                                        double* __restrict__ resid_out)
{
    extern __shared__ double lds[];
    __shared__ double red[kSorBlock / kWave];
    __shared__ int stop;
    const int nx = L.nx;
    const int mx = (nx - 1) / L.sx, my = (L.ny - 1) / L.sy;
    const int comp = blockIdx.x & 1;
    const int sub = blockIdx.x >> 1;
    const int a = sub % L.sx, b = sub / L.sx;
    const int i0 = a * mx, j0 = b * my;
    const int W = mx + 1;  // local row length
    auto gidx = [&](int li, int lj) { return (int64_t)(j0 + lj) * nx + (i0 + li); };
    double* val = kLds ? lds : nullptr;
    auto ref = [&](int li, int lj) -> double& {
        return kLds ? val[lj * W + li] : mesh[2 * gidx(li, lj) + comp];
    };
    if (kLds) {
        for (int q = threadIdx.x; q < W * (my + 1); q += blockDim.x) {
            const int li = q % W, lj = q / W;
            val[q] = mesh[2 * gidx(li, lj) + comp];
        }
    }
    if (threadIdx.x == 0) stop = 0;
    __syncthreads();
    const int half = mx / 2 + 1;         // candidates per row and colour
    const int ncand = half * (my - 1);
    int sweep = 0;
    double last = 0.0;
    double best = __builtin_inf();  // thread 0 only
    int since = 0;                  // checks since the last halving of the change
    while (sweep < max_sweeps) {
        double dmax = 0.0;
        for (int colour = 0; colour < 2; ++colour) {
            for (int q = threadIdx.x; q < ncand; q += blockDim.x) {
                const int lj = 1 + q / half;
                const int first = (((1 + lj) & 1) == colour) ? 1 : 2;
                const int li = first + 2 * (q % half);
                if (li > mx - 1) continue;
                const int64_t g = gidx(li, lj);
                const double e = aE[g], w = aE[g - 1], n = aN[g], s = aN[g - nx];
                const double old = ref(li, lj);
                const double gs = (e * ref(li + 1, lj) + w * ref(li - 1, lj) + n * ref(li, lj + 1) +
                                   s * ref(li, lj - 1)) / (e + w + n + s);
                const double nv = old + omega * (gs - old);
                ref(li, lj) = nv;
                dmax = fmax(dmax, fabs(nv - old));
            }
            __syncthreads();
        }
        ++sweep;
        if (sweep % kSorCheck == 0 || sweep == max_sweeps) {
            for (int m = kWave / 2; m >= 1; m >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, m, kWave));
            if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = dmax;
            __syncthreads();
            if (threadIdx.x == 0) {
                double r = 0.0;
                for (int i = 0; i < (int)(blockDim.x / kWave); ++i) r = fmax(r, red[i]);
                last = r;
                // converged, or stalled at the rounding floor: no halving of
                // the largest change within 64 checks
                if (r < 0.5 * best) {
                    best = r;
                    since = 0;
                } else {
                    ++since;
                }
                stop = (r <= tol || since >= 64) ? 1 : 0;
                red[0] = r;
            }
            __syncthreads();
            last = red[0];
            if (stop) break;
            __syncthreads();
        }
    }
    if (kLds) {
        for (int q = threadIdx.x; q < W * (my + 1); q += blockDim.x) {
            const int li = q % W, lj = q / W;
            if (li > 0 && li < mx && lj > 0 && lj < my) mesh[2 * gidx(li, lj) + comp] = val[q];
        }
    }
    if (threadIdx.x == 0) {
        sweeps_out[blockIdx.x] = sweep;
        resid_out[blockIdx.x] = last;
    }
}

__global__ void sor_report_kernel(int nsub, const int32_t* __restrict__ sw, const double* __restrict__ rs,
                                  int32_t* __restrict__ sweeps, double* __restrict__ resid)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsub) return;
    if (sweeps) sweeps[s] = max(sw[2 * s], sw[2 * s + 1]);
    if (resid) resid[s] = fmax(rs[2 * s], rs[2 * s + 1]);
}

size_t subdomain_workspace_bytes(const sdd_layout& L)
{
    const size_t nodes = (size_t)L.nx * L.ny;
    const size_t nsub = (size_t)L.sx * L.sy;
    return 2 * nodes * sizeof(double) + 2 * nsub * (sizeof(int32_t) + sizeof(double)) + 256;
}

static size_t lds_limit()
{
    static const size_t lim = [] {  // once (thread-safe initialisation)
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 64 * 1024;
        return (size_t)v;
    }();
    return lim;
}

hipError_t launch_subdomain_solve(const Density& D, const Bmap& B, const sdd_layout& L, const double* vert,
                                  const double* horiz, double tol, int max_sweeps, double* mesh, int32_t* sweeps,
                                  double* resid, void* workspace, hipStream_t stream)
{
    const int64_t nodes = (int64_t)L.nx * L.ny;
    const int nsub = L.sx * L.sy;
    char* ws = (char*)workspace;
    double* aE = (double*)ws;
    double* aN = aE + nodes;
    int32_t* sw = (int32_t*)(aN + nodes);
    double* rs = (double*)(((uintptr_t)(sw + 2 * nsub) + 7) & ~(uintptr_t)7);
    const unsigned nb = (unsigned)((nodes + 255) / 256);
    hipLaunchKernelGGL(frame_kernel, dim3(nb), dim3(256), 0, stream, L, B, vert, horiz, mesh);
    hipLaunchKernelGGL(coons_kernel, dim3(nb), dim3(256), 0, stream, L, mesh);
    hipLaunchKernelGGL(coef_kernel, dim3(nb), dim3(256), 0, stream, L, D, aE, aN);
    const int mx = (L.nx - 1) / L.sx, my = (L.ny - 1) / L.sy;
    // SOR factor from the Jacobi radius of the constant-coefficient problem
    const double hx = 1.0 / (L.nx - 1), hy = 1.0 / (L.ny - 1);
    const double cxx = 1.0 / (hx * hx), cyy = 1.0 / (hy * hy);
    const double pi = 3.14159265358979323846;
    const double rho = (cxx * cos(pi / mx) + cyy * cos(pi / my)) / (cxx + cyy);
    const double omega = 2.0 / (1.0 + sqrt(1.0 - rho * rho));
    const size_t lds = (size_t)(mx + 1) * (my + 1) * sizeof(double);
    if (lds + 2048 <= lds_limit()) {
        hipLaunchKernelGGL(sor_kernel<true>, dim3(2 * nsub), dim3(kSorBlock), lds, stream, L, aE, aN, omega, tol,
                           max_sweeps, mesh, sw, rs);
    } else {
        hipLaunchKernelGGL(sor_kernel<false>, dim3(2 * nsub), dim3(kSorBlock), 0, stream, L, aE, aN, omega, tol,
                           max_sweeps, mesh, sw, rs);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sor_report_kernel, dim3((nsub + 255) / 256), dim3(256), 0, stream, nsub, sw, rs, sweeps, resid);
    return hipGetLastError();
}

}  // namespace sdd
