// postprocess.hip -- mesh quality and smoothing (gfx950).
//
// Sec. 3.1, eq. (11): geometric quality Q(K) of every cell; Sec. 3.3: its
// maximum and mean, and the l_inf measure of the density at the nodes of two
// meshes; Sec. 3.4, eq. (12): Perona-Malik anisotropic diffusion of the mesh
// by forward-in-time centred-in-space steps, per subdomain (Sec. 3.5) or on
// the whole grid; Sec. 4: interface values smoothed by local quadratic
// regression before the subdomain solves.
//
// All of these are streaming stencils over the [ny][nx][2] mesh in HBM:
// each node is read a few times through L2 and written once per pass, so
// they are bandwidth and launch bound and finish in microseconds next to
// the walk.  Reductions go through per-block partials in a fixed grid and a
// single finishing block, so results do not depend on scheduling.
#include "common.h"
#include "kernels.h"

namespace sdd {

constexpr int kPostBlock = 256;
constexpr int kPostMaxBlocks = 1024;

static inline size_t align_up_bytes(size_t b) { return (b + 255) & ~(size_t)255; }

__device__ __forceinline__ double block_sum(double v, double* sh)
{
    for (int m = kWave / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < kPostBlock / kWave; ++i) t += sh[i];
    return t;
}

__device__ __forceinline__ double block_max(double v, double* sh)
{
    for (int m = kWave / 2; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, kWave));
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) sh[w] = v;
    __syncthreads();
    double t = sh[0];
    for (int i = 1; i < kPostBlock / kWave; ++i) t = fmax(t, sh[i]);
    return t;
}

int post_blocks(int64_t n)
{
    const int64_t b = (n + kPostBlock - 1) / kPostBlock;
    return (int)(b < 1 ? 1 : b > kPostMaxBlocks ? kPostMaxBlocks : b);
}

size_t post_workspace_bytes() { return (size_t)kPostMaxBlocks * 3 * sizeof(double); }

// ---------------------------------------------------------------- quality

// Q of one cell from its corners: J at the centre of the bilinear map,
// Q = |J|_F^2 / (2 |det J|) (= tr(J^T J) / (2 sqrt(det J^T J))); a cell
// with det J = 0 has Q = inf, also when it has collapsed to a point (J = 0,
// where the quotient is 0/0).
__device__ __forceinline__ double cell_quality(const double2* m, int nx, int i, int j, double ihx, double ihy,
                                               double& detj)
{
    const double2 p00 = m[(size_t)j * nx + i], p10 = m[(size_t)j * nx + i + 1];
    const double2 p01 = m[(size_t)(j + 1) * nx + i], p11 = m[(size_t)(j + 1) * nx + i + 1];
    const double a = ((p10.x + p11.x) - (p00.x + p01.x)) * (0.5 * ihx);  // x_xi
    const double c = ((p10.y + p11.y) - (p00.y + p01.y)) * (0.5 * ihx);  // y_xi
    const double b = ((p01.x + p11.x) - (p00.x + p10.x)) * (0.5 * ihy);  // x_eta
    const double d = ((p01.y + p11.y) - (p00.y + p10.y)) * (0.5 * ihy);  // y_eta
    detj = a * d - b * c;
    return detj != 0.0 ? 0.5 * (a * a + b * b + c * c + d * d) / fabs(detj) : __builtin_inf();
}

__global__ __launch_bounds__(kPostBlock) void quality_kernel(const double2* __restrict__ mesh, int nx, int ny,
                                                             double* __restrict__ q, double* __restrict__ part)
{
    __shared__ double sh[kPostBlock / kWave];
    const int cx = nx - 1;
    const int64_t cells = (int64_t)cx * (ny - 1);
    const double ihx = (double)(nx - 1), ihy = (double)(ny - 1);
    double mx = 0.0, sm = 0.0, folded = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * kPostBlock + threadIdx.x; t < cells; t += (int64_t)gridDim.x * kPostBlock) {
        const int j = (int)(t / cx), i = (int)(t - (int64_t)j * cx);
        double detj;
        const double v = cell_quality(mesh, nx, i, j, ihx, ihy, detj);
        if (q) q[t] = v;
        mx = fmax(mx, v);
        sm += v;
        folded += detj <= 0.0 ? 1.0 : 0.0;
    }
    mx = block_max(mx, sh);
    sm = block_sum(sm, sh);
    folded = block_sum(folded, sh);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = mx;
        part[3 * blockIdx.x + 1] = sm;
        part[3 * blockIdx.x + 2] = folded;
    }
}

// out = {Q_max, Q_mean, folded cells}: the blocks' partials in block order.
__global__ void quality_finish_kernel(const double* __restrict__ part, int nblocks, int64_t cells,
                                      double* __restrict__ out)
{
    if (threadIdx.x != 0) return;
    double mx = 0.0, sm = 0.0, f = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        mx = fmax(mx, part[3 * b]);
        sm += part[3 * b + 1];
        f += part[3 * b + 2];
    }
    out[0] = mx;
    out[1] = sm / (double)cells;
    out[2] = f;
}

hipError_t launch_quality(int nx, int ny, const double* mesh, double* q, double* out, void* ws, hipStream_t stream)
{
    const int64_t cells = (int64_t)(nx - 1) * (ny - 1);
    const int nb = post_blocks(cells);
    double* part = (double*)ws;
    hipLaunchKernelGGL(quality_kernel, dim3(nb), dim3(kPostBlock), 0, stream, (const double2*)mesh, nx, ny, q, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(quality_finish_kernel, dim3(1), dim3(kWave), 0, stream, part, nb, cells, out);
    return hipGetLastError();
}

// --------------------------------------------------------------- compare

__global__ __launch_bounds__(kPostBlock) void compare_kernel(const Density D, const double2* __restrict__ a,
                                                             const double2* __restrict__ b, int64_t n,
                                                             double* __restrict__ part)
{
    __shared__ double sh[kPostBlock / kWave];
    double dw = 0.0, dx = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * kPostBlock + threadIdx.x; t < n; t += (int64_t)gridDim.x * kPostBlock) {
        const double2 p = a[t], r = b[t];
        dw = fmax(dw, fabs(density_value(D, p.x, p.y) - density_value(D, r.x, r.y)));
        dx = fmax(dx, hypot(p.x - r.x, p.y - r.y));
    }
    dw = block_max(dw, sh);
    dx = block_max(dx, sh);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = dw;
        part[3 * blockIdx.x + 1] = dx;
    }
}

__global__ void compare_finish_kernel(const double* __restrict__ part, int nblocks, double* __restrict__ out)
{
    if (threadIdx.x != 0) return;
    double dw = 0.0, dx = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        dw = fmax(dw, part[3 * b]);
        dx = fmax(dx, part[3 * b + 1]);
    }
    out[0] = dw;
    out[1] = dx;
}

hipError_t launch_compare(int nx, int ny, const Density& D, const double* mesh, const double* ref, double* out,
                          void* ws, hipStream_t stream)
{
    const int64_t n = (int64_t)nx * ny;
    const int nb = post_blocks(n);
    double* part = (double*)ws;
    hipLaunchKernelGGL(compare_kernel, dim3(nb), dim3(kPostBlock), 0, stream, D, (const double2*)mesh,
                       (const double2*)ref, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(compare_finish_kernel, dim3(1), dim3(kWave), 0, stream, part, nb, out);
    return hipGetLastError();
}

// ---------------------------------------------------------- Perona-Malik

// One FTCS step, src -> dst, of u_t = div(exp(-|grad u|^2/k^2) grad u) for
// each mesh component; the face coefficient comes from the one-sided
// difference across the face.  Fixed: the boundary ring and, when
// mx > 0, the columns i = ox (mod mx) and rows j = oy (mod my) (the
// interface lines, or those of the subdomains shifted by ox, oy).
__global__ __launch_bounds__(kPostBlock) void smooth_step_kernel(const double2* __restrict__ src,
                                                                 double2* __restrict__ dst, int nx, int ny, int mx,
                                                                 int my, int ox, int oy, double dt_hx2,
                                                                 double dt_hy2, double ihx, double ihy, double ik2)
{
    const int i = blockIdx.x * 16 + (threadIdx.x & 15);
    const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= nx || j >= ny) return;
    const size_t p = (size_t)j * nx + i;
    const double2 P = src[p];
    bool fixed = i == 0 || j == 0 || i == nx - 1 || j == ny - 1;
    if (mx > 0) fixed = fixed || (i % mx) == ox || (j % my) == oy;
    if (fixed) {
        dst[p] = P;
        return;
    }
    const double2 E = src[p + 1], W = src[p - 1], N = src[p + nx], S = src[p - nx];
    double2 out;
    {
        const double dE = E.x - P.x, dW = W.x - P.x, dN = N.x - P.x, dS = S.x - P.x;
        const double gE = dE * ihx, gW = dW * ihx, gN = dN * ihy, gS = dS * ihy;
        const double cE = exp(-gE * gE * ik2), cW = exp(-gW * gW * ik2);
        const double cN = exp(-gN * gN * ik2), cS = exp(-gS * gS * ik2);
        out.x = P.x + ((cE * dE + cW * dW) * dt_hx2 + (cN * dN + cS * dS) * dt_hy2);
    }
    {
        const double dE = E.y - P.y, dW = W.y - P.y, dN = N.y - P.y, dS = S.y - P.y;
        const double gE = dE * ihx, gW = dW * ihx, gN = dN * ihy, gS = dS * ihy;
        const double cE = exp(-gE * gE * ik2), cW = exp(-gW * gW * ik2);
        const double cN = exp(-gN * gN * ik2), cS = exp(-gS * gS * ik2);
        out.y = P.y + ((cE * dE + cW * dW) * dt_hx2 + (cN * dN + cS * dS) * dt_hy2);
    }
    dst[p] = out;
}

hipError_t launch_smooth(const sdd_layout& L, int per_subdomain, double dt, double k, int steps, double* mesh,
                         void* ws, hipStream_t stream)
{
    const int nx = L.nx, ny = L.ny;
    const int mx = per_subdomain ? (nx - 1) / L.sx : 0;
    const int my = per_subdomain ? (ny - 1) / L.sy : 0;
    const int ox = per_subdomain == 2 ? mx / 2 : 0, oy = per_subdomain == 2 ? my / 2 : 0;
    const double ihx = (double)(nx - 1), ihy = (double)(ny - 1);
    const dim3 grid((unsigned)((nx + 15) / 16), (unsigned)((ny + 15) / 16));
    double2* a = (double2*)mesh;
    double2* b = (double2*)ws;
    for (int s = 0; s < steps; ++s) {
        hipLaunchKernelGGL(smooth_step_kernel, grid, dim3(kPostBlock), 0, stream, a, b, nx, ny, mx, my, ox, oy,
                           dt * ihx * ihx, dt * ihy * ihy, ihx, ihy, 1.0 / (k * k));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        double2* t = a;
        a = b;
        b = t;
    }
    if (a != (double2*)mesh)
        return hipMemcpyAsync(mesh, a, (size_t)nx * ny * sizeof(double2), hipMemcpyDeviceToDevice, stream);
    return hipSuccess;
}

// ---------------------------------------------- interface pre-smoothing

// One thread per point of every interface line: the value at the point of
// the quadratic fitted by weighted least squares to the `span` points
// nearest in index (window shifted to stay on the line), tricube weights
// (1 - (|t|/d)^3)^3 with d the largest |t| in the window.  Outer-boundary
// ends and crosspoints (every m-th point) keep their values.  The normal
// equations in the scaled parameter t/d are solved by Cramer's rule.
__global__ __launch_bounds__(kPostBlock) void loess_kernel(const double2* __restrict__ src, double2* __restrict__ dst,
                                                           int lines, int n, int m, int span)
{
    const int64_t t = (int64_t)blockIdx.x * kPostBlock + threadIdx.x;
    if (t >= (int64_t)lines * n) return;
    const int l = (int)(t / n), i = (int)(t - (int64_t)l * n);
    const double2* v = src + (size_t)l * n;
    if (i % m == 0 || i == n - 1) {
        dst[t] = v[i];
        return;
    }
    int a = i - span / 2;
    a = a < 0 ? 0 : a;
    a = a > n - span ? n - span : a;
    const int dmax = max(i - a, a + span - 1 - i);
    const double id = 1.0 / (double)dmax;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
    double2 r0 = make_double2(0, 0), r1 = r0, r2 = r0;
    for (int j = a; j < a + span; ++j) {
        const double u = (double)(j - i) * id;
        const double au = fabs(u);
        const double c = 1.0 - au * au * au;
        const double w = c * c * c;
        const double wu = w * u, wu2 = wu * u;
        s0 += w;
        s1 += wu;
        s2 += wu2;
        s3 += wu2 * u;
        s4 += wu2 * u * u;
        const double2 y = v[j];
        r0.x += w * y.x;
        r0.y += w * y.y;
        r1.x += wu * y.x;
        r1.y += wu * y.y;
        r2.x += wu2 * y.x;
        r2.y += wu2 * y.y;
    }
    // a = det([r0 s1 s2; r1 s2 s3; r2 s3 s4]) / det([s0 s1 s2; s1 s2 s3; s2 s3 s4])
    const double m00 = s2 * s4 - s3 * s3, m01 = s1 * s4 - s2 * s3, m02 = s1 * s3 - s2 * s2;
    const double det = s0 * m00 - s1 * m01 + s2 * m02;
    const double c0 = m00 / det, c1 = -m01 / det, c2 = m02 / det;
    dst[t] = make_double2(c0 * r0.x + c1 * r1.x + c2 * r2.x, c0 * r0.y + c1 * r1.y + c2 * r2.y);
}

hipError_t launch_smooth_interfaces(const sdd_layout& L, int span, double* vert, double* horiz, void* ws,
                                    hipStream_t stream)
{
    const int nx = L.nx, ny = L.ny, sx = L.sx, sy = L.sy;
    char* w = (char*)ws;
    const size_t vbytes = (size_t)(sx - 1) * ny * sizeof(double2);
    const size_t hbytes = (size_t)(sy - 1) * nx * sizeof(double2);
    hipError_t e = hipSuccess;
    if (sx > 1) {
        e = hipMemcpyAsync(w, vert, vbytes, hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) return e;
        const int64_t n = (int64_t)(sx - 1) * ny;
        hipLaunchKernelGGL(loess_kernel, dim3((unsigned)((n + kPostBlock - 1) / kPostBlock)), dim3(kPostBlock), 0,
                           stream, (const double2*)w, (double2*)vert, sx - 1, ny, (ny - 1) / sy, span);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (sy > 1) {
        char* w2 = w + align_up_bytes(vbytes);
        e = hipMemcpyAsync(w2, horiz, hbytes, hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) return e;
        const int64_t n = (int64_t)(sy - 1) * nx;
        hipLaunchKernelGGL(loess_kernel, dim3((unsigned)((n + kPostBlock - 1) / kPostBlock)), dim3(kPostBlock), 0,
                           stream, (const double2*)w2, (double2*)horiz, sy - 1, nx, (nx - 1) / sx, span);
        e = hipGetLastError();
    }
    return e;
}

size_t smooth_interfaces_workspace_bytes(const sdd_layout& L)
{
    return align_up_bytes((size_t)(L.sx - 1) * L.ny * sizeof(double2)) +
           align_up_bytes((size_t)(L.sy - 1) * L.nx * sizeof(double2)) + 256;
}

}  // namespace sdd
