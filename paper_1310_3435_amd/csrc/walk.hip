// walk.hip -- interface Monte Carlo walk (gfx950).
//
// Each wavefront owns one work item: a node g and a chunk of consecutive
// path indices.  One lane walks one path at a time; when its path exits the
// lane takes the chunk's next unassigned path (ballot + mbcnt, so the
// assignment is the same on every run).  A loop iteration is one Philox
// block, i.e. two Euler-Maruyama steps (Sec. 2.2) with an exit test after
// each; a path always starts at an even step, so every lane consumes its
// four random words in the same iteration.  At exit the step's segment is
// projected onto the boundary in double, the boundary map is evaluated there
// (eq. (7a)) and the value enters the lane's compensated double sums.  The
// wave reduces its lanes with cross-lane shuffles and writes one slot per
// item; the finalize kernel adds a node's slots in chunk order.
//
// Nothing on the walk path touches HBM except the node read at the start
// and the slot write at the end (plus optional per-path records).
#include "common.h"
#include "kernels.h"

namespace sdd {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// Philox4x32-10 (Salmon et al., SC'11).  The key schedule is wave-uniform.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Box-Muller pair from two words: u = ((r >> 9) + 1/2) 2^-23 (exact in both
// precisions), (z0, z1) = sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b).
__device__ __forceinline__ void normals(uint32_t ra, uint32_t rb, float& z0, float& z1)
{
    const float ua = __builtin_fmaf((float)(ra >> 9), 0x1p-23f, 0x1p-24f);
    const float ub = __builtin_fmaf((float)(rb >> 9), 0x1p-23f, 0x1p-24f);
    // -2 ln u = -2 ln2 log2 u
    const float radius = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));
    z0 = radius * __builtin_amdgcn_cosf(ub);
    z1 = radius * __builtin_amdgcn_sinf(ub);
}

__device__ __forceinline__ void normals(uint32_t ra, uint32_t rb, double& z0, double& z1)
{
    const double ua = ((double)(ra >> 9) + 0.5) * 0x1p-23;
    const double ub = ((double)(rb >> 9) + 0.5) * 0x1p-23;
    const double radius = sqrt(-2.0 * log(ua));
    double sn, cs;
    sincos(kTwoPi * ub, &sn, &cs);
    z0 = radius * cs;
    z1 = radius * sn;
}

__device__ __forceinline__ void drift(const Density& D, float x, float y, float& bx, float& by)
{
    drift_f32(D, x, y, bx, by);
}
__device__ __forceinline__ void drift(const Density& D, double x, double y, double& bx, double& by)
{
    drift_f64(D, x, y, bx, by);
}

__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ bool outside(float x, float y) { return x <= 0.0f || x >= 1.0f || y <= 0.0f || y >= 1.0f; }
__device__ __forceinline__ bool outside(double x, double y) { return x <= 0.0 || x >= 1.0 || y <= 0.0 || y >= 1.0; }

__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, kWave); }
__device__ __forceinline__ long long shfl_xor_l(long long v, int m) { return __shfl_xor(v, m, kWave); }

template <typename R>
__global__ __launch_bounds__(256) void walk_kernel(const WalkArgs A)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t item = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave;
    if (item >= A.n_items) return;  // whole wave
    const int64_t g = item / A.n_chunks;
    const int64_t chunk = item - g * A.n_chunks;
    const int64_t p_lo = chunk * A.chunk;
    const int32_t count = (int32_t)min((int64_t)A.chunk, A.paths - p_lo);
    Slot* slot = A.slots + item;

    const double node_x = A.nodes[2 * g], node_y = A.nodes[2 * g + 1];
    if (!(node_x > 0.0 && node_x < 1.0 && node_y > 0.0 && node_y < 1.0)) {
        if (lane == 0) {
            const double nan = __builtin_nan("");
            slot->s[0] = slot->s[1] = slot->s[2] = slot->s[3] = nan;
            slot->steps = 0;
            slot->capped = 0;
        }
        return;
    }
    const R x0 = (R)node_x, y0 = (R)node_y;
    const R dt = (R)A.dt;
    const R sd = (R)A.sqrt2dt;
    const uint32_t gw = (uint32_t)g;
    const uint32_t pbase = (uint32_t)(A.path_begin + p_lo);

    int32_t pl = lane;  // path index within the chunk
    bool live = pl < count;
    R X = x0, Y = y0;
    int32_t k = 0;
    int32_t next = kWave;

    double sx = 0, cx = 0, sy = 0, cy = 0, sxx = 0, cxx = 0, syy = 0, cyy = 0;
    long long nsteps = 0;
    int32_t ncapped = 0;

    while (__ballot(live) != 0) {
        const uint4 r = philox((uint32_t)(k >> 1), pbase + (uint32_t)pl, gw, 0u, A.key0, A.key1);
        R bx, by, z0, z1;
        // step 2m
        normals(r.x, r.y, z0, z1);
        drift(A.dens, X, Y, bx, by);
        const R XA = fmar(sd, z0, fmar(bx, dt, X));
        const R YA = fmar(sd, z1, fmar(by, dt, Y));
        // step 2m+1
        normals(r.z, r.w, z0, z1);
        drift(A.dens, XA, YA, bx, by);
        const R XB = fmar(sd, z0, fmar(bx, dt, XA));
        const R YB = fmar(sd, z1, fmar(by, dt, YA));

        const bool outA = outside(XA, YA);
        const bool endA = outA || (k + 1 >= A.kmax);
        const bool outB = outside(XB, YB);
        const bool fin = live && (endA || outB || (k + 2 >= A.kmax));

        const uint64_t fmask = __ballot(fin);
        if (fmask != 0) {
            if (fin) {
                double px, py, qx, qy, ex, ey;
                int32_t steps, side, capped;
                bool exited;
                if (endA) {
                    px = (double)X; py = (double)Y; qx = (double)XA; qy = (double)YA;
                    steps = k + 1;
                    exited = outA;
                } else {
                    px = (double)XA; py = (double)YA; qx = (double)XB; qy = (double)YB;
                    steps = k + 2;
                    exited = outB;
                }
                if (exited) {
                    side = exit_point(px, py, qx, qy, ex, ey);
                    capped = 0;
                } else {
                    side = nearest_side(qx, qy, ex, ey);
                    capped = 1;
                }
                double vx, vy;
                bmap_eval(A.bmap, side, ex, ey, vx, vy);
                nadd(sx, cx, vx);
                nadd(sy, cy, vy);
                nadd(sxx, cxx, vx * vx);
                nadd(syy, cyy, vy * vy);
                nsteps += steps;
                ncapped += capped;
                if (A.per_path) {
                    sdd_path_record* rec = A.per_path + g * A.paths + (p_lo + pl);
                    rec->exit_xi = ex;
                    rec->exit_eta = ey;
                    rec->steps = steps;
                    rec->side = side;
                    rec->capped = capped;
                }
            }
            // refill finished lanes with the chunk's next paths, in lane order
            const uint32_t rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(fmask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)fmask, 0u));
            if (fin) {
                const int32_t np = next + (int32_t)rank;
                if (np < count) {
                    pl = np;
                    X = x0;
                    Y = y0;
                    k = 0;
                } else {
                    live = false;
                }
            }
            next += __popcll(fmask);
        }
        if (live && !fin) {
            X = XB;
            Y = YB;
            k += 2;
        }
    }

    // wave reduction of the lane sums
    double v[4] = { sx + cx, sy + cy, sxx + cxx, syy + cyy };
    long long st = nsteps;
    long long cp = ncapped;
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += shfl_xor_d(v[q], m);
        st += shfl_xor_l(st, m);
        cp += shfl_xor_l(cp, m);
    }
    if (lane == 0) {
        slot->s[0] = v[0];
        slot->s[1] = v[1];
        slot->s[2] = v[2];
        slot->s[3] = v[3];
        slot->steps = st;
        slot->capped = cp;
    }
}

// One thread per node: slots in chunk order, compensated; mean, SE, sums.
__global__ void finalize_kernel(const Slot* __restrict__ slots, int64_t n_nodes, int64_t n_chunks, int64_t paths,
                                double* __restrict__ mean, double* __restrict__ se, double* __restrict__ sums,
                                long long* __restrict__ node_tot)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_nodes) return;
    double s[4] = { 0, 0, 0, 0 }, c[4] = { 0, 0, 0, 0 };
    long long st = 0, cp = 0;
    for (int64_t j = 0; j < n_chunks; ++j) {
        const Slot& S = slots[g * n_chunks + j];
#pragma unroll
        for (int q = 0; q < 4; ++q) nadd(s[q], c[q], S.s[q]);
        st += S.steps;
        cp += S.capped;
    }
    double tot[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) tot[q] = s[q] + c[q];
    const double N = (double)paths;
    const double mx = tot[0] / N, my = tot[1] / N;
    mean[2 * g] = mx;
    mean[2 * g + 1] = my;
    if (se) {
        if (paths > 1) {
            const double vx = tot[2] - N * mx * mx, vy = tot[3] - N * my * my;
            se[2 * g] = sqrt(fmax(vx, 0.0) / (N * (N - 1.0)));
            se[2 * g + 1] = sqrt(fmax(vy, 0.0) / (N * (N - 1.0)));
        } else {
            se[2 * g] = 0.0;
            se[2 * g + 1] = 0.0;
        }
    }
    if (sums) {
#pragma unroll
        for (int q = 0; q < 4; ++q) sums[4 * g + q] = tot[q];
    }
    node_tot[2 * g] = st;
    node_tot[2 * g + 1] = cp;
}

// Single workgroup: totals over nodes (integer sums, order-free).
__global__ __launch_bounds__(1024) void stats_kernel(const long long* __restrict__ node_tot, int64_t n_nodes,
                                                     int64_t paths, sdd_walk_stats* __restrict__ stats)
{
    __shared__ long long part[2][1024 / kWave];
    long long st = 0, cp = 0;
    for (int64_t g = threadIdx.x; g < n_nodes; g += blockDim.x) {
        st += node_tot[2 * g];
        cp += node_tot[2 * g + 1];
    }
    for (int m = kWave / 2; m >= 1; m >>= 1) {
        st += shfl_xor_l(st, m);
        cp += shfl_xor_l(cp, m);
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        part[0][w] = st;
        part[1][w] = cp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long a = 0, b = 0;
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
            a += part[0][i];
            b += part[1][i];
        }
        stats->steps = a;
        stats->paths = n_nodes * paths;
        stats->capped = b;
    }
}

hipError_t launch_walk(const WalkArgs& A, int prec, double* mean, double* se, double* sums, sdd_walk_stats* stats,
                       long long* node_tot, hipStream_t stream)
{
    const int waves_per_block = 4;
    const int64_t blocks = (A.n_items + waves_per_block - 1) / waves_per_block;
    if (prec == SDD_FP32)
        hipLaunchKernelGGL(walk_kernel<float>, dim3((unsigned)blocks), dim3(kWave * waves_per_block), 0, stream, A);
    else
        hipLaunchKernelGGL(walk_kernel<double>, dim3((unsigned)blocks), dim3(kWave * waves_per_block), 0, stream, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int tb = 256;
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((A.n_nodes + tb - 1) / tb)), dim3(tb), 0, stream, A.slots,
                       A.n_nodes, A.n_chunks, A.paths, mean, se, sums, node_tot);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (stats) {
        hipLaunchKernelGGL(stats_kernel, dim3(1), dim3(1024), 0, stream, node_tot, A.n_nodes, A.paths, stats);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace sdd
