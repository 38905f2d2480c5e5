// walk.hip -- interface Monte Carlo walk (gfx950).
//
// A persistent grid of wavefronts draws path tickets (node g, path p) from a
// device counter, 64 at a time per wave.  One lane walks one path; when its
// path exits, the lane takes the wave's next ticket, whatever node it
// belongs to, so lanes stay busy until the ticket range is exhausted.  A
// loop iteration is one Philox block, i.e. three Euler-Maruyama steps (Sec.
// 2.2) with an exit test after each; a path always starts a block.
// With the Brownian-bridge option the step also exits, with the bridge's
// conditional probability, when both its ends are inside (rng.h).
// At exit the lane stores the last step's endpoints P, Q and the step count
// (with the side of a bridged exit) in the path's own slot.  A second kernel
// projects P -> Q onto the boundary in double, evaluates the boundary map
// there (eq. (7a)) and reduces each node's paths in a fixed order, so every
// result is independent of the schedule, and the walk keeps no
// double-precision state.
//
// The walk itself touches HBM only to read a node at path start and to
// write 20 bytes (float walk) or 36 bytes (double walk) per finished path.
#include <stdlib.h>

#include "common.h"
#include "rng.h"
#include "walk.h"

namespace sdd {

// Noise factor of one step: sqrt(2 dt) times the normals' scale above.
__device__ __forceinline__ float noise_scale(const WalkArgs& A, float) { return (float)A.noise_f32; }
__device__ __forceinline__ double noise_scale(const WalkArgs& A, double) { return A.sqrt2dt; }

template <int KIND>
__device__ __forceinline__ void drift(const Density& D, float x, float y, float& bx, float& by)
{
    drift_f32<KIND>(D, x, y, bx, by);
}
template <int KIND>
__device__ __forceinline__ void drift(const Density& D, double x, double y, double& bx, double& by)
{
    drift_f64<KIND>(D, x, y, bx, by);
}


__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, kWave); }
__device__ __forceinline__ long long shfl_xor_l(long long v, int m) { return __shfl_xor(v, m, kWave); }

__device__ __forceinline__ void store_pq(const WalkArgs& A, uint32_t t, float px, float py, float qx, float qy)
{
    reinterpret_cast<float4*>(A.pq)[t] = make_float4(px, py, qx, qy);
}
__device__ __forceinline__ void store_pq(const WalkArgs& A, uint32_t t, double px, double py, double qx, double qy)
{
    double2* d = reinterpret_cast<double2*>(A.pq) + 2 * (size_t)t;
    d[0] = make_double2(px, py);
    d[1] = make_double2(qx, qy);
}

__device__ __forceinline__ void load_pq(const void* pq, size_t t, float, double& px, double& py, double& qx,
                                        double& qy)
{
    const float4 v = reinterpret_cast<const float4*>(pq)[t];
    px = v.x; py = v.y; qx = v.z; qy = v.w;
}
__device__ __forceinline__ void load_pq(const void* pq, size_t t, double, double& px, double& py, double& qx,
                                        double& qy)
{
    const double2* d = reinterpret_cast<const double2*>(pq) + 2 * t;
    px = d[0].x; py = d[0].y; qx = d[1].x; qy = d[1].y;
}

constexpr uint32_t kTicketBatch = 64;
// Steps below this make paths of thousands of steps (the unit square's exit
// time is O(0.1)); launch choices below are measured on either side of it.
constexpr double kLongPathDt = 2e-5;
constexpr int kWalkBlock = 256;

// Constant of the bridge test: -log2(e)/dt in float, dt in double.
__device__ __forceinline__ float bridge_const(const WalkArgs& A, float) { return (float)(-1.4426950408889634 / A.dt); }
__device__ __forceinline__ double bridge_const(const WalkArgs& A, double) { return A.dt; }

// PIPE: each iteration also computes the next three steps' Philox block (it
// depends on the counters only), so that the waves left at the end of the
// launch have independent work to overlap with the steps' latency; a new
// path then computes its first block when it starts.  The random numbers,
// and hence all results, are the same either way; which kernels it speeds
// up is measured (launch_walk_prec).
template <typename R, int KIND, bool BRIDGE, bool PIPE>
__global__ __launch_bounds__(kWalkBlock) void walk_kernel(const WalkArgs A)
{
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t N = (uint32_t)A.paths;
    const R dt = (R)A.dt;
    const R sd = noise_scale(A, R(0));
    const R bc = bridge_const(A, R(0));

    // wave-uniform ticket pool
    uint32_t pool_lo = 0, pool_hi = 0;
    bool exhausted = false;
    // lane state
    bool live = false;
    uint32_t t = 0, g = 0, pc = 0;  // ticket, node, path counter word
    uint4 rc = make_uint4(0, 0, 0, 0);  // Philox block of the lane's current three steps
    R X = 0, Y = 0;
    uint32_t m = 0;                    // Philox block index: steps 3m .. 3m+2
    const uint32_t mmax = (uint32_t)(A.kmax / 3);

    for (;;) {
        // hand the wave's tickets to idle lanes, in lane order
        uint64_t need = __ballot(!live);
        while (need != 0 && !exhausted) {
            if (pool_lo == pool_hi) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(A.counter, (unsigned long long)kTicketBatch);
                base = __shfl(base, 0, kWave);
                if (base >= A.total) {
                    exhausted = true;
                    break;
                }
                pool_lo = (uint32_t)base;
                pool_hi = (uint32_t)min((unsigned long long)A.total, base + kTicketBatch);
            }
            const uint32_t avail = pool_hi - pool_lo;
            const uint32_t want = (uint32_t)__popcll(need);
            const uint32_t take = want < avail ? want : avail;
            const uint32_t rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
            if (!live && rank < take) {
                t = pool_lo + rank;
                g = t / N;
                pc = (uint32_t)A.path_begin + (t - g * N);
                const double nx0 = A.nodes[2 * (size_t)g], ny0 = A.nodes[2 * (size_t)g + 1];
                if (nx0 > 0.0 && nx0 < 1.0 && ny0 > 0.0 && ny0 < 1.0) {
                    X = (R)nx0;
                    Y = (R)ny0;
                    m = 0;
                    live = true;
                    if constexpr (PIPE) rc = philox(0u, pc, g, 0u, A.key0, A.key1);
                } else {
                    // a node off the open square walks nothing: NaN result
                    const R nan = (R)__builtin_nan("");
                    store_pq(A, t, nan, nan, nan, nan);
                    A.info[t] = 0;
                }
            }
            pool_lo += take;
            need = __ballot(!live);
        }
        if (__ballot(live) == 0) break;

        uint4 r;
        if constexpr (PIPE) {
            r = rc;
            rc = philox(m + 1u, pc, g, 0u, A.key0, A.key1);
        } else {
            r = philox(m, pc, g, 0u, A.key0, A.key1);
        }
        R bx, by, z0, z1;
        // step 3m
        normals(field_hi(r.x, R(0)), field_hi(r.y, R(0)), z0, z1);
        drift<KIND>(A.dens, X, Y, bx, by);
        const R XA = fmar(sd, z0, fmar(bx, dt, X));
        const R YA = fmar(sd, z1, fmar(by, dt, Y));
        // step 3m+1
        normals(field_hi(r.z, R(0)), field_hi(r.w, R(0)), z0, z1);
        drift<KIND>(A.dens, XA, YA, bx, by);
        const R XB = fmar(sd, z0, fmar(bx, dt, XA));
        const R YB = fmar(sd, z1, fmar(by, dt, YA));
        // step 3m+2
        normals(field_lo(r.x, r.y, R(0)), field_lo(r.z, r.w, R(0)), z0, z1);
        drift<KIND>(A.dens, XB, YB, bx, by);
        const R XC = fmar(sd, z0, fmar(bx, dt, XB));
        const R YC = fmar(sd, z1, fmar(by, dt, YB));

        // the step cap is a whole number of blocks, so it can only fall
        // after step 3m+2
        const bool outA = outside(XA, YA);
        const bool outB = outside(XB, YB);
        const bool outC = outside(XC, YC);
        bool exA = outA, exB = outB, exC = outC;
        if constexpr (BRIDGE) {
            const R PA = bridge_prob(X, Y, XA, YA, bc);
            const R PB = bridge_prob(XA, YA, XB, YB, bc);
            const R PC = bridge_prob(XB, YB, XC, YC, bc);
            const bool may = (!outA && bridge_may_exit(PA)) || (!outB && bridge_may_exit(PB)) ||
                             (!outC && bridge_may_exit(PC));
            if (__ballot(live && may) != 0) {
                // some lane is near a wall: draw the bridge block (wave-uniform branch)
                const uint4 q = philox(m, pc, g, 1u, A.key0, A.key1);
                exA = outA || uniform23(q.x, R(0)) < PA;
                exB = outB || uniform23(q.y, R(0)) < PB;
                exC = outC || uniform23(q.z, R(0)) < PC;
            }
        }
        const bool fin = live && (exA || exB || exC || (m + 1u >= mmax));

        if (fin) {
            // the first exiting step's ends; the exit projection and the
            // boundary map run in the reduction
            const R px = exA ? X : (exB ? XA : XB), py = exA ? Y : (exB ? YA : YB);
            const R qx = exA ? XA : (exB ? XB : XC), qy = exA ? YA : (exB ? YB : YC);
            store_pq(A, t, px, py, qx, qy);
            uint32_t w = 3u * m + (exA ? 1u : (exB ? 2u : 3u));
            if (!(exA || exB || exC))
                w |= kInfoCapped;
            else if (BRIDGE && !(exA ? outA : (exB ? outB : outC)))
                w |= kInfoBridged | (bridge_side(px, py, qx, qy) << kInfoSideShift);
            A.info[t] = w;
            live = false;
        }
        // finished and idle lanes carry garbage until their next start
        X = XC;
        Y = YC;
        ++m;
    }
}

__global__ void reset_counter_kernel(unsigned long long* counter) { *counter = 0ull; }

constexpr int kReduceBlock = 256;

__device__ __forceinline__ uint32_t in_info(const uint32_t* info, size_t t) { return info[t]; }

// One block per node.  Each path's last step P -> Q is projected onto the
// boundary in double (first crossing; nearest boundary point for a capped
// path) and mapped through the boundary map; the node's values are summed in
// a fixed order (thread j takes paths j, j+256, ... with compensated sums,
// then a fixed tree), so results do not depend on how the walk was
// scheduled.
template <typename R>
__global__ __launch_bounds__(kReduceBlock) void reduce_kernel(const void* __restrict__ pq,
                                                              const uint32_t* __restrict__ info, int64_t paths,
                                                              const Bmap B, double* __restrict__ mean,
                                                              double* __restrict__ se, double* __restrict__ sums,
                                                              long long* __restrict__ node_tot,
                                                              sdd_path_record* __restrict__ per_path)
{
    __shared__ double part[4][kReduceBlock / kWave];
    __shared__ long long ipart[2][kReduceBlock / kWave];
    const int64_t g = blockIdx.x;
    double s[4] = { 0, 0, 0, 0 }, c[4] = { 0, 0, 0, 0 };
    long long st = 0, cp = 0;
    for (int64_t j = threadIdx.x; j < paths; j += kReduceBlock) {
        const size_t t = (size_t)(g * paths + j);
        double px, py, qx, qy, ex, ey;
        load_pq(pq, t, R(0), px, py, qx, qy);
        const uint32_t w = in_info(info, t);
        const bool capped = (w & kInfoCapped) != 0;
        int side;
        if (w & kInfoBridged) {
            // bridged exit: the end of the step moved onto the wall it crossed
            side = (int)((w >> kInfoSideShift) & 3u);
            ex = side == 0 ? 0.0 : side == 1 ? 1.0 : qx;
            ey = side == 2 ? 0.0 : side == 3 ? 1.0 : qy;
        } else {
            side = capped ? nearest_side(qx, qy, ex, ey) : exit_point(px, py, qx, qy, ex, ey);
        }
        double x, y;
        bmap_eval(B, side, ex, ey, x, y);
        if (px != px) x = y = px;  // node off the square: NaN
        nadd(s[0], c[0], x);
        nadd(s[1], c[1], y);
        nadd(s[2], c[2], x * x);
        nadd(s[3], c[3], y * y);
        st += w & kInfoSteps;
        cp += capped ? 1 : 0;
        if (per_path) {
            sdd_path_record* rec = per_path + t;
            rec->exit_xi = ex;
            rec->exit_eta = ey;
            rec->steps = w & kInfoSteps;
            rec->side = side;
            rec->capped = capped ? 1 : 0;
        }
    }
    double tot[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) tot[q] = s[q] + c[q];
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1) {
#pragma unroll
        for (int q = 0; q < 4; ++q) tot[q] += shfl_xor_d(tot[q], m);
        st += shfl_xor_l(st, m);
        cp += shfl_xor_l(cp, m);
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) part[q][w] = tot[q];
        ipart[0][w] = st;
        ipart[1][w] = cp;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double T[4] = { 0, 0, 0, 0 };
    long long ST = 0, CP = 0;
    for (int i = 0; i < kReduceBlock / kWave; ++i) {
#pragma unroll
        for (int q = 0; q < 4; ++q) T[q] += part[q][i];
        ST += ipart[0][i];
        CP += ipart[1][i];
    }
    const double Nd = (double)paths;
    const double mx = T[0] / Nd, my = T[1] / Nd;
    mean[2 * g] = mx;
    mean[2 * g + 1] = my;
    if (se) {
        if (paths > 1) {
            const double vx = T[2] - Nd * mx * mx, vy = T[3] - Nd * my * my;
            se[2 * g] = sqrt(fmax(vx, 0.0) / (Nd * (Nd - 1.0)));
            se[2 * g + 1] = sqrt(fmax(vy, 0.0) / (Nd * (Nd - 1.0)));
        } else {
            se[2 * g] = 0.0;
            se[2 * g + 1] = 0.0;
        }
    }
    if (sums) {
#pragma unroll
        for (int q = 0; q < 4; ++q) sums[4 * g + q] = T[q];
    }
    node_tot[2 * g] = ST;
    node_tot[2 * g + 1] = CP;
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

template <typename R, int KIND, bool BRIDGE, bool PIPE>
static hipError_t launch_walk_kernel(const WalkArgs& A, hipStream_t stream)
{
    // A persistent grid of a few waves per SIMD (SDD_WALK_WAVES_PER_SIMD
    // overrides; capped by what the device keeps resident), never more than
    // there are tickets.  More waves hide latency better but split the paths
    // over more lanes, and the last, longest paths then leave more lanes
    // idle.  Measured same-box: a single-term kernel runs paths of thousands
    // of steps (dt < 2e-5) 1-4% faster with 3 waves than with 4 (ring,
    // sin^2, sech^2), shorter paths up to 4.5% faster with 4, and loses 2-4%
    // with 6 or 8; the general sum of terms, whose term loop leaves more
    // latency to hide, gains 14-21% from 4 to 8.
    struct Grid {
        int occ, cus, env;
    };
    static const Grid grid = [] {  // once per instance (thread-safe initialisation)
        Grid G{ 2, 256, 0 };
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        if (hipDeviceGetAttribute(&G.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || G.cus <= 0)
            G.cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&G.occ, walk_kernel<R, KIND, BRIDGE, PIPE>, kWalkBlock,
                                                         0) != hipSuccess ||
            G.occ <= 0)
            G.occ = 2;
        const char* env = getenv("SDD_WALK_WAVES_PER_SIMD");
        if (env && atoi(env) > 0) G.env = atoi(env);
        return G;
    }();
    int want = KIND == kAnyTerms ? 8 : A.dt < kLongPathDt ? 3 : 4;  // blocks of 4 waves: one per SIMD
    if (grid.env > 0) want = grid.env;
    const int per_cu_blocks = want < grid.occ ? want : grid.occ;
    const int64_t need = ((int64_t)A.total + kWave - 1) / kWave;
    int64_t blocks = (int64_t)per_cu_blocks * grid.cus;
    const int64_t most = (need + kWalkBlock / kWave - 1) / (kWalkBlock / kWave);
    if (blocks > most) blocks = most;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((walk_kernel<R, KIND, BRIDGE, PIPE>), dim3((unsigned)blocks), dim3(kWalkBlock), 0, stream, A);
    return hipGetLastError();
}

// Single-term densities run a kernel specialised on their kind.
inline int walk_kind(const WalkArgs& A) { return A.dens.n_terms == 1 ? A.dens.kind[0] : kAnyTerms; }

template <typename R, bool BRIDGE, bool PIPE>
static hipError_t launch_walk_kind(const WalkArgs& A, hipStream_t stream)
{
    switch (walk_kind(A)) {
    case SDD_TERM_GAUSS: return launch_walk_kernel<R, SDD_TERM_GAUSS, BRIDGE, PIPE>(A, stream);
    case SDD_TERM_RING: return launch_walk_kernel<R, SDD_TERM_RING, BRIDGE, PIPE>(A, stream);
    case SDD_TERM_SECH2: return launch_walk_kernel<R, SDD_TERM_SECH2, BRIDGE, PIPE>(A, stream);
    case SDD_TERM_SIN2: return launch_walk_kernel<R, SDD_TERM_SIN2, BRIDGE, PIPE>(A, stream);
    default: return launch_walk_kernel<R, kAnyTerms, BRIDGE, PIPE>(A, stream);
    }
}

// Float walks with small steps may compute the next block's Philox beside
// the current steps (PIPE).  Whether that pays depends on how the compiler
// schedules each drift and exit test; measured same-box (1521 nodes,
// steps/s, 4 waves per SIMD, pipelined against plain loop):
//
//   dt = 1e-5      gauss   ring    sech^2  sin^2   sum of terms
//   end of step    -1%     -4%     +5%     +7%     +1.5% (-2% at 8 waves)
//   bridge         -1.5%   +1.5%   -3%     -4%     +4% (0 at 8 waves)
//
// The sum of terms runs 8 waves per SIMD (launch_walk_kernel), where it no
// longer pays.  At dt = 1e-4 and 1e-3 it ties or loses for every kind (up
// to 9%).

inline bool pipe_pays(const WalkArgs& A)
{
    if (!(A.dt < kLongPathDt)) return false;
    const int kind = walk_kind(A);
    if (A.bridge) return kind == SDD_TERM_RING;
    return kind == SDD_TERM_SECH2 || kind == SDD_TERM_SIN2;
}

template <typename R>
static hipError_t launch_walk_prec(const WalkArgs& A, hipStream_t stream)
{
    if constexpr (sizeof(R) == sizeof(float)) {
        if (pipe_pays(A))
            return A.bridge ? launch_walk_kind<R, true, true>(A, stream) : launch_walk_kind<R, false, true>(A, stream);
    }
    return A.bridge ? launch_walk_kind<R, true, false>(A, stream) : launch_walk_kind<R, false, false>(A, stream);
}

hipError_t launch_walk(const WalkArgs& A, int prec, double* mean, double* se, double* sums, sdd_walk_stats* stats,
                       long long* node_tot, hipStream_t stream)
{
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, A.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = (prec == SDD_FP32) ? launch_walk_prec<float>(A, stream) : launch_walk_prec<double>(A, stream);
    if (e != hipSuccess) return e;
    if (prec == SDD_FP32)
        hipLaunchKernelGGL(reduce_kernel<float>, dim3((unsigned)A.n_nodes), dim3(kReduceBlock), 0, stream, A.pq,
                           A.info, A.paths, A.bmap, mean, se, sums, node_tot, A.per_path);
    else
        hipLaunchKernelGGL(reduce_kernel<double>, dim3((unsigned)A.n_nodes), dim3(kReduceBlock), 0, stream, A.pq,
                           A.info, A.paths, A.bmap, mean, se, sums, node_tot, A.per_path);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (stats) {
        hipLaunchKernelGGL(stats_kernel, dim3(1), dim3(1024), 0, stream, node_tot, A.n_nodes, A.paths, stats);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace sdd
