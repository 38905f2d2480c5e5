// walk.hip -- launches of the interface walk (walk_core.h) and the
// kernels around it: node sums set-up, finalize and totals.
//
// An estimate call runs four kernels on its stream: acc_init_kernel (zero
// the node sums, set their scale, record the start time), the walk, the
// finalize (means, standard errors, raw sums) and, if asked, the totals.
#include <stdlib.h>

#include "walk_core.h"

namespace sdd {

// ------------------------------------------------------------ set-up

constexpr int kInitBlock = 256;

// Grid-stride zeroing of the node sums.  Block 0 also zeroes the pool
// counter, records the start time and writes the scale: from the host's
// bound, or from the largest |entry| of a TABLE map's table.
__global__ __launch_bounds__(kInitBlock) void acc_init_kernel(NodeAcc* __restrict__ acc, int64_t n,
                                                              AccScale* __restrict__ scale, const Bmap B,
                                                              int host_scale, const AccScale hs,
                                                              unsigned long long* counter,
                                                              unsigned long long* clock0)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (clock0) *clock0 = wall_clock64();
        if (counter) *counter = 0ull;
    }
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        NodeAcc& a = acc[g];
#pragma unroll
        for (int q = 0; q < 4; ++q) a.lo[q] = a.hi[q] = 0ull;
        a.steps = 0ull;
        a.capped = 0ull;
        a.invalid = 0u;
    }
    if (blockIdx.x != 0) return;
    if (host_scale) {
        if (threadIdx.x == 0) *scale = hs;
        return;
    }
    __shared__ double part[kInitBlock / kWave];
    double mx = 0.0;
    const int64_t cnt = (int64_t)4 * B.n * 2;
    for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) mx = fmax(mx, fabs(B.table[i]));
#pragma unroll
    for (int s = kWave / 2; s >= 1; s >>= 1) mx = fmax(mx, __shfl_xor(mx, s, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kInitBlock / kWave; ++i) mx = fmax(mx, part[i]);
        *scale = scale_for_bound(mx);
    }
}

hipError_t launch_acc_init(NodeAcc* acc, int64_t n, AccScale* scale, const Bmap& B, bool host_scale,
                           const AccScale& hs, unsigned long long* counter, unsigned long long* clock0,
                           hipStream_t stream)
{
    int64_t blocks = (n + kInitBlock - 1) / kInitBlock;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(acc_init_kernel, dim3((unsigned)blocks), dim3(kInitBlock), 0, stream, acc, n, scale, B,
                       host_scale ? 1 : 0, hs, counter, clock0);
    return hipGetLastError();
}

__global__ void reset_counter_kernel(unsigned long long* counter) { *counter = 0ull; }

hipError_t launch_reset_counter(unsigned long long* counter, hipStream_t stream)
{
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, counter);
    return hipGetLastError();
}

bool bmap_host_bound(const Bmap& B, double& vmax)
{
    switch (B.kind) {
    case SDD_BMAP_IDENTITY: vmax = 1.0; return true;
    case SDD_BMAP_AFFINE:
        vmax = fmax(fabs(B.p[0]) + fabs(B.p[1]) + fabs(B.p[2]), fabs(B.p[3]) + fabs(B.p[4]) + fabs(B.p[5]));
        return true;
    case SDD_BMAP_ANNULUS: vmax = fmax(fabs(B.p[0]), fabs(B.p[1])); return true;
    default: return false;
    }
}

// ------------------------------------------------------------ finalize

// One thread per node: exact sums -> mean, SE and raw sums (R8:
// SE = sqrt(max(0, S2 - N mean^2) / (N (N - 1))), 0 for N = 1).
__global__ __launch_bounds__(256) void finalize_kernel(const NodeAcc* __restrict__ acc,
                                                       const AccScale* __restrict__ scale, int64_t n, double N,
                                                       double* __restrict__ mean, double* __restrict__ se,
                                                       double* __restrict__ sums)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const NodeAcc& a = acc[g];
    double T[4];
    if (a.invalid) {
#pragma unroll
        for (int q = 0; q < 4; ++q) T[q] = __builtin_nan("");
    } else {
        const AccScale S = *scale;
#pragma unroll
        for (int q = 0; q < 4; ++q) T[q] = limb_value(a.lo[q], a.hi[q]) / S.s[q < 2 ? 0 : 1];
    }
    const double mx = T[0] / N, my = T[1] / N;
    mean[2 * g] = mx;
    mean[2 * g + 1] = my;
    if (se) {
        if (N > 1.0) {
            se[2 * g] = sqrt(fmax(T[2] - N * mx * mx, 0.0) / (N * (N - 1.0)));
            se[2 * g + 1] = sqrt(fmax(T[3] - N * my * my, 0.0) / (N * (N - 1.0)));
            if (a.invalid) se[2 * g] = se[2 * g + 1] = __builtin_nan("");
        } else {
            se[2 * g] = a.invalid ? __builtin_nan("") : 0.0;
            se[2 * g + 1] = se[2 * g];
        }
    }
    if (sums) {
#pragma unroll
        for (int q = 0; q < 4; ++q) sums[4 * g + q] = T[q];
    }
}

// Single workgroup: totals over nodes (integer sums, order-free) and the
// time since clock0.
__global__ __launch_bounds__(1024) void stats_kernel(const NodeAcc* __restrict__ acc, int64_t n, int64_t paths,
                                                     sdd_walk_stats* __restrict__ stats,
                                                     const unsigned long long* __restrict__ clock0, double rate_khz)
{
    __shared__ unsigned long long part[2][1024 / kWave];
    unsigned long long st = 0, cp = 0;
    for (int64_t g = threadIdx.x; g < n; g += blockDim.x) {
        st += acc[g].steps;
        cp += acc[g].capped;
    }
    for (int s = kWave / 2; s >= 1; s >>= 1) {
        st += __shfl_xor(st, s, kWave);
        cp += __shfl_xor(cp, s, kWave);
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        part[0][w] = st;
        part[1][w] = cp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
            a += part[0][i];
            b += part[1][i];
        }
        stats->steps = (int64_t)a;
        stats->paths = n * paths;
        stats->capped = (int64_t)b;
        stats->t_stoc_ms = (clock0 && rate_khz > 0.0) ? (double)(wall_clock64() - *clock0) / rate_khz : 0.0;
    }
}

hipError_t launch_finalize(const NodeAcc* acc, const AccScale* scale, int64_t n, double paths, double* mean,
                           double* se, double* sums, sdd_walk_stats* stats, const unsigned long long* clock0,
                           double wall_rate_khz, hipStream_t stream)
{
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, acc, scale, n,
                       paths, mean, se, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !stats) return e;
    hipLaunchKernelGGL(stats_kernel, dim3(1), dim3(1024), 0, stream, acc, n, (int64_t)paths, stats, clock0,
                       wall_rate_khz);
    return hipGetLastError();
}

// ------------------------------------------------------------ launches

// Steps below this make paths of thousands of steps (the unit square's exit
// time is O(0.1)); launch choices below are measured on either side of it.
constexpr double kLongPathDt = 2e-5;

template <typename R, int KIND, int EXIT, bool PIPE, bool WIDE = false>
static hipError_t launch_walk_kernel(const WalkArgs& A, hipStream_t stream)
{
    // A persistent grid of a few waves per SIMD (SDD_WALK_WAVES_PER_SIMD
    // overrides; capped by what the device keeps resident), never more than
    // there are paths.  More waves hide latency better but split the paths
    // over more lanes, and the last, longest paths then leave more lanes
    // idle.  Measured same-box: a single-term kernel runs paths of thousands
    // of steps (dt < 2e-5) 1-4% faster with 3 waves than with 4 (ring,
    // sin^2), shorter paths up to 4.5% faster with 4, and loses 2-4% with 6
    // or 8.  The sech^2 walk with the end-of-step test, whose exit drain
    // keeps node sums in LDS slots, runs 1.4% faster with 4 (the ring 1.5%
    // slower), so it takes 4 at any dt.  The general sum of terms, whose
    // term loop leaves more latency to hide, runs its 64-VGPR instance with
    // 8 waves on short paths (19% faster than 4 waves of the full-register
    // one at dt = 1e-4, 5% slower at 1e-5, where it keeps the full-register
    // one).
    constexpr auto kernel = [] {
        if constexpr (WIDE)
            return walk_kernel_wide<R, KIND, EXIT>;
        else
            return walk_kernel<R, KIND, EXIT, PIPE, false>;
    }();
    struct Grid {
        int occ, cus, env;
    };
    static const Grid grid = [] {  // once per instance (thread-safe initialisation)
        Grid G{ 2, 256, 0 };
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        if (hipDeviceGetAttribute(&G.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || G.cus <= 0)
            G.cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&G.occ, kernel, kWalkBlock, 0) != hipSuccess ||
            G.occ <= 0)
            G.occ = 2;
        const char* env = getenv("SDD_WALK_WAVES_PER_SIMD");
        if (env && atoi(env) > 0) G.env = atoi(env);
        return G;
    }();
    constexpr bool kSech2Step = KIND == SDD_TERM_SECH2 && EXIT == kExitStep;
    int want = WIDE ? 8 : (KIND == kAnyTerms || kSech2Step) ? 4 : A.dt < kLongPathDt ? 3 : 4;  // blocks of 4 waves: one per SIMD
    if (grid.env > 0) want = grid.env;
    const int per_cu_blocks = want < grid.occ ? want : grid.occ;
    // paths to walk, hence waves worth launching
    const uint64_t paths = (uint64_t)A.seg.n_nodes * (A.seg.p_hi - A.seg.p_lo);
    const uint64_t need = (paths + kWave - 1) / kWave;
    int64_t blocks = (int64_t)per_cu_blocks * grid.cus;
    const uint64_t most = (need + kWavesPerBlock - 1) / kWavesPerBlock;
    if ((uint64_t)blocks > most) blocks = (int64_t)most;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(kWalkBlock), 0, stream, A);
    return hipGetLastError();
}

// Float Gaussian sums take gauss_sum_drift (the request server's drift);
// other single-term densities a kernel specialised on their kind; mixed
// sums the general loop over terms.
inline int walk_kind(const Density& D, int prec)
{
    bool gauss = true;
    for (int t = 0; t < D.n_terms; ++t) gauss = gauss && D.kind[t] == SDD_TERM_GAUSS;
    if (prec == SDD_FP32 && gauss) return kGaussSum;
    if (D.n_terms == 1) return D.kind[0];
    return kAnyTerms;
}

// Float walks with small steps may compute the next block's Philox beside
// the current steps (PIPE).  Whether that pays depends on how the compiler
// schedules each drift and exit test; measured same-box (dt = 1e-5, 3
// waves per SIMD, steps/s, pipelined against plain loop):
//
//                  Gaussian sum   ring    sech^2   sin^2
//   end of step    +7%            -0.6%   -3%      +0.2%
//   bridge         --             +4%     +3%      +5%
//
// (the Gaussian-sum figure on a small job of 53 nodes x 2e4 paths).  The
// general sum of terms takes the plain loop, and on short paths the
// 64-VGPR instance.  At dt = 1e-4 and 1e-3 the pipelined loop tied or lost
// for every kind (up to 9%).
template <int KIND, int EXIT>
static hipError_t launch_f32(const WalkArgs& A, hipStream_t stream)
{
    if constexpr (KIND == kAnyTerms) {
        if (A.dt >= kLongPathDt) return launch_walk_kernel<float, KIND, EXIT, false, true>(A, stream);
    }
    constexpr bool pipe_kind = KIND != kAnyTerms && (EXIT == kExitBridge || (EXIT == kExitStep &&
                                                     (KIND == kGaussSum || KIND == SDD_TERM_SIN2)));
    if constexpr (pipe_kind) {
        if (A.dt < kLongPathDt) return launch_walk_kernel<float, KIND, EXIT, true>(A, stream);
    }
    return launch_walk_kernel<float, KIND, EXIT, false>(A, stream);
}

template <int EXIT>
static hipError_t launch_exit(const WalkArgs& A, int prec, hipStream_t stream)
{
    if (prec == SDD_FP32) {
        switch (walk_kind(A.dens, prec)) {
        case kGaussSum: return launch_f32<kGaussSum, EXIT>(A, stream);
        case SDD_TERM_RING: return launch_f32<SDD_TERM_RING, EXIT>(A, stream);
        case SDD_TERM_SECH2: return launch_f32<SDD_TERM_SECH2, EXIT>(A, stream);
        case SDD_TERM_SIN2: return launch_f32<SDD_TERM_SIN2, EXIT>(A, stream);
        default: return launch_f32<kAnyTerms, EXIT>(A, stream);
        }
    }
    switch (walk_kind(A.dens, prec)) {
    case SDD_TERM_GAUSS: return launch_walk_kernel<double, SDD_TERM_GAUSS, EXIT, false>(A, stream);
    case SDD_TERM_RING: return launch_walk_kernel<double, SDD_TERM_RING, EXIT, false>(A, stream);
    case SDD_TERM_SECH2: return launch_walk_kernel<double, SDD_TERM_SECH2, EXIT, false>(A, stream);
    case SDD_TERM_SIN2: return launch_walk_kernel<double, SDD_TERM_SIN2, EXIT, false>(A, stream);
    default: return launch_walk_kernel<double, kAnyTerms, EXIT, false>(A, stream);
    }
}

hipError_t launch_walk(const WalkArgs& A, int prec, int exit_kind, hipStream_t stream)
{
    switch (exit_kind) {
    case kExitBridge: return launch_exit<kExitBridge>(A, prec, stream);
    case kExitExpo: return launch_exit<kExitExpo>(A, prec, stream);
    default: return launch_exit<kExitStep>(A, prec, stream);
    }
}

// ------------------------------------------------------------ server

int serve_walk_occupancy()
{
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, walk_kernel<float, kGaussSum, kExitLane, false, true>,
                                                     kWalkBlock, 0) != hipSuccess)
        return 0;
    return occ;
}

hipError_t launch_serve_walk(const WalkArgs& A, int blocks, hipStream_t stream)
{
    hipLaunchKernelGGL((walk_kernel<float, kGaussSum, kExitLane, false, true>), dim3((unsigned)blocks),
                       dim3(kWalkBlock), 0, stream, A);
    return hipGetLastError();
}

}  // namespace sdd
