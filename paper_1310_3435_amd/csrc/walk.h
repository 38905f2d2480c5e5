// walk.h -- launch interface of the interface walk (walk_core.h, walk.hip,
// serve.hip): jobs, segments, the exact per-node sums and the exit queue.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "sdd.h"

namespace sdd {

// Paths of one node handed to a wave by one atomic: a pool never spans two
// nodes, so a ticket is (node, first path, count) decoded once per pool.
// Pools hold kPoolPaths paths, or up to four times as many on jobs large
// enough to keep every wave busy with them (fewer nodes per exit drain).
constexpr uint32_t kPoolPaths = 64;
constexpr uint32_t kMaxPoolPaths = 4 * kPoolPaths;

// Per-path info word carried from the walk to the exit processing.
constexpr uint32_t kInfoSteps = 0x0fffffffu;
constexpr uint32_t kInfoBridged = 0x40000000u;
constexpr uint32_t kInfoCapped = 0x80000000u;
constexpr int kInfoSideShift = 28;
constexpr int64_t kMaxSteps = (int64_t)kInfoSteps;

// Exit tests of a step (Sec. 2.2).  kExitLane: per lane, from its job
// (the request server mixes jobs with either test in one wave).
enum ExitKind { kExitStep = 0, kExitBridge = 1, kExitLane = 2, kExitExpo = 3 };

// Exact per-node sums.  A path's value v (x, y, x^2 or y^2 at its exit
// point) is rounded to the integer n = rint(v 2^F) with |n| <= 2^54 (F from a
// bound of the boundary map's image, the same for every path of a job); a
// wave adds the n of up to 64 paths of a node (|sum| <= 2^60) and adds the
// sum as two limbs, sum mod 2^31 and floor(sum / 2^31), into 64-bit integer
// sums: exact for up to 2^32 additions per node.  Integer addition is
// associative, so the sums do not depend on the order in which paths finish
// and the estimate is reproducible bit for bit under any schedule.
struct NodeAcc {
    unsigned long long lo[4];  // x, y, x^2, y^2: sums of the low limbs
    unsigned long long hi[4];  // sums of the high limbs (two's complement)
    unsigned long long steps;  // exit step counts
    unsigned long long capped; // paths stopped by the step cap
    uint32_t invalid;          // the node is not strictly inside the square
    uint32_t pad[3];
};

// Scale of a job's sums: s[0] = 2^F for x and y, s[1] = 2^F2 for squares.
struct AccScale {
    double s[2];
};

// One job: an estimate call or one served request.
struct WalkJob {
    const double* nodes;        // device [n][2]
    NodeAcc* acc;               // device [n]
    const AccScale* scale;      // device
    sdd_path_record* per_path;  // device [n][paths] or null (parity mode)
    uint64_t paths;             // paths per node of the job (per_path row length)
    Bmap bmap;
    GaussParams gp;             // float Gaussian-sum density (request server)
    float dt, noise, bridge_c;  // float step, sqrt(2 dt) sqrt(2 ln 2), -log2(e)/dt
    int32_t exit_test;          // sdd_exit_test
    uint32_t kblocks;           // step cap in three-step blocks
    uint32_t path0;             // counter word of the job's path 0
    uint32_t key0, key1;        // Philox key (seed)
    uint32_t n_nodes;
};

// A launch walks a table of segments.  Segment s covers paths
// [p_lo, p_hi) of every node of job `job`, in pools of pool_paths
// consecutive paths of one node: pools [pool_base, pool_base + n_nodes *
// chunks) of the launch, chunks = ceil((p_hi - p_lo) / pool_paths), pool
// j n_nodes + g holding chunk j of node g.
struct WalkSeg {
    uint64_t pool_base;
    const WalkJob* job;  // server: device copy of the job; unused by an estimate call
    uint32_t n_nodes;
    uint32_t chunks;
    uint32_t p_lo, p_hi;
};

// Launch arguments of the walk kernel.  An estimate call has one job and
// one segment, both passed here (wave-uniform: they land in scalar
// registers, as do the density terms); the request server passes tables in
// device memory and per-lane parameters.
struct WalkArgs {
    Density dens;
    WalkJob job;                // estimate: the job
    WalkSeg seg;                // estimate: its segment
    const WalkSeg* segs;        // server: device table, pool_base increasing
    int32_t nseg;
    int32_t kmax;               // step cap (multiple of 3)
    double dt;                  // step; with exponential stepping the mean step 1/lambda
    double sqrt2dt;
    double noise_f32;           // sqrt(2 dt) sqrt(2 ln 2): the float walk's normals come scaled
    uint64_t total_pools;
    uint32_t pool_paths;        // paths per pool: a multiple of 64, <= kMaxPoolPaths
    uint32_t pad;
    unsigned long long* counter;  // pool counter, zeroed before the walk
};

// Exit queue entry: the last step's ends P, Q in the walk precision, the
// info word, the node, the path and (server) the segment.
template <typename R>
struct ExitEntry {
    R px, py, qx, qy;
    uint32_t info, g, p, seg;
};

// Scale of the sums for values bounded by vmax in magnitude: the smallest
// e with 2^e >= vmax gives F = 54 - e (|v 2^F| <= 2^54) and F2 = 54 - 2e.
// A value is then rounded to 2^-54 of the bound, below a double's own
// rounding of values of that size.
__host__ __device__ inline AccScale scale_for_bound(double vmax)
{
    int e = 0;
    if (vmax > 0.0) (void)frexp(vmax, &e);  // vmax = f 2^e, 1/2 <= f < 1, so 2^e > vmax
    if (e < -200) e = -200;
    if (e > 200) e = 200;
    AccScale S;
    S.s[0] = ldexp(1.0, 54 - e);
    S.s[1] = ldexp(1.0, 54 - 2 * e);
    return S;
}

// Value of a limb pair: (signed) hi 2^31 + lo, both sums of integers, as
// the correctly rounded double.
__host__ __device__ inline double limb_value(unsigned long long lo, unsigned long long hi)
{
    const long long H = (long long)hi + (long long)(lo >> 31);
    const double hd = (double)H;
    const double herr = (double)(H - (long long)hd);  // exact: |H - hd| <= ulp(hd) / 2 <= 2^9
    const double b = (double)(lo & 0x7fffffffull);
    return hd * 0x1p31 + (herr * 0x1p31 + b);        // one rounding of the exact value
}

// Workspace of an estimate call: the pool counter, the scale and the start
// time of the walk (a 256-byte header), then one NodeAcc per node.
struct WalkWorkspace {
    size_t counter_off, scale_off, clock_off, acc_off, bytes;
};
WalkWorkspace walk_workspace(int64_t n_nodes);

// A bound of |x_b| and |y_b| over the boundary, known on the host for
// every map but TABLE (whose table the device bounds).
bool bmap_host_bound(const Bmap& B, double& vmax);

// Zero the node sums, set the scale (from hs, or for a TABLE map from its
// table), zero the pool counter and record the start time (clock0, if not
// null).
hipError_t launch_acc_init(NodeAcc* acc, int64_t n, AccScale* scale, const Bmap& B, bool host_scale,
                           const AccScale& hs, unsigned long long* counter, unsigned long long* clock0,
                           hipStream_t stream);

// Zero a pool counter (a kernel, so that the call may be captured in a graph).
hipError_t launch_reset_counter(unsigned long long* counter, hipStream_t stream);

// Walk of an estimate call (A.job, A.seg, A.dens) after launch_acc_init.
hipError_t launch_walk(const WalkArgs& A, int prec, int exit_kind, hipStream_t stream);

// Node means, standard errors and raw sums from the node sums; stats totals
// and the walk time (wall clock from clock0, rate in kHz) if stats.
hipError_t launch_finalize(const NodeAcc* acc, const AccScale* scale, int64_t n, double paths, double* mean,
                           double* se, double* sums, sdd_walk_stats* stats, const unsigned long long* clock0,
                           double wall_rate_khz, hipStream_t stream);

// Request server: one walk launch over A.segs (float, Gaussian sums,
// per-lane parameters) on `blocks` blocks of kWalkBlock threads.
constexpr int kWalkBlock = 256;
hipError_t launch_serve_walk(const WalkArgs& A, int blocks, hipStream_t stream);
int serve_walk_occupancy();

}  // namespace sdd
