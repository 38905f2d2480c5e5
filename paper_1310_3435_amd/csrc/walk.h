// walk.h -- launch interface of the interface walk (walk.hip): arguments,
// the per-path record word and the workspace layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "sdd.h"

namespace sdd {

// Walk launch arguments.  Path tickets t = g * paths + (p - path_begin)
// enumerate every (node g, path p) pair; a persistent grid of waves draws
// them from a device counter.
struct WalkArgs {
    Density dens;
    Bmap bmap;
    const double* nodes;
    int64_t n_nodes;
    int64_t paths;       // N per node
    int64_t path_begin;  // counter word of the first path
    uint32_t total;      // n_nodes * paths (< 2^32)
    int32_t kmax;
    double dt;
    double sqrt2dt;
    double noise_f32;    // sqrt(2 dt) sqrt(2 ln 2): the float walk's normals come scaled
    int32_t bridge;      // 1: Brownian-bridge exit test after every step
    uint32_t key0, key1;
    void* pq;                     // [total] (P.x, P.y, Q.x, Q.y) of the last step, walk precision
    uint32_t* info;               // [total] exit step | side << 28 | bridged << 30 | capped << 31
    unsigned long long* counter;  // ticket counter, zeroed before the walk
    sdd_path_record* per_path;    // optional [total]
};

// Per-path info word written by the walk.
constexpr uint32_t kInfoSteps = 0x0fffffffu;
constexpr uint32_t kInfoBridged = 0x40000000u;
constexpr uint32_t kInfoCapped = 0x80000000u;
constexpr int kInfoSideShift = 28;
constexpr int64_t kMaxSteps = (int64_t)kInfoSteps;

// Workspace carving of sdd_interface_estimate.
struct WalkWorkspace {
    size_t pq_off, info_off, counter_off, node_tot_off, bytes;
};
WalkWorkspace walk_workspace(int64_t n_nodes, int64_t paths, int prec);

hipError_t launch_walk(const WalkArgs& A, int prec, double* mean, double* se, double* sums, sdd_walk_stats* stats,
                       long long* node_tot, hipStream_t stream);

}  // namespace sdd
