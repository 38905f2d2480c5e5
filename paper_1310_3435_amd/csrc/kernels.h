// kernels.h -- launch interface between the C ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "sdd.h"

namespace sdd {

// Per-item partial sums written by the walk: sum x, sum y, sum x^2, sum y^2,
// step total and capped count of one (node, chunk) work item.
struct Slot {
    double s[4];
    long long steps;
    long long capped;
};

struct WalkArgs {
    Density dens;
    Bmap bmap;
    const double* nodes;
    int64_t n_nodes;
    int64_t paths;       // N per node
    int64_t path_begin;  // counter word of the first path
    int64_t chunk;       // paths per work item
    int64_t n_chunks;    // work items per node
    int64_t n_items;     // n_nodes * n_chunks
    double dt;
    double sqrt2dt;
    int32_t kmax;
    uint32_t key0, key1;
    Slot* slots;
    sdd_path_record* per_path;
};

// Paths per work item for a given problem size; fixed by (n_nodes, paths)
// alone so that results do not depend on the device.
int64_t walk_chunk(int64_t n_nodes, int64_t paths);

hipError_t launch_walk(const WalkArgs& A, int prec, double* mean, double* se, double* sums, sdd_walk_stats* stats,
                       long long* node_tot, hipStream_t stream);

// mesh.hip
hipError_t launch_layout_nodes(const sdd_layout& L, int k, int placement, const Density& D, double* nodes,
                               hipStream_t stream);
hipError_t launch_edge1d_table(const Density& D, int n, double* table, hipStream_t stream);
hipError_t launch_fill(const sdd_layout& L, int k, const Bmap& B, const double* nodes, const double* values,
                       int interp, double* vert, double* horiz, hipStream_t stream);
hipError_t launch_subdomain_solve(const Density& D, const Bmap& B, const sdd_layout& L, const double* vert,
                                  const double* horiz, double tol, int max_sweeps, double* mesh, int32_t* sweeps,
                                  double* resid, void* workspace, hipStream_t stream);
size_t subdomain_workspace_bytes(const sdd_layout& L);

}  // namespace sdd
