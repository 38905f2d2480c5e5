// kernels.h -- launch interface between the C ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "sdd.h"
#include "walk.h"

namespace sdd {

// mesh.hip
hipError_t launch_layout_nodes(const sdd_layout& L, int k, int placement, const Density& D, double* nodes,
                               hipStream_t stream);
hipError_t launch_edge1d_table(const Density& D, int n, double* table, hipStream_t stream);
hipError_t launch_layout_extrema(const sdd_layout& L, int cap, const Density& D, double* nodes, int32_t* counts,
                                 hipStream_t stream);
hipError_t launch_fill(const sdd_layout& L, int k, const int32_t* counts, const Bmap& B, const double* nodes,
                       const double* values, int interp, double* vert, double* horiz, hipStream_t stream);
hipError_t launch_subdomain_solve(const Density& D, const Bmap& B, const sdd_layout& L, const double* vert,
                                  const double* horiz, double tol, int max_sweeps, double* mesh, int32_t* sweeps,
                                  double* resid, void* workspace, hipStream_t stream);
size_t subdomain_workspace_bytes(const sdd_layout& L);
hipError_t launch_grid_nodes(int nx, int ny, double* nodes, hipStream_t stream);
hipError_t launch_assemble(int nx, int ny, const Bmap& B, const double* values, double* mesh, hipStream_t stream);

// postprocess.hip
size_t post_workspace_bytes();
hipError_t launch_quality(int nx, int ny, const double* mesh, double* q, double* out, void* ws, hipStream_t stream);
hipError_t launch_compare(int nx, int ny, const Density& D, const double* mesh, const double* ref, double* out,
                          void* ws, hipStream_t stream);
hipError_t launch_smooth(const sdd_layout& L, int per_subdomain, double dt, double k, int steps, double* mesh,
                         void* ws, hipStream_t stream);
hipError_t launch_smooth_interfaces(const sdd_layout& L, int span, double* vert, double* horiz, void* ws,
                                    hipStream_t stream);
size_t smooth_interfaces_workspace_bytes(const sdd_layout& L);

}  // namespace sdd
