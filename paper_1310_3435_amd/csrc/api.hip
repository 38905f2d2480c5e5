// api.hip -- the extern "C" entry points declared in include/sdd.h.
//
// Host-side validation, workspace carving and kernel launches; every step of
// the path itself runs in the kernels of walk.hip and mesh.hip.
#include <math.h>
#include <string.h>

#include <new>

#include "common.h"
#include "host.h"
#include "kernels.h"
#include "sdd.h"


using namespace sdd;

namespace sdd {

// Scratch of sdd_interface_estimate_noalloc: the walk workspace (a 256-byte
// header and the node sums) for up to kNoAllocMaxNodes nodes, in a
// file-scope device array that every GPU the library runs on holds until
// the process ends.  Host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (sdd_ctx::scratch).
constexpr int64_t kNoAllocMaxNodes = (int64_t)1 << 16;
constexpr size_t kNoAllocBytes = 256 + (size_t)kNoAllocMaxNodes * sizeof(NodeAcc);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

WalkWorkspace walk_workspace(int64_t n_nodes)
{
    WalkWorkspace W;
    W.counter_off = 0;
    W.scale_off = 64;
    W.clock_off = 128;
    W.acc_off = 256;
    W.bytes = align_up(W.acc_off + (size_t)n_nodes * sizeof(NodeAcc), 256);
    return W;
}

}  // namespace sdd

extern "C" {

const char* sdd_status_string(int status)
{
    switch (status) {
    case SDD_OK: return "ok";
    case SDD_WARN_CAPPED: return "some paths stopped at the step cap";
    case SDD_EINVAL: return "invalid argument";
    case SDD_ENOSPC: return "workspace too small";
    case SDD_EDEVICE: return "HIP runtime error";
    case SDD_EAGAIN: return "not finished yet";
    case SDD_ECANCELED: return "cancelled";
    case SDD_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

int32_t sdd_version(void) { return 200; }

sdd_status sdd_create(int32_t device, sdd_ctx** out)
{
    if (!out) return SDD_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return SDD_EDEVICE;
    if (device < 0 || device >= count) return SDD_EINVAL;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return SDD_EDEVICE;
    sdd_ctx* c = new (std::nothrow) sdd_ctx;
    if (!c) return SDD_EDEVICE;
    c->device = device;
    c->cu_count = prop.multiProcessorCount;
    int rate = 0;
    if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, device) != hipSuccess) rate = 0;
    c->wall_rate_khz = rate;
    // this device's address of the static scratch array, with the device
    // current (each GPU holds its own copy)
    int prev = 0;
    c->scratch = nullptr;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess ||
        hipGetSymbolAddress(&c->scratch, HIP_SYMBOL(scratch)) != hipSuccess || !c->scratch) {
        (void)hipSetDevice(prev);
        delete c;
        return SDD_EDEVICE;
    }
    (void)hipSetDevice(prev);
    *out = c;
    return SDD_OK;
}

void sdd_destroy(sdd_ctx* ctx) { delete ctx; }

size_t sdd_workspace_bytes(int64_t n_nodes, int64_t paths_per_node, int32_t prec)
{
    (void)prec;
    if (n_nodes < 1 || n_nodes > kMaxNodes || paths_per_node < 1 || paths_per_node > kMaxPathsPerNode) return 0;
    return walk_workspace(n_nodes).bytes;
}

namespace {

// Validation shared by sdd_interface_estimate and its allocation-free
// variant; fills A (without the workspace pointers) and the step cap.
sdd_status prepare_estimate(const sdd_density* w, const sdd_bmap* bmap, const double* nodes, int64_t n_nodes,
                            int64_t paths_per_node, int64_t path_begin, double dt, uint64_t seed, int32_t prec,
                            double t_max, int32_t exit_test, const double* mean, int cu_count, WalkArgs& A)
{
    if (!nodes || !mean) return SDD_EINVAL;
    sdd_status s = check_density(w);
    if (s != SDD_OK) return s;
    if ((s = check_bmap(bmap)) != SDD_OK) return s;
    if (n_nodes < 1 || n_nodes > kMaxNodes) return SDD_EINVAL;
    if (paths_per_node < 1 || paths_per_node > kMaxPathsPerNode || path_begin < 0) return SDD_EINVAL;
    if (path_begin + paths_per_node > ((int64_t)1 << 32)) return SDD_EINVAL;
    if (!(dt > 0.0) || !(dt < 1.0)) return SDD_EINVAL;
    if (prec != SDD_FP32 && prec != SDD_FP64) return SDD_EINVAL;
    if (exit_test != SDD_EXIT_END_OF_STEP && exit_test != SDD_EXIT_BRIDGE && exit_test != SDD_EXIT_EXPONENTIAL)
        return SDD_EINVAL;
    if (!(t_max > 0.0)) t_max = 8.0;
    if (!is_finite(t_max)) return SDD_EINVAL;
    const int32_t kmax = step_cap(t_max, dt);
    if (kmax < 0) return SDD_EINVAL;

    memset(&A, 0, sizeof(A));
    A.dens = to_device(w);
    WalkJob& J = A.job;
    J.nodes = nodes;
    J.paths = (uint64_t)paths_per_node;
    J.bmap = to_device(bmap);
    J.gp = gauss_params(A.dens);
    J.dt = (float)dt;
    J.noise = (float)noise_f32(dt);
    J.bridge_c = (float)(-1.4426950408889634 / dt);
    J.exit_test = exit_test;
    J.kblocks = (uint32_t)(kmax / 3);
    J.path0 = (uint32_t)path_begin;
    J.key0 = (uint32_t)seed;
    J.key1 = (uint32_t)(seed >> 32);
    J.n_nodes = (uint32_t)n_nodes;
    A.pool_paths = pool_paths_for(n_nodes * paths_per_node, cu_count);
    const uint32_t chunks = (uint32_t)((paths_per_node + A.pool_paths - 1) / A.pool_paths);
    A.seg.pool_base = 0;
    A.seg.job = nullptr;
    A.seg.n_nodes = (uint32_t)n_nodes;
    A.seg.chunks = chunks;
    A.seg.p_lo = 0;
    A.seg.p_hi = (uint32_t)paths_per_node;
    A.total_pools = (uint64_t)n_nodes * chunks;
    A.kmax = kmax;
    A.dt = dt;
    A.sqrt2dt = sqrt(2.0 * dt);
    A.noise_f32 = noise_f32(dt);
    return SDD_OK;
}

// Enqueue set-up, walk and finalize of a prepared estimate whose workspace
// starts at ws.
sdd_status run_estimate(sdd_ctx* ctx, WalkArgs& A, char* ws, int32_t prec, int32_t exit_test, double* mean,
                        double* se, double* sums, sdd_walk_stats* stats, sdd_path_record* per_path,
                        hipStream_t stream)
{
    const int64_t n = A.job.n_nodes;
    const WalkWorkspace W = walk_workspace(n);
    A.counter = (unsigned long long*)(ws + W.counter_off);
    A.job.acc = (NodeAcc*)(ws + W.acc_off);
    A.job.scale = (const AccScale*)(ws + W.scale_off);
    A.job.per_path = per_path;
    unsigned long long* clock0 = (unsigned long long*)(ws + W.clock_off);
    double vmax = 0.0;
    const bool host_scale = bmap_host_bound(A.job.bmap, vmax);
    const AccScale hs = scale_for_bound(vmax);
    hipError_t e = launch_acc_init(A.job.acc, n, (AccScale*)(ws + W.scale_off), A.job.bmap, host_scale, hs,
                                   A.counter, clock0, stream);
    const int kind = exit_test == SDD_EXIT_BRIDGE ? kExitBridge
                     : exit_test == SDD_EXIT_EXPONENTIAL ? kExitExpo : kExitStep;
    if (e == hipSuccess) e = launch_walk(A, prec, kind, stream);
    if (e == hipSuccess)
        e = launch_finalize(A.job.acc, A.job.scale, n, (double)A.job.paths, mean, se, sums, stats, clock0,
                            (double)ctx->wall_rate_khz, stream);
    return from_hip(e);
}

}  // namespace

sdd_status sdd_interface_estimate(sdd_ctx* ctx, const sdd_density* w, const sdd_bmap* bmap, const double* nodes,
                                  int64_t n_nodes, int64_t paths_per_node, int64_t path_begin, double dt,
                                  uint64_t seed, int32_t prec, double t_max, int32_t exit_test, double* mean,
                                  double* se, double* sums,
                                  sdd_walk_stats* stats, sdd_path_record* per_path, void* workspace, size_t ws_bytes,
                                  void* stream)
{
    if (!ctx || !workspace) return SDD_EINVAL;
    WalkArgs A;
    sdd_status s = prepare_estimate(w, bmap, nodes, n_nodes, paths_per_node, path_begin, dt, seed, prec, t_max,
                                    exit_test, mean, ctx->cu_count, A);
    if (s != SDD_OK) return s;
    if (ws_bytes < walk_workspace(n_nodes).bytes) return SDD_ENOSPC;
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    return run_estimate(ctx, A, (char*)workspace, prec, exit_test, mean, se, sums, stats, per_path,
                        (hipStream_t)stream);
}

sdd_status sdd_interface_estimate_noalloc(sdd_ctx* ctx, const sdd_density* w, const sdd_bmap* bmap,
                                          const double* nodes, int64_t n_nodes, int64_t paths_per_node,
                                          int64_t path_begin, double dt, uint64_t seed, int32_t prec, double t_max,
                                          int32_t exit_test, double* mean, double* se, double* sums,
                                          sdd_walk_stats* stats, sdd_path_record* per_path, void* stream)
{
    if (!ctx || !ctx->scratch) return SDD_EINVAL;
    WalkArgs A;
    sdd_status s = prepare_estimate(w, bmap, nodes, n_nodes, paths_per_node, path_begin, dt, seed, prec, t_max,
                                    exit_test, mean, ctx->cu_count, A);
    if (s != SDD_OK) return s;
    if (n_nodes > kNoAllocMaxNodes || walk_workspace(n_nodes).bytes > kNoAllocBytes) return SDD_ENOSPC;
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    // the header (pool counter, scale, start time) and the node sums are
    // set by the first kernel of the call, so nothing of an earlier call
    // carries over
    return run_estimate(ctx, A, (char*)ctx->scratch, prec, exit_test, mean, se, sums, stats, per_path,
                        (hipStream_t)stream);
}

int64_t sdd_noalloc_max_nodes(void) { return kNoAllocMaxNodes; }

sdd_status sdd_walk_status(const sdd_walk_stats* stats)
{
    if (!stats) return SDD_EINVAL;
    return stats->capped > 0 ? SDD_WARN_CAPPED : SDD_OK;
}

int64_t sdd_layout_node_count(const sdd_layout* L, int32_t k)
{
    if (check_layout(L) != SDD_OK || k < 0) return -1;
    return (int64_t)(L->sx - 1) * (L->sy - 1) + (int64_t)k * ((int64_t)(L->sx - 1) * L->sy + (int64_t)(L->sy - 1) * L->sx);
}

sdd_status sdd_layout_nodes(sdd_ctx* ctx, const sdd_layout* L, int32_t k, int32_t placement, const sdd_density* w,
                            double* nodes, void* stream)
{
    if (!ctx || !nodes) return SDD_EINVAL;
    sdd_status s = check_layout(L);
    if (s != SDD_OK) return s;
    if (k < 0 || placement < 0 || placement > 1) return SDD_EINVAL;
    if (placement == 1 && (s = check_density(w)) != SDD_OK) return s;
    if (sdd_layout_node_count(L, k) == 0) return SDD_OK;
    Density D;
    memset(&D, 0, sizeof(D));
    if (w) D = to_device(w);
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    return from_hip(launch_layout_nodes(*L, k, placement, D, nodes, (hipStream_t)stream));
}

sdd_status sdd_bmap_edge1d_table(sdd_ctx* ctx, const sdd_density* w, int32_t n_per_edge, double* table, void* stream)
{
    if (!ctx || !table || n_per_edge < 3) return SDD_EINVAL;
    sdd_status s = check_density(w);
    if (s != SDD_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    return from_hip(launch_edge1d_table(to_device(w), n_per_edge, table, (hipStream_t)stream));
}

sdd_status sdd_fill_interfaces(sdd_ctx* ctx, const sdd_layout* L, int32_t k, const sdd_bmap* bmap,
                               const double* nodes, const double* values, int32_t interp, double* vert,
                               double* horiz, void* stream)
{
    if (!ctx) return SDD_EINVAL;
    sdd_status s = check_layout(L);
    if (s != SDD_OK) return s;
    if ((s = check_bmap(bmap)) != SDD_OK) return s;
    if (k < 0 || interp < 0 || interp > 1) return SDD_EINVAL;
    if (L->sx > 1 && !vert) return SDD_EINVAL;
    if (L->sy > 1 && !horiz) return SDD_EINVAL;
    if (sdd_layout_node_count(L, k) > 0 && (!nodes || !values)) return SDD_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    return from_hip(
        launch_fill(*L, k, nullptr, to_device(bmap), nodes, values, interp, vert, horiz, (hipStream_t)stream));
}

sdd_status sdd_layout_nodes_extrema(sdd_ctx* ctx, const sdd_layout* L, const sdd_density* w, int32_t cap,
                                    double* nodes, int32_t* counts, void* stream)
{
    if (!ctx || !nodes || !counts || cap < 0) return SDD_EINVAL;
    sdd_status s = check_layout(L);
    if (s != SDD_OK) return s;
    if ((s = check_density(w)) != SDD_OK) return s;
    if (sdd_layout_node_count(L, cap) == 0) return SDD_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    return from_hip(launch_layout_extrema(*L, cap, to_device(w), nodes, counts, (hipStream_t)stream));
}

sdd_status sdd_fill_interfaces_counts(sdd_ctx* ctx, const sdd_layout* L, int32_t cap, const int32_t* counts,
                                      const sdd_bmap* bmap, const double* nodes, const double* values,
                                      int32_t interp, double* vert, double* horiz, void* stream)
{
    if (!ctx || !counts) return SDD_EINVAL;
    sdd_status s = check_layout(L);
    if (s != SDD_OK) return s;
    if ((s = check_bmap(bmap)) != SDD_OK) return s;
    if (cap < 0 || interp < 0 || interp > 1) return SDD_EINVAL;
    if (L->sx > 1 && !vert) return SDD_EINVAL;
    if (L->sy > 1 && !horiz) return SDD_EINVAL;
    if (sdd_layout_node_count(L, cap) > 0 && (!nodes || !values)) return SDD_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    return from_hip(
        launch_fill(*L, cap, counts, to_device(bmap), nodes, values, interp, vert, horiz, (hipStream_t)stream));
}

size_t sdd_subdomain_workspace_bytes(const sdd_layout* L)
{
    if (check_layout(L) != SDD_OK) return 0;
    return subdomain_workspace_bytes(*L);
}

sdd_status sdd_subdomain_solve(sdd_ctx* ctx, const sdd_density* w, const sdd_bmap* bmap, const sdd_layout* L,
                               const double* vert, const double* horiz, double tol, int32_t max_sweeps,
                               double* mesh, int32_t* sweeps, double* resid, void* workspace, size_t ws_bytes,
                               void* stream)
{
    if (!ctx || !mesh || !workspace) return SDD_EINVAL;
    sdd_status s = check_density(w);
    if (s != SDD_OK) return s;
    if ((s = check_bmap(bmap)) != SDD_OK) return s;
    if ((s = check_layout(L)) != SDD_OK) return s;
    if (L->sx > 1 && !vert) return SDD_EINVAL;
    if (L->sy > 1 && !horiz) return SDD_EINVAL;
    if (ws_bytes < subdomain_workspace_bytes(*L)) return SDD_ENOSPC;
    if (!(tol > 0.0)) tol = 1e-13;
    if (max_sweeps <= 0) max_sweeps = 100000;
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    return from_hip(launch_subdomain_solve(to_device(w), to_device(bmap), *L, vert, horiz, tol, max_sweeps, mesh,
                                           sweeps, resid, workspace, (hipStream_t)stream));
}

// ---------------------------------------------------- whole-grid node set

sdd_status sdd_grid_nodes(sdd_ctx* ctx, int32_t nx, int32_t ny, double* nodes, void* stream)
{
    if (!ctx || nx < 3 || ny < 3 || !nodes) return SDD_EINVAL;
    if ((int64_t)nx * ny > ((int64_t)1 << 31)) return SDD_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    return from_hip(launch_grid_nodes(nx, ny, nodes, (hipStream_t)stream));
}

sdd_status sdd_assemble_mesh(sdd_ctx* ctx, int32_t nx, int32_t ny, const sdd_bmap* bmap, const double* values,
                             double* mesh, void* stream)
{
    if (!ctx || nx < 3 || ny < 3 || !values || !mesh) return SDD_EINVAL;
    if ((int64_t)nx * ny > ((int64_t)1 << 31)) return SDD_EINVAL;
    sdd_status s = check_bmap(bmap);
    if (s != SDD_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    return from_hip(launch_assemble(nx, ny, to_device(bmap), values, mesh, (hipStream_t)stream));
}

// ------------------------------------------------------ quality, smoothing

size_t sdd_quality_workspace_bytes(int32_t nx, int32_t ny)
{
    if (nx < 2 || ny < 2) return 0;
    return post_workspace_bytes();
}

sdd_status sdd_mesh_quality(sdd_ctx* ctx, int32_t nx, int32_t ny, const double* mesh, double* q, double* out,
                            void* workspace, size_t ws_bytes, void* stream)
{
    if (!ctx || !mesh || !out || !workspace || nx < 2 || ny < 2) return SDD_EINVAL;
    if ((int64_t)nx * ny > ((int64_t)1 << 31)) return SDD_EINVAL;
    if (ws_bytes < post_workspace_bytes()) return SDD_ENOSPC;
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    return from_hip(launch_quality(nx, ny, mesh, q, out, workspace, (hipStream_t)stream));
}

sdd_status sdd_mesh_compare(sdd_ctx* ctx, int32_t nx, int32_t ny, const sdd_density* w, const double* mesh,
                            const double* ref, double* out, void* workspace, size_t ws_bytes, void* stream)
{
    if (!ctx || !mesh || !ref || !out || !workspace || nx < 2 || ny < 2) return SDD_EINVAL;
    if ((int64_t)nx * ny > ((int64_t)1 << 31)) return SDD_EINVAL;
    sdd_status s = check_density(w);
    if (s != SDD_OK) return s;
    if (ws_bytes < post_workspace_bytes()) return SDD_ENOSPC;
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    return from_hip(launch_compare(nx, ny, to_device(w), mesh, ref, out, workspace, (hipStream_t)stream));
}

size_t sdd_smooth_workspace_bytes(const sdd_layout* L)
{
    if (check_layout(L) != SDD_OK) return 0;
    return (size_t)L->nx * L->ny * 2 * sizeof(double);
}

sdd_status sdd_mesh_smooth(sdd_ctx* ctx, const sdd_layout* L, int32_t per_subdomain, double dt, double k,
                           int32_t steps, double* mesh, void* workspace, size_t ws_bytes, void* stream)
{
    if (!ctx || !mesh || !workspace) return SDD_EINVAL;
    sdd_status s = check_layout(L);
    if (s != SDD_OK) return s;
    if (per_subdomain < 0 || per_subdomain > 2) return SDD_EINVAL;
    if (!(dt > 0.0) || !(k > 0.0) || !is_finite(k) || steps < 0) return SDD_EINVAL;
    const double hx2 = (double)(L->nx - 1) * (L->nx - 1), hy2 = (double)(L->ny - 1) * (L->ny - 1);
    if (!(dt * (2.0 * hx2 + 2.0 * hy2) <= 1.0)) return SDD_EINVAL;  // FTCS stability
    if (ws_bytes < sdd_smooth_workspace_bytes(L)) return SDD_ENOSPC;
    if (steps == 0) return SDD_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    return from_hip(launch_smooth(*L, per_subdomain, dt, k, steps, mesh, workspace, (hipStream_t)stream));
}

size_t sdd_smooth_interfaces_workspace_bytes(const sdd_layout* L)
{
    if (check_layout(L) != SDD_OK) return 0;
    return smooth_interfaces_workspace_bytes(*L);
}

sdd_status sdd_smooth_interfaces(sdd_ctx* ctx, const sdd_layout* L, int32_t span, double* vert, double* horiz,
                                 void* workspace, size_t ws_bytes, void* stream)
{
    if (!ctx || !workspace) return SDD_EINVAL;
    sdd_status s = check_layout(L);
    if (s != SDD_OK) return s;
    if (span < 5 || (span & 1) == 0) return SDD_EINVAL;
    if (L->sx > 1 && (!vert || span > L->ny)) return SDD_EINVAL;
    if (L->sy > 1 && (!horiz || span > L->nx)) return SDD_EINVAL;
    if (ws_bytes < smooth_interfaces_workspace_bytes(*L)) return SDD_ENOSPC;
    if (hipSetDevice(ctx->device) != hipSuccess) return SDD_EDEVICE;
    return from_hip(launch_smooth_interfaces(*L, span, vert, horiz, workspace, (hipStream_t)stream));
}

}  // extern "C"
