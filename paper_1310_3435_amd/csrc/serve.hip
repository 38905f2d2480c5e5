// serve.hip -- continuous batching of mesh requests (sdd_server_*).
//
// Every walk launch is one persistent grid of the interface walk
// (walk_core.h) over a table of segments, each a run of whole 1024-path
// blocks of one admitted request; lanes load their request's parameters
// when they start a path, so one wave may mix requests.  A request's paths
// add into its own exact per-node sums, which do not depend on the order
// in which paths finish, and a path's random numbers depend only on its
// counters: a request's result is bitwise the same alone, in any mix, and
// as an sdd_interface_estimate call with the same inputs.
// A scheduler thread admits requests (first come, first served, while a
// slot and arena memory are free), keeps up to two walk launches in
// flight on two streams (a launch's last, longest paths overlap the next
// launch), runs the pilot -> paths decision, and finishes each request with
// the interface fill, the subdomain solves and a copy of its mesh to the
// caller (Sec. 2.1: estimate on the interfaces, then independent subdomain
// solves; Sec. 2.2: Euler-Maruyama walks averaged over pseudo-random paths).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "common.h"
#include "host.h"
#include "kernels.h"
#include "rng.h"
#include "sdd.h"

namespace sdd {

constexpr uint32_t kBlockPaths = 1024;  // paths per node in a scheduling block
constexpr int kMaxSegments = 256;
constexpr int kServeReservedCUs = 0;  // CUs the walk launches leave free (see sdd_server_create)

// ------------------------------------------------------------------ host

static double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over the device arena (offsets; no device calls).
class Arena {
public:
    void init(size_t bytes) { free_[0] = bytes; }
    bool alloc(size_t bytes, size_t& off)
    {
        bytes = align_up(bytes, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes, 256);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;
};

enum State { QUEUED, PILOT, MAIN, FINISHING, DONE };

struct Request {
    uint64_t id = 0;
    sdd_request spec;
    double* user_mesh = nullptr;
    State state = QUEUED;
    bool cancelled = false;
    sdd_status status = SDD_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int64_t n_nodes = 0, points = 0;
    int slot = -1;
    size_t arena_off = 0, arena_bytes = 0;
    AccScale scale_h;  // the scale of its sums (host copy)
    // device pieces (inside the arena)
    WalkJob* djob = nullptr;
    AccScale* scale = nullptr;
    double* nodes = nullptr;
    NodeAcc* acc = nullptr;
    double* mean = nullptr;
    double* se = nullptr;
    double* vert = nullptr;
    double* horiz = nullptr;
    double* mesh = nullptr;
    void* fd_ws = nullptr;
    // blocks: total (known after the pilot), scheduled, walked
    uint32_t nb_total = 1, nb_sched = 0, nb_done = 0;
    bool pilot_copy = false;  // sums copied to pinned after the pilot
    hipEvent_t ev_pilot = nullptr, ev_done = nullptr;
    hipEvent_t ev_fin[3] = { nullptr, nullptr, nullptr };  // finish: start, fill done, solves done (timed)
    double walk_t0 = -1.0, walk_t1 = -1.0;               // device times of its first and last walk launch (ms)
    int64_t paths = 0, steps = 0, capped = 0;
    double max_se = 0;
    float t_fill_ms = 0, t_sub_ms = 0;
};

struct Launch {
    hipEvent_t ev_start = nullptr, ev = nullptr;        // walk start and end (timed)
    std::vector<std::pair<Request*, uint32_t>> blocks;  // request, blocks in this launch
    bool busy = false;
};

}  // namespace sdd

using namespace sdd;

struct sdd_server {
    sdd_ctx* ctx = nullptr;
    int device = 0;
    int max_slots = 0;
    int64_t max_nodes = 0, max_points = 0, launch_paths = 0;
    size_t budget = 0;
    char* arena_base = nullptr;
    Arena arena;
    // two walk launches in flight, each with its own segment table and counter
    hipStream_t walk_stream[2] = { nullptr, nullptr };
    hipStream_t finish_stream = nullptr;
    hipStream_t setup_stream = nullptr;  // admissions: staging copy + nodes
    WalkSeg* dsegs[2] = { nullptr, nullptr };
    WalkSeg* hsegs[2] = { nullptr, nullptr };  // pinned
    unsigned long long* counter[2] = { nullptr, nullptr };
    hipEvent_t ev_ref = nullptr;  // time origin of the device times
    Launch launches[2];
    int next_launch = 0;
    // pinned staging per slot
    char* pinned = nullptr;
    size_t slot_stride = 0;
    std::vector<int> free_slots;
    // requests
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<uint64_t, Request*> all;
    std::deque<Request*> queued;
    std::vector<Request*> active;  // admitted, in admission order
    uint64_t next_id = 1;
    bool stopping = false;
    std::thread worker;
    int walk_blocks = 0;
    uint32_t pool_paths = kPoolPaths;  // divides kBlockPaths
};

namespace {

// Staging of a slot: the job (admission), then the node sums, the node SEs
// and the mesh (results).
size_t stage_acc_off() { return align_up(sizeof(WalkJob), 256); }
size_t stage_se_off(const sdd_server* S) { return stage_acc_off() + align_up((size_t)S->max_nodes * sizeof(NodeAcc), 256); }
size_t stage_mesh_off(const sdd_server* S)
{
    return stage_se_off(S) + align_up((size_t)S->max_nodes * 2 * sizeof(double), 256);
}
char* stage(sdd_server* S, const Request* r) { return S->pinned + (size_t)r->slot * S->slot_stride; }

size_t request_bytes(const sdd_request& q, int64_t n_nodes)
{
    const sdd_layout& L = q.layout;
    size_t b = 0;
    b += align_up(sizeof(WalkJob), 256) + align_up(sizeof(AccScale), 256);
    b += align_up((size_t)n_nodes * 2 * sizeof(double), 256) * 3;  // nodes, mean, se
    b += align_up((size_t)n_nodes * sizeof(NodeAcc), 256);
    b += align_up((size_t)(L.sx - 1) * L.ny * 2 * sizeof(double), 256);
    b += align_up((size_t)(L.sy - 1) * L.nx * 2 * sizeof(double), 256);
    b += align_up((size_t)L.nx * L.ny * 2 * sizeof(double), 256);
    b += align_up(subdomain_workspace_bytes(L), 256);
    return b;
}

sdd_status check_request(const sdd_server* S, const sdd_request* q, int64_t& n_nodes)
{
    if (!q) return SDD_EINVAL;
    sdd_status s = check_density(&q->w);
    if (s != SDD_OK) return s;
    if ((s = check_bmap(&q->bmap)) != SDD_OK) return s;
    if ((s = check_layout(&q->layout)) != SDD_OK) return s;
    for (int t = 0; t < q->w.n_terms; ++t)
        if (q->w.term[t].kind != SDD_TERM_GAUSS) return SDD_EUNSUPPORTED;
    if (q->bmap.kind == SDD_BMAP_TABLE) return SDD_EUNSUPPORTED;
    if (q->k < 0 || q->placement < 0 || q->placement > 1 || q->interp < 0 || q->interp > 1) return SDD_EINVAL;
    if (!(q->dt > 0.0) || !(q->dt < 1.0)) return SDD_EINVAL;
    if (!(q->se_target > 0.0) && q->paths_per_node < 2) return SDD_EINVAL;
    if (q->paths_per_node > ((int64_t)1 << 30)) return SDD_EINVAL;
    const double tmax = q->t_max > 0.0 ? q->t_max : 8.0;
    if (!is_finite(tmax) || step_cap(tmax, q->dt) < 0) return SDD_EINVAL;
    if (q->exit_test == SDD_EXIT_EXPONENTIAL) return SDD_EUNSUPPORTED;
    if (q->exit_test != SDD_EXIT_END_OF_STEP && q->exit_test != SDD_EXIT_BRIDGE) return SDD_EINVAL;
    const sdd_layout& L = q->layout;
    n_nodes = (int64_t)(L.sx - 1) * (L.sy - 1) + (int64_t)q->k * ((int64_t)(L.sx - 1) * L.sy + (int64_t)(L.sy - 1) * L.sx);
    if (n_nodes < 1 || n_nodes > S->max_nodes) return SDD_EINVAL;
    if ((int64_t)L.nx * L.ny > S->max_points) return SDD_EINVAL;
    if ((int64_t)n_nodes * kBlockPaths > S->launch_paths) return SDD_EINVAL;  // one block must fit a launch
    if (request_bytes(*q, n_nodes) > S->budget) return SDD_EINVAL;
    return SDD_OK;
}

// The request's job: exactly the parameters sdd_interface_estimate derives
// from the same inputs (float walk, path 0 at counter 0).
void fill_job(const Request* r, WalkJob& J)
{
    const sdd_request& q = r->spec;
    memset(&J, 0, sizeof(J));
    const Density D = to_device(&q.w);
    J.nodes = r->nodes;
    J.acc = r->acc;
    J.scale = r->scale;
    J.per_path = nullptr;
    J.paths = 0;
    J.bmap = to_device(&q.bmap);
    J.gp = gauss_params(D);
    J.dt = (float)q.dt;
    J.noise = (float)noise_f32(q.dt);
    J.bridge_c = (float)(-1.4426950408889634 / q.dt);
    J.exit_test = q.exit_test;
    J.kblocks = (uint32_t)(step_cap(q.t_max > 0.0 ? q.t_max : 8.0, q.dt) / 3);
    J.path0 = 0;
    J.key0 = (uint32_t)q.seed;
    J.key1 = (uint32_t)(q.seed >> 32);
    J.n_nodes = (uint32_t)r->n_nodes;
}

// Admit queued requests while a slot and arena memory are free (FIFO).
void admit(sdd_server* S, std::unique_lock<std::mutex>& lk)
{
    while (!S->queued.empty() && !S->free_slots.empty()) {
        Request* r = S->queued.front();
        size_t off = 0;
        if (!S->arena.alloc(r->arena_bytes, off)) break;
        S->queued.pop_front();
        r->slot = S->free_slots.back();
        S->free_slots.pop_back();
        r->arena_off = off;
        if (r->spec.se_target > 0.0) {
            r->state = PILOT;  // one block first: its spread decides the paths
        } else {
            // the paths are given: every block is a main block
            r->nb_total = (uint32_t)((r->spec.paths_per_node + kBlockPaths - 1) / kBlockPaths);
            r->state = MAIN;
        }
        r->t_admit = now_s();
        S->active.push_back(r);
        lk.unlock();
        // carve the arena
        char* p = S->arena_base + off;
        auto take = [&](size_t b) {
            char* q = p;
            p += align_up(b, 256);
            return q;
        };
        const sdd_layout& L = r->spec.layout;
        r->djob = (WalkJob*)take(sizeof(WalkJob));
        r->scale = (AccScale*)take(sizeof(AccScale));
        r->nodes = (double*)take((size_t)r->n_nodes * 2 * sizeof(double));
        r->mean = (double*)take((size_t)r->n_nodes * 2 * sizeof(double));
        r->se = (double*)take((size_t)r->n_nodes * 2 * sizeof(double));
        r->acc = (NodeAcc*)take((size_t)r->n_nodes * sizeof(NodeAcc));
        r->vert = (double*)take((size_t)(L.sx - 1) * L.ny * 2 * sizeof(double));
        r->horiz = (double*)take((size_t)(L.sy - 1) * L.nx * 2 * sizeof(double));
        r->mesh = (double*)take((size_t)L.nx * L.ny * 2 * sizeof(double));
        r->fd_ws = (void*)take(subdomain_workspace_bytes(L));
        hipStream_t st = S->setup_stream;
        // the job goes through the slot's pinned staging
        WalkJob* hjob = (WalkJob*)stage(S, r);
        fill_job(r, *hjob);
        double vmax = 1.0;
        (void)bmap_host_bound(hjob->bmap, vmax);  // no TABLE maps here
        r->scale_h = scale_for_bound(vmax);
        hipError_t e = hipMemcpyAsync(r->djob, hjob, sizeof(WalkJob), hipMemcpyHostToDevice, st);
        const Density D = to_device(&r->spec.w);
        if (e == hipSuccess) e = launch_layout_nodes(L, r->spec.k, r->spec.placement, D, r->nodes, st);
        if (e == hipSuccess)
            e = launch_acc_init(r->acc, r->n_nodes, r->scale, hjob->bmap, true, r->scale_h, nullptr, nullptr, st);
        // the staging copy must finish before the slot's staging is reused
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        lk.lock();
        if (e != hipSuccess) {
            r->status = SDD_EDEVICE;
            r->cancelled = true;
        }
    }
}

// Build and enqueue one walk launch from the admitted requests' unscheduled
// blocks (admission order), up to launch_paths paths.
bool launch(sdd_server* S, std::unique_lock<std::mutex>& lk)
{
    Launch& Lh = S->launches[S->next_launch];
    if (Lh.busy) return false;
    const int li = S->next_launch;
    WalkSeg* hs = S->hsegs[li];
    int nseg = 0;
    uint64_t paths = 0, pools = 0;
    Lh.blocks.clear();
    for (Request* r : S->active) {
        if (nseg == kMaxSegments) break;
        if (r->cancelled || (r->state != PILOT && r->state != MAIN)) continue;
        if (r->nb_sched >= r->nb_total) continue;
        const uint64_t per_block = (uint64_t)r->n_nodes * kBlockPaths;
        const uint64_t room = (uint64_t)S->launch_paths - paths;
        const uint32_t nb = (uint32_t)std::min<uint64_t>(room / per_block, r->nb_total - r->nb_sched);
        if (nb == 0) continue;
        WalkSeg& G = hs[nseg++];
        G.pool_base = pools;
        G.job = r->djob;
        G.n_nodes = (uint32_t)r->n_nodes;
        G.chunks = nb * (kBlockPaths / S->pool_paths);
        G.p_lo = r->nb_sched * kBlockPaths;
        G.p_hi = (r->nb_sched + nb) * kBlockPaths;
        paths += per_block * nb;
        pools += (uint64_t)G.n_nodes * G.chunks;
        r->nb_sched += nb;
        Lh.blocks.push_back({ r, nb });
    }
    if (nseg == 0) return false;
    Lh.busy = true;
    S->next_launch ^= 1;
    lk.unlock();
    hipStream_t st = S->walk_stream[li];
    hipError_t e = hipMemcpyAsync(S->dsegs[li], hs, nseg * sizeof(WalkSeg), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_reset_counter(S->counter[li], st);
    if (e == hipSuccess) e = hipEventRecord(Lh.ev_start, st);
    if (e == hipSuccess) {
        WalkArgs A;
        memset(&A, 0, sizeof(A));
        A.segs = S->dsegs[li];
        A.nseg = nseg;
        A.total_pools = pools;
        A.pool_paths = S->pool_paths;
        A.counter = S->counter[li];
        const int64_t most = ((int64_t)paths + kWalkBlock - 1) / kWalkBlock;
        const int blocks = (int)std::min<int64_t>(S->walk_blocks, most);
        e = launch_serve_walk(A, blocks, st);
    }
    if (e == hipSuccess) e = hipEventRecord(Lh.ev, st);
    lk.lock();
    if (e != hipSuccess) {
        for (auto& b : Lh.blocks) {
            b.first->status = SDD_EDEVICE;
            b.first->cancelled = true;
        }
    }
    return true;
}

// Sample mean and variance of one value from the host copy of node sums
// over n paths.
void node_moments(const NodeAcc& a, const AccScale& sc, int q, double n, double& mean, double& var)
{
    const double s1 = limb_value(a.lo[q], a.hi[q]) / sc.s[0];
    const double s2 = limb_value(a.lo[q + 2], a.hi[q + 2]) / sc.s[1];
    mean = s1 / n;
    var = fmax(s2 - n * mean * mean, 0.0) / (n - 1.0);
}

// The pilot's sums are on the host: choose the request's paths per node.
void decide_paths(sdd_server* S, Request* r)
{
    const NodeAcc* a = (const NodeAcc*)(stage(S, r) + stage_acc_off());
    const double n = kBlockPaths;
    double smax = 0.0;
    for (int64_t g = 0; g < r->n_nodes; ++g) {
        for (int q = 0; q < 2; ++q) {
            double m, v;
            node_moments(a[g], r->scale_h, q, n, m, v);
            smax = fmax(smax, sqrt(v));
        }
    }
    const double want = ceil((smax / r->spec.se_target) * (smax / r->spec.se_target));
    double nb = ceil(fmax(want, n) / n);
    const double cap = (double)(1u << 20);  // at most 2^30 paths per node
    if (!(nb >= 1.0)) nb = 1.0;
    if (nb > cap) nb = cap;
    r->nb_total = (uint32_t)nb;
}

// Called once every block of the request has been walked: the launches
// that held them have retired, so the sums are final and the finish stream
// waits for nothing.
void finish(sdd_server* S, Request* r)
{
    hipStream_t st = S->finish_stream;
    const sdd_request& q = r->spec;
    const double paths = (double)r->nb_total * kBlockPaths;
    hipError_t e = hipEventRecord(r->ev_fin[0], st);
    if (e == hipSuccess)
        e = launch_finalize(r->acc, r->scale, r->n_nodes, paths, r->mean, r->se, nullptr, nullptr, nullptr, 0.0, st);
    const Bmap B = to_device(&q.bmap);
    if (e == hipSuccess) e = launch_fill(q.layout, q.k, nullptr, B, r->nodes, r->mean, q.interp, r->vert, r->horiz, st);
    if (e == hipSuccess) e = hipEventRecord(r->ev_fin[1], st);
    if (e == hipSuccess)
        e = launch_subdomain_solve(to_device(&q.w), B, q.layout, r->vert, r->horiz, 1e-13, 100000, r->mesh, nullptr,
                                   nullptr, r->fd_ws, st);
    if (e == hipSuccess) e = hipEventRecord(r->ev_fin[2], st);
    char* stg = stage(S, r);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stg + stage_acc_off(), r->acc, (size_t)r->n_nodes * sizeof(NodeAcc), hipMemcpyDeviceToHost,
                           st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stg + stage_se_off(S), r->se, (size_t)r->n_nodes * 2 * sizeof(double), hipMemcpyDeviceToHost,
                           st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stg + stage_mesh_off(S), r->mesh, (size_t)q.layout.nx * q.layout.ny * 2 * sizeof(double),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(r->ev_done, st);
    if (e != hipSuccess) r->status = SDD_EDEVICE;
}

void complete(sdd_server* S, Request* r)
{
    // called with the lock held, after ev_done
    if (r->status == SDD_OK && !r->cancelled) {
        char* stg = stage(S, r);
        const NodeAcc* a = (const NodeAcc*)(stg + stage_acc_off());
        const double* se = (const double*)(stg + stage_se_off(S));
        const double* mesh = (const double*)(stg + stage_mesh_off(S));
        long long steps = 0, capped = 0;
        double mse = 0.0;
        for (int64_t g = 0; g < r->n_nodes; ++g) {
            steps += (long long)a[g].steps;
            capped += (long long)a[g].capped;
            mse = fmax(mse, fmax(se[2 * g], se[2 * g + 1]));
        }
        r->steps = steps;
        r->capped = capped;
        r->max_se = mse;
        r->paths = (int64_t)r->nb_total * kBlockPaths;
        if (hipEventElapsedTime(&r->t_fill_ms, r->ev_fin[0], r->ev_fin[1]) != hipSuccess) r->t_fill_ms = 0;
        if (hipEventElapsedTime(&r->t_sub_ms, r->ev_fin[1], r->ev_fin[2]) != hipSuccess) r->t_sub_ms = 0;
        memcpy(r->user_mesh, mesh, (size_t)r->spec.layout.nx * r->spec.layout.ny * 2 * sizeof(double));
        if (capped > 0) r->status = SDD_WARN_CAPPED;
    } else if (r->status == SDD_OK) {
        r->status = SDD_ECANCELED;
    }
    r->t_done = now_s();
    r->state = DONE;
    S->arena.release(r->arena_off, r->arena_bytes);
    S->free_slots.push_back(r->slot);
    S->active.erase(std::find(S->active.begin(), S->active.end(), r));
    S->cv_done.notify_all();
}

void worker_loop(sdd_server* S)
{
    if (hipSetDevice(S->device) != hipSuccess) return;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        if (S->stopping && S->queued.empty() && S->active.empty() && !S->launches[0].busy && !S->launches[1].busy)
            break;
        bool progress = false;
        admit(S, lk);
        // retire finished launches
        for (int i = 0; i < 2; ++i) {
            Launch& Lh = S->launches[i];
            if (!Lh.busy) continue;
            lk.unlock();
            const bool done = hipEventQuery(Lh.ev) == hipSuccess;
            float t0 = -1.0f, t1 = -1.0f;
            if (done && (hipEventElapsedTime(&t0, S->ev_ref, Lh.ev_start) != hipSuccess ||
                         hipEventElapsedTime(&t1, S->ev_ref, Lh.ev) != hipSuccess))
                t0 = t1 = -1.0f;
            lk.lock();
            if (!done) continue;
            for (auto& b : Lh.blocks) {
                Request* r = b.first;
                r->nb_done += b.second;
                if (t0 >= 0.0f) {
                    if (r->walk_t0 < 0.0 || t0 < r->walk_t0) r->walk_t0 = t0;
                    if (t1 > r->walk_t1) r->walk_t1 = t1;
                }
            }
            Lh.blocks.clear();
            Lh.busy = false;
            progress = true;
        }
        // pilots (requests with an SE target): copy the sums to the host,
        // then decide the paths (the pilot block's launch has retired, so
        // its sums are final)
        for (Request* r : std::vector<Request*>(S->active)) {
            if (r->state == PILOT && !r->cancelled && r->nb_done >= 1 && !r->pilot_copy) {
                char* stg = stage(S, r) + stage_acc_off();
                lk.unlock();
                hipError_t e = hipMemcpyAsync(stg, r->acc, (size_t)r->n_nodes * sizeof(NodeAcc),
                                              hipMemcpyDeviceToHost, S->finish_stream);
                if (e == hipSuccess) e = hipEventRecord(r->ev_pilot, S->finish_stream);
                lk.lock();
                if (e != hipSuccess) {
                    r->status = SDD_EDEVICE;
                    r->cancelled = true;
                }
                r->pilot_copy = true;
                progress = true;
            }
            if (r->state == PILOT && r->pilot_copy && !r->cancelled) {
                lk.unlock();
                const bool ready = hipEventQuery(r->ev_pilot) == hipSuccess;
                lk.lock();
                if (!ready) continue;
                decide_paths(S, r);
                r->state = MAIN;
                progress = true;
            }
        }
        // requests whose blocks have all been walked: finish them
        for (Request* r : std::vector<Request*>(S->active)) {
            const bool walked = r->nb_done >= r->nb_sched;
            if ((r->state == MAIN && r->nb_done >= r->nb_total) || (r->cancelled && r->state != FINISHING && walked)) {
                if (!r->cancelled) {
                    lk.unlock();
                    finish(S, r);
                    lk.lock();
                } else {
                    // every scheduled block has retired: nothing of the
                    // request's is in flight, and its memory can go back
                    lk.unlock();
                    (void)hipEventRecord(r->ev_done, S->finish_stream);
                    lk.lock();
                }
                r->state = FINISHING;
                progress = true;
            }
        }
        for (Request* r : std::vector<Request*>(S->active)) {
            if (r->state != FINISHING) continue;
            lk.unlock();
            const bool ready = hipEventQuery(r->ev_done) == hipSuccess;
            lk.lock();
            if (ready) {
                complete(S, r);
                progress = true;
            }
        }
        // keep two walk launches in flight
        while (launch(S, lk)) progress = true;
        if (!progress) S->cv_work.wait_for(lk, std::chrono::microseconds(200));
    }
}

void destroy_request_events(Request* r)
{
    (void)hipEventDestroy(r->ev_pilot);
    (void)hipEventDestroy(r->ev_done);
    for (int i = 0; i < 3; ++i)
        if (r->ev_fin[i]) (void)hipEventDestroy(r->ev_fin[i]);
}

}  // namespace

extern "C" {

sdd_status sdd_server_create(sdd_ctx* ctx, size_t hbm_budget_bytes, int32_t max_slots, int64_t max_nodes,
                             int64_t max_points, int64_t launch_paths, sdd_server** out)
{
    if (!ctx || !out) return SDD_EINVAL;
    *out = nullptr;
    if (max_slots < 1 || max_slots > 256 || max_nodes < 1 || max_points < 9 || hbm_budget_bytes < 4096)
        return SDD_EINVAL;
    if (launch_paths <= 0) launch_paths = (int64_t)1 << 25;
    if (launch_paths < kBlockPaths || launch_paths > ((int64_t)1 << 40)) return SDD_EINVAL;
    sdd_server* S = new (std::nothrow) sdd_server;
    if (!S) return SDD_EDEVICE;
    S->ctx = ctx;
    const int dev = ctx->device;
    S->device = dev;
    if (hipSetDevice(dev) != hipSuccess) {
        delete S;
        return SDD_EDEVICE;
    }
    S->max_slots = max_slots;
    S->max_nodes = max_nodes;
    S->max_points = max_points;
    S->launch_paths = launch_paths;
    S->budget = hbm_budget_bytes;
    bool ok = hipMalloc((void**)&S->arena_base, hbm_budget_bytes) == hipSuccess;
    if (ok) S->arena.init(hbm_budget_bytes);
    int cus = 0;
    ok = ok && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0;
    // CUs the walk streams leave to the finish stream (SDD_SERVE_RESERVED_CUS
    // overrides): walk launches otherwise hold every CU, and a subdomain
    // solve block, which needs a CU's worth of free wave slots, waits for a
    // launch to end.
    int reserve = kServeReservedCUs;
    if (const char* env = getenv("SDD_SERVE_RESERVED_CUS")) reserve = atoi(env);
    if (reserve < 0 || reserve >= cus) reserve = 0;
    for (int i = 0; i < 2 && ok; ++i) {
        ok = hipMalloc((void**)&S->dsegs[i], kMaxSegments * sizeof(WalkSeg)) == hipSuccess &&
             hipMalloc((void**)&S->counter[i], 256) == hipSuccess &&
             hipHostMalloc((void**)&S->hsegs[i], kMaxSegments * sizeof(WalkSeg), hipHostMallocDefault) == hipSuccess &&
             hipEventCreate(&S->launches[i].ev_start) == hipSuccess &&
             hipEventCreate(&S->launches[i].ev) == hipSuccess;
        if (ok && reserve > 0) {
            std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0u);
            for (int c = reserve; c < cus; ++c) mask[(size_t)c / 32] |= 1u << (c % 32);
            ok = hipExtStreamCreateWithCUMask(&S->walk_stream[i], (uint32_t)mask.size(), mask.data()) == hipSuccess;
        } else if (ok) {
            ok = hipStreamCreateWithFlags(&S->walk_stream[i], hipStreamNonBlocking) == hipSuccess;
        }
    }
    ok = ok && hipStreamCreateWithFlags(&S->finish_stream, hipStreamNonBlocking) == hipSuccess &&
         hipStreamCreateWithFlags(&S->setup_stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreate(&S->ev_ref) == hipSuccess && hipEventRecord(S->ev_ref, S->setup_stream) == hipSuccess &&
         hipEventSynchronize(S->ev_ref) == hipSuccess;
    S->slot_stride = align_up(sizeof(WalkJob), 256) + align_up((size_t)max_nodes * sizeof(NodeAcc), 256) +
                     align_up((size_t)max_nodes * 2 * sizeof(double), 256) +
                     align_up((size_t)max_points * 2 * sizeof(double), 256);
    ok = ok && hipHostMalloc((void**)&S->pinned, S->slot_stride * max_slots, hipHostMallocDefault) == hipSuccess;
    const int occ = ok ? serve_walk_occupancy() : 0;
    ok = ok && occ > 0;
    if (!ok) {
        sdd_server_destroy(S);
        return SDD_EDEVICE;
    }
    // Waves per SIMD of each walk launch (blocks of 4 waves per CU;
    // SDD_SERVE_WAVES_PER_SIMD overrides).  Two launches are in flight, and
    // the finish stream's subdomain solves need wave slots beside them:
    // measured same-box, 3 waves give 3% more capacity and 4-7% lower p50
    // and p99 than 4 (which fill every SIMD with the two walks); 2 lose
    // capacity.
    int want = 3;
    if (const char* env = getenv("SDD_SERVE_WAVES_PER_SIMD"))
        if (atoi(env) > 0) want = atoi(env);
    S->walk_blocks = std::max(1, std::min(occ, want)) * (cus - reserve);
    S->pool_paths = pool_paths_for(launch_paths, cus);
    for (int i = max_slots - 1; i >= 0; --i) S->free_slots.push_back(i);
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return SDD_OK;
}

sdd_status sdd_server_submit(sdd_server* S, const sdd_request* req, double* mesh, uint64_t* id)
{
    if (!S || !req || !mesh || !id) return SDD_EINVAL;
    int64_t n_nodes = 0;
    sdd_status s = check_request(S, req, n_nodes);
    if (s != SDD_OK) return s;
    Request* r = new (std::nothrow) Request;
    if (!r) return SDD_EDEVICE;
    r->spec = *req;
    r->user_mesh = mesh;
    r->n_nodes = n_nodes;
    r->points = (int64_t)req->layout.nx * req->layout.ny;
    r->arena_bytes = request_bytes(*req, n_nodes);
    if (hipEventCreateWithFlags(&r->ev_pilot, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&r->ev_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&r->ev_fin[0]) != hipSuccess || hipEventCreate(&r->ev_fin[1]) != hipSuccess ||
        hipEventCreate(&r->ev_fin[2]) != hipSuccess) {
        destroy_request_events(r);
        delete r;
        return SDD_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) {
        destroy_request_events(r);
        delete r;
        return SDD_ECANCELED;
    }
    r->id = S->next_id++;
    r->t_submit = now_s();
    S->all[r->id] = r;
    S->queued.push_back(r);
    *id = r->id;
    S->cv_work.notify_all();
    return SDD_OK;
}

static sdd_status take_result(sdd_server* S, std::map<uint64_t, Request*>::iterator it, sdd_result* out)
{
    Request* r = it->second;
    if (out) {
        memset(out, 0, sizeof(*out));
        out->status = r->status;
        out->n_nodes = r->n_nodes;
        out->paths_per_node = r->paths;
        out->steps = r->steps;
        out->max_se = r->max_se;
        out->t_submit = r->t_submit;
        out->t_admit = r->t_admit;
        out->t_done = r->t_done;
        out->capped = r->capped;
        out->t_queue_ms = r->t_admit > 0.0 ? (r->t_admit - r->t_submit) * 1e3 : 0.0;
        out->t_stoc_ms = r->walk_t1 >= r->walk_t0 && r->walk_t0 >= 0.0 ? r->walk_t1 - r->walk_t0 : 0.0;
        out->t_fill_ms = r->t_fill_ms;
        out->t_sub_ms = r->t_sub_ms;
    }
    const sdd_status st = r->status;
    S->all.erase(it);
    destroy_request_events(r);
    delete r;
    return st;
}

sdd_status sdd_server_poll(sdd_server* S, uint64_t id, sdd_result* out)
{
    if (!S) return SDD_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(id);
    if (it == S->all.end()) return SDD_EINVAL;
    if (it->second->state != DONE) return SDD_EAGAIN;
    return take_result(S, it, out);
}

sdd_status sdd_server_wait(sdd_server* S, uint64_t id, sdd_result* out)
{
    if (!S) return SDD_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        auto it = S->all.find(id);
        if (it == S->all.end()) return SDD_EINVAL;
        if (it->second->state == DONE) return take_result(S, it, out);
        S->cv_done.wait(lk);
    }
}

sdd_status sdd_server_cancel(sdd_server* S, uint64_t id)
{
    if (!S) return SDD_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(id);
    if (it == S->all.end()) return SDD_EINVAL;
    Request* r = it->second;
    if (r->state == DONE) return SDD_OK;
    if (r->state == QUEUED) {
        S->queued.erase(std::find(S->queued.begin(), S->queued.end(), r));
        r->status = SDD_ECANCELED;
        r->t_done = now_s();
        r->state = DONE;
        S->cv_done.notify_all();
        return SDD_OK;
    }
    r->cancelled = true;
    if (r->status == SDD_OK) r->status = SDD_ECANCELED;
    S->cv_work.notify_all();
    return SDD_OK;
}

double sdd_server_clock(sdd_server* S)
{
    (void)S;
    return now_s();
}

sdd_status sdd_server_destroy(sdd_server* S)
{
    if (!S) return SDD_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
        for (Request* r : S->queued) {
            r->status = SDD_ECANCELED;
            r->state = DONE;
        }
        S->queued.clear();
        for (Request* r : S->active) {
            r->cancelled = true;
            if (r->status == SDD_OK) r->status = SDD_ECANCELED;
        }
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    for (auto& kv : S->all) {
        destroy_request_events(kv.second);
        delete kv.second;
    }
    for (int i = 0; i < 2; ++i) {
        if (S->walk_stream[i]) (void)hipStreamSynchronize(S->walk_stream[i]);
    }
    if (S->finish_stream) (void)hipStreamSynchronize(S->finish_stream);
    if (S->setup_stream) (void)hipStreamSynchronize(S->setup_stream);
    for (int i = 0; i < 2; ++i) {
        if (S->dsegs[i]) (void)hipFree(S->dsegs[i]);
        if (S->counter[i]) (void)hipFree(S->counter[i]);
        if (S->hsegs[i]) (void)hipHostFree(S->hsegs[i]);
        if (S->walk_stream[i]) (void)hipStreamDestroy(S->walk_stream[i]);
        if (S->launches[i].ev) (void)hipEventDestroy(S->launches[i].ev);
        if (S->launches[i].ev_start) (void)hipEventDestroy(S->launches[i].ev_start);
    }
    if (S->finish_stream) (void)hipStreamDestroy(S->finish_stream);
    if (S->setup_stream) (void)hipStreamDestroy(S->setup_stream);
    if (S->ev_ref) (void)hipEventDestroy(S->ev_ref);
    if (S->pinned) (void)hipHostFree(S->pinned);
    if (S->arena_base) (void)hipFree(S->arena_base);
    delete S;
    return SDD_OK;
}

}  // extern "C"
