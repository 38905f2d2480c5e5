// serve.hip -- continuous batching of mesh requests (sdd_server_*).
//
// Every walk launch is a persistent grid over a table of segments, each a
// run of whole 1024-path blocks of one admitted request; lanes carry their
// request's parameters in registers, so one wave may mix requests.  Block b
// of a request is reduced into that request's compensated per-node sums
// before block b+1, in a fixed order, so results do not depend on the mix.
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

constexpr uint32_t kBlockPaths = 1024;  // paths per node in a block
constexpr int kServeTerms = SDD_MAX_TERMS;
constexpr int kMaxSegments = 256;
constexpr int kServeBlock = 256;

// Device copy of one request's walk parameters.
struct ServeReq {
    float fbase;
    int32_t n_terms;
    float cx[kServeTerms], cy[kServeTerms], k2[kServeTerms], la[kServeTerms], m2c[kServeTerms];
    float dt, noise;
    float bridge_c;   // -log2(e)/dt
    int32_t bridge;   // 1: Brownian-bridge exit test
    int32_t kmax;
    uint32_t key0, key1;
    uint32_t n_nodes;
    const double* nodes;
    Bmap bmap;
};

// Compensated per-node sums of one request.
struct NodeAcc {
    double s[4], c[4];
    long long steps, capped;
};

// One launch segment: blocks [b0, b0 + nb) of one request.
struct ServeSeg {
    uint32_t ticket_base;  // first ticket of the segment in the launch
    uint32_t node_base;    // first reduce block of the segment in the launch
    uint32_t n_nodes;
    uint32_t b0, nb;
    uint32_t pad;
    uint64_t rec_base;  // record index of the segment's first ticket
    const ServeReq* req;
    NodeAcc* acc;
};

// ------------------------------------------------------------------ kernels

__device__ __forceinline__ int find_segment(const ServeSeg* segs, int nseg, uint32_t t)
{
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (segs[mid].ticket_base <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// Float walk with per-lane request parameters; Gaussian-sum drift.
__global__ __launch_bounds__(256) void serve_walk_kernel(const ServeSeg* __restrict__ segs, int nseg, uint32_t total,
                                                         unsigned long long* __restrict__ counter,
                                                         float4* __restrict__ pq, uint32_t* __restrict__ info)
{
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t pool_lo = 0, pool_hi = 0;
    bool exhausted = false;
    bool live = false;
    uint64_t rec = 0;
    uint32_t g = 0, pc = 0;
    float X = 0, Y = 0;
    uint32_t m = 0;  // Philox block index: steps 3m .. 3m+2
    // the lane's request
    float fbase = 1, dt = 0, sd = 0, bc = 0;
    int32_t nterm = 0;
    uint32_t mmax = 0;  // step cap in blocks
    bool bridge = false;
    uint32_t key0 = 0, key1 = 0;
    float cx[kServeTerms], cy[kServeTerms], k2[kServeTerms], la[kServeTerms], m2c[kServeTerms];
#pragma unroll
    for (int q = 0; q < kServeTerms; ++q) cx[q] = cy[q] = k2[q] = la[q] = m2c[q] = 0.0f;

    for (;;) {
        uint64_t need = __ballot(!live);
        while (need != 0 && !exhausted) {
            if (pool_lo == pool_hi) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(counter, 64ull);
                base = __shfl(base, 0, kWave);
                if (base >= total) {
                    exhausted = true;
                    break;
                }
                pool_lo = (uint32_t)base;
                pool_hi = (uint32_t)min((unsigned long long)total, base + 64ull);
            }
            const uint32_t avail = pool_hi - pool_lo;
            const uint32_t want = (uint32_t)__popcll(need);
            const uint32_t take = want < avail ? want : avail;
            const uint32_t rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
            if (!live && rank < take) {
                const uint32_t t = pool_lo + rank;
                const ServeSeg& S = segs[find_segment(segs, nseg, t)];
                const uint32_t local = t - S.ticket_base;
                const uint32_t per_block = S.n_nodes * kBlockPaths;
                const uint32_t blk = local / per_block;
                const uint32_t rem = local - blk * per_block;
                g = rem / kBlockPaths;
                pc = (S.b0 + blk) * kBlockPaths + (rem - g * kBlockPaths);
                rec = S.rec_base + local;
                const ServeReq* R = S.req;
                fbase = R->fbase;
                nterm = R->n_terms;
#pragma unroll
                for (int q = 0; q < kServeTerms; ++q) {
                    cx[q] = R->cx[q];
                    cy[q] = R->cy[q];
                    k2[q] = R->k2[q];
                    la[q] = R->la[q];
                    m2c[q] = R->m2c[q];
                }
                dt = R->dt;
                sd = R->noise;
                bc = R->bridge_c;
                bridge = R->bridge != 0;
                mmax = (uint32_t)(R->kmax / 3);
                key0 = R->key0;
                key1 = R->key1;
                X = (float)R->nodes[2 * (size_t)g];
                Y = (float)R->nodes[2 * (size_t)g + 1];
                m = 0;
                live = true;
            }
            pool_lo += take;
            need = __ballot(!live);
        }
        if (__ballot(live) == 0) break;

        const uint4 r = philox(m, pc, g, 0u, key0, key1);
        // one Euler-Maruyama step of the lane's Gaussian-sum density
        auto em = [&](float x, float y, float z0, float z1, float& xn, float& yn) {
            float W = fbase, Gx = 0.0f, Gy = 0.0f;
#pragma unroll
            for (int q = 0; q < kServeTerms; ++q) {
                if (q < nterm) {
                    const float dx = x - cx[q], dy = y - cy[q];
                    const float e = __builtin_amdgcn_exp2f(__builtin_fmaf(k2[q], __builtin_fmaf(dx, dx, dy * dy), la[q]));
                    W += e;
                    const float h = m2c[q] * e;
                    Gx = __builtin_fmaf(h, dx, Gx);
                    Gy = __builtin_fmaf(h, dy, Gy);
                }
            }
            const float iw = __builtin_amdgcn_rcpf(W);
            xn = fmar(sd, z0, fmar(Gx * iw, dt, x));
            yn = fmar(sd, z1, fmar(Gy * iw, dt, y));
        };
        float z0, z1, XA, YA, XB, YB, XC, YC;
        normals(field_hi(r.x, 0.0f), field_hi(r.y, 0.0f), z0, z1);
        em(X, Y, z0, z1, XA, YA);
        normals(field_hi(r.z, 0.0f), field_hi(r.w, 0.0f), z0, z1);
        em(XA, YA, z0, z1, XB, YB);
        normals(field_lo(r.x, r.y, 0.0f), field_lo(r.z, r.w, 0.0f), z0, z1);
        em(XB, YB, z0, z1, XC, YC);

        const bool outA = outside(XA, YA);
        const bool outB = outside(XB, YB);
        const bool outC = outside(XC, YC);
        bool exA = outA, exB = outB, exC = outC;
        if (__ballot(live && bridge) != 0) {
            // some lane's request asks for the bridge test (wave-uniform branch)
            const float PA = bridge_prob(X, Y, XA, YA, bc);
            const float PB = bridge_prob(XA, YA, XB, YB, bc);
            const float PC = bridge_prob(XB, YB, XC, YC, bc);
            const bool may = (!outA && bridge_may_exit(PA)) || (!outB && bridge_may_exit(PB)) ||
                             (!outC && bridge_may_exit(PC));
            if (__ballot(live && bridge && may) != 0) {
                const uint4 q = philox(m, pc, g, 1u, key0, key1);
                exA = outA || (bridge && uniform23(q.x, 0.0f) < PA);
                exB = outB || (bridge && uniform23(q.y, 0.0f) < PB);
                exC = outC || (bridge && uniform23(q.z, 0.0f) < PC);
            }
        }
        const bool fin = live && (exA || exB || exC || (m + 1u >= mmax));
        if (fin) {
            const float px = exA ? X : (exB ? XA : XB), py = exA ? Y : (exB ? YA : YB);
            const float qx = exA ? XA : (exB ? XB : XC), qy = exA ? YA : (exB ? YB : YC);
            pq[rec] = make_float4(px, py, qx, qy);
            uint32_t w = 3u * m + (exA ? 1u : (exB ? 2u : 3u));
            if (!(exA || exB || exC))
                w |= kInfoCapped;
            else if (!(exA ? outA : (exB ? outB : outC)))
                w |= kInfoBridged | (bridge_side(px, py, qx, qy) << kInfoSideShift);
            info[rec] = w;
            live = false;
        }
        X = XC;
        Y = YC;
        ++m;
    }
}

// One block per (segment, node): the node's blocks in order; each block's
// 1024 paths projected in double, mapped, summed in a fixed order, then
// added into the node's compensated sums.
__global__ __launch_bounds__(kServeBlock) void serve_reduce_kernel(const ServeSeg* __restrict__ segs, int nseg,
                                                                   const float4* __restrict__ pq,
                                                                   const uint32_t* __restrict__ info)
{
    __shared__ double part[4][kServeBlock / kWave];
    __shared__ long long ipart[2][kServeBlock / kWave];
    int s = 0;
    {
        int lo = 0, hi = nseg;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (segs[mid].node_base <= blockIdx.x) lo = mid; else hi = mid;
        }
        s = lo;
    }
    const ServeSeg& S = segs[s];
    const uint32_t g = blockIdx.x - S.node_base;
    const Bmap B = S.req->bmap;
    NodeAcc* acc = S.acc + g;
    for (uint32_t blk = 0; blk < S.nb; ++blk) {
        const uint64_t base = S.rec_base + ((uint64_t)blk * S.n_nodes + g) * kBlockPaths;
        double sm[4] = { 0, 0, 0, 0 }, cm[4] = { 0, 0, 0, 0 };
        long long st = 0, cp = 0;
        for (uint32_t j = threadIdx.x; j < kBlockPaths; j += kServeBlock) {
            const float4 v = pq[base + j];
            const uint32_t w = info[base + j];
            double ex, ey;
            const bool capped = (w & kInfoCapped) != 0;
            int side;
            if (w & kInfoBridged) {
                side = (int)((w >> kInfoSideShift) & 3u);
                ex = side == 0 ? 0.0 : side == 1 ? 1.0 : (double)v.z;
                ey = side == 2 ? 0.0 : side == 3 ? 1.0 : (double)v.w;
            } else {
                side = capped ? nearest_side(v.z, v.w, ex, ey) : exit_point(v.x, v.y, v.z, v.w, ex, ey);
            }
            double x, y;
            bmap_eval(B, side, ex, ey, x, y);
            nadd(sm[0], cm[0], x);
            nadd(sm[1], cm[1], y);
            nadd(sm[2], cm[2], x * x);
            nadd(sm[3], cm[3], y * y);
            st += w & kInfoSteps;
            cp += capped ? 1 : 0;
        }
        double tot[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) tot[q] = sm[q] + cm[q];
#pragma unroll
        for (int m = kWave / 2; m >= 1; m >>= 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) tot[q] += __shfl_xor(tot[q], m, kWave);
            st += __shfl_xor(st, m, kWave);
            cp += __shfl_xor(cp, m, kWave);
        }
        const int wv = threadIdx.x / kWave;
        if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) part[q][wv] = tot[q];
            ipart[0][wv] = st;
            ipart[1][wv] = cp;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 0; q < 4; ++q) {
                double b = 0.0;
                for (int i = 0; i < kServeBlock / kWave; ++i) b += part[q][i];
                nadd(acc->s[q], acc->c[q], b);
            }
            for (int i = 0; i < kServeBlock / kWave; ++i) {
                acc->steps += ipart[0][i];
                acc->capped += ipart[1][i];
            }
        }
        __syncthreads();
    }
}

__global__ void serve_zero_kernel(NodeAcc* acc, uint32_t n)
{
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    for (int q = 0; q < 4; ++q) acc[g].s[q] = acc[g].c[q] = 0.0;
    acc[g].steps = 0;
    acc[g].capped = 0;
}

// Node means and standard errors of a finished request.
__global__ void serve_finalize_kernel(const NodeAcc* __restrict__ acc, uint32_t n, double paths,
                                      double* __restrict__ mean, double* __restrict__ se)
{
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    double t[4];
    for (int q = 0; q < 4; ++q) t[q] = acc[g].s[q] + acc[g].c[q];
    const double mx = t[0] / paths, my = t[1] / paths;
    mean[2 * g] = mx;
    mean[2 * g + 1] = my;
    se[2 * g] = sqrt(fmax(t[2] - paths * mx * mx, 0.0) / (paths * (paths - 1.0)));
    se[2 * g + 1] = sqrt(fmax(t[3] - paths * my * my, 0.0) / (paths * (paths - 1.0)));
}

__global__ void serve_counter_kernel(unsigned long long* c) { *c = 0ull; }

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
    // device pieces (inside the arena)
    ServeReq* dreq = nullptr;
    double* nodes = nullptr;
    NodeAcc* acc = nullptr;
    double* mean = nullptr;
    double* se = nullptr;
    double* vert = nullptr;
    double* horiz = nullptr;
    double* mesh = nullptr;
    void* fd_ws = nullptr;
    // blocks: total (known after the pilot), scheduled, reduced
    uint32_t nb_total = 1, nb_sched = 0, nb_done = 0;
    bool pilot_copy = false;  // acc copied to pinned after the pilot
    hipEvent_t ev_pilot = nullptr, ev_done = nullptr;
    int64_t paths = 0, steps = 0;
    double max_se = 0;
};

struct Launch {
    hipEvent_t ev = nullptr;                       // walk and reduce done
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
    // two walk launches in flight, each with its own records and segment table
    hipStream_t walk_stream[2] = { nullptr, nullptr };
    hipStream_t finish_stream = nullptr;
    hipStream_t setup_stream = nullptr;  // admissions: staging copy + nodes
    float4* pq[2] = { nullptr, nullptr };
    uint32_t* info[2] = { nullptr, nullptr };
    ServeSeg* dsegs[2] = { nullptr, nullptr };
    ServeSeg* hsegs[2] = { nullptr, nullptr };  // pinned
    unsigned long long* counter[2] = { nullptr, nullptr };
    hipEvent_t reduce_done = nullptr;  // last reduce issued (orders reduces across the two streams)
    bool have_reduce = false;
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
};

namespace {

size_t request_bytes(const sdd_request& q, int64_t n_nodes)
{
    const sdd_layout& L = q.layout;
    size_t b = 0;
    b += align_up(sizeof(ServeReq), 256);
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
    const double tmax = q->t_max > 0.0 ? q->t_max : 8.0;
    if (!is_finite(tmax) || ceil(tmax / q->dt) >= (double)(kMaxSteps - 2)) return SDD_EINVAL;
    if (q->exit_test != SDD_EXIT_END_OF_STEP && q->exit_test != SDD_EXIT_BRIDGE) return SDD_EINVAL;
    const sdd_layout& L = q->layout;
    n_nodes = (int64_t)(L.sx - 1) * (L.sy - 1) + (int64_t)q->k * ((int64_t)(L.sx - 1) * L.sy + (int64_t)(L.sy - 1) * L.sx);
    if (n_nodes < 1 || n_nodes > S->max_nodes) return SDD_EINVAL;
    if ((int64_t)L.nx * L.ny > S->max_points) return SDD_EINVAL;
    if ((int64_t)n_nodes * kBlockPaths > S->launch_paths) return SDD_EINVAL;  // one block must fit a launch
    if (request_bytes(*q, n_nodes) > S->budget) return SDD_EINVAL;
    return SDD_OK;
}

void fill_serve_req(const sdd_request& q, const double* nodes, uint32_t n_nodes, ServeReq& R)
{
    memset(&R, 0, sizeof(R));
    R.fbase = (float)q.w.base;
    R.n_terms = q.w.n_terms;
    for (int t = 0; t < q.w.n_terms; ++t) {
        const sdd_density_term& T = q.w.term[t];
        R.cx[t] = (float)T.cx;
        R.cy[t] = (float)T.cy;
        R.k2[t] = (float)(-T.coef * 1.4426950408889634073599246810019);
        R.la[t] = (float)log2(T.amp);
        R.m2c[t] = (float)(-2.0 * T.coef);
    }
    R.dt = (float)q.dt;
    R.noise = (float)(sqrt(2.0 * q.dt) * sqrt(2.0 * 0.69314718055994530942));
    R.bridge_c = (float)(-1.4426950408889634 / q.dt);
    R.bridge = q.exit_test == SDD_EXIT_BRIDGE ? 1 : 0;
    const double tmax = q.t_max > 0.0 ? q.t_max : 8.0;
    double kd = ceil(tmax / q.dt);
    kd += fmod(3.0 - fmod(kd, 3.0), 3.0);  // a whole number of three-step Philox blocks
    R.kmax = (int32_t)kd;
    R.key0 = (uint32_t)q.seed;
    R.key1 = (uint32_t)(q.seed >> 32);
    R.n_nodes = n_nodes;
    R.nodes = nodes;
    R.bmap = to_device(&q.bmap);
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
        r->state = PILOT;
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
        r->dreq = (ServeReq*)take(sizeof(ServeReq));
        r->nodes = (double*)take((size_t)r->n_nodes * 2 * sizeof(double));
        r->mean = (double*)take((size_t)r->n_nodes * 2 * sizeof(double));
        r->se = (double*)take((size_t)r->n_nodes * 2 * sizeof(double));
        r->acc = (NodeAcc*)take((size_t)r->n_nodes * sizeof(NodeAcc));
        r->vert = (double*)take((size_t)(L.sx - 1) * L.ny * 2 * sizeof(double));
        r->horiz = (double*)take((size_t)(L.sy - 1) * L.nx * 2 * sizeof(double));
        r->mesh = (double*)take((size_t)L.nx * L.ny * 2 * sizeof(double));
        r->fd_ws = (void*)take(subdomain_workspace_bytes(L));
        hipStream_t st = S->setup_stream;
        // request parameters go through the slot's pinned staging
        char* stage = S->pinned + (size_t)r->slot * S->slot_stride;
        ServeReq* hreq = (ServeReq*)stage;
        fill_serve_req(r->spec, r->nodes, (uint32_t)r->n_nodes, *hreq);
        hipError_t e = hipMemcpyAsync(r->dreq, hreq, sizeof(ServeReq), hipMemcpyHostToDevice, st);
        Density D = to_device(&r->spec.w);
        if (e == hipSuccess) e = launch_layout_nodes(L, r->spec.k, r->spec.placement, D, r->nodes, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(serve_zero_kernel, dim3((unsigned)((r->n_nodes + 255) / 256)), dim3(256), 0, st,
                               r->acc, (uint32_t)r->n_nodes);
            e = hipGetLastError();
        }
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
    ServeSeg* hs = S->hsegs[li];
    int nseg = 0;
    uint64_t tickets = 0;
    uint32_t nodes = 0;
    Lh.blocks.clear();
    for (Request* r : S->active) {
        if (nseg == kMaxSegments) break;
        if (r->cancelled || (r->state != PILOT && r->state != MAIN)) continue;
        if (r->nb_sched >= r->nb_total) continue;
        const uint64_t per_block = (uint64_t)r->n_nodes * kBlockPaths;
        uint64_t room = (uint64_t)S->launch_paths - tickets;
        uint32_t nb = (uint32_t)std::min<uint64_t>(room / per_block, r->nb_total - r->nb_sched);
        if (nb == 0) continue;
        ServeSeg& G = hs[nseg++];
        G.ticket_base = (uint32_t)tickets;
        G.node_base = nodes;
        G.n_nodes = (uint32_t)r->n_nodes;
        G.b0 = r->nb_sched;
        G.nb = nb;
        G.pad = 0;
        G.rec_base = tickets;
        G.req = r->dreq;
        G.acc = r->acc;
        tickets += per_block * nb;
        nodes += (uint32_t)r->n_nodes;
        r->nb_sched += nb;
        Lh.blocks.push_back({ r, nb });
    }
    if (nseg == 0) return false;
    Lh.busy = true;
    S->next_launch ^= 1;
    const bool have_prev = S->have_reduce;
    lk.unlock();
    hipStream_t st = S->walk_stream[li];
    hipError_t e = hipMemcpyAsync(S->dsegs[li], hs, nseg * sizeof(ServeSeg), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(serve_counter_kernel, dim3(1), dim3(1), 0, st, S->counter[li]);
        const int64_t most = ((int64_t)tickets + 255) / 256;
        const int blocks = (int)std::min<int64_t>(S->walk_blocks, most);
        hipLaunchKernelGGL(serve_walk_kernel, dim3(blocks), dim3(256), 0, st, S->dsegs[li], nseg,
                           (uint32_t)tickets, S->counter[li], S->pq[li], S->info[li]);
        e = hipGetLastError();
    }
    // reduces run in launch order: block b of a request before block b+1
    if (e == hipSuccess && have_prev) e = hipStreamWaitEvent(st, S->reduce_done, 0);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(serve_reduce_kernel, dim3(nodes), dim3(kServeBlock), 0, st, S->dsegs[li], nseg,
                           S->pq[li], S->info[li]);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(S->reduce_done, st);
    if (e == hipSuccess) e = hipEventRecord(Lh.ev, st);
    lk.lock();
    S->have_reduce = true;
    if (e != hipSuccess) {
        for (auto& b : Lh.blocks) {
            b.first->status = SDD_EDEVICE;
            b.first->cancelled = true;
        }
    }
    return true;
}

// The pilot's sums are on the host: choose the request's paths per node.
void decide_paths(sdd_server* S, Request* r)
{
    const NodeAcc* a = (const NodeAcc*)(S->pinned + (size_t)r->slot * S->slot_stride + align_up(sizeof(ServeReq), 256));
    const double n = kBlockPaths;
    double smax = 0.0;
    for (int64_t g = 0; g < r->n_nodes; ++g) {
        for (int q = 0; q < 2; ++q) {
            const double m = (a[g].s[q] + a[g].c[q]) / n;
            const double v = fmax((a[g].s[q + 2] + a[g].c[q + 2]) - n * m * m, 0.0) / (n - 1.0);
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

// Called once every block of the request is reduced: the launches that held
// them have retired (their events, recorded after their reduces, have
// completed), so the sums are final and the finish stream waits for nothing.
void finish(sdd_server* S, Request* r)
{
    hipStream_t st = S->finish_stream;
    const sdd_request& q = r->spec;
    const double paths = (double)r->nb_total * kBlockPaths;
    hipLaunchKernelGGL(serve_finalize_kernel, dim3((unsigned)((r->n_nodes + 255) / 256)), dim3(256), 0, st,
                       r->acc, (uint32_t)r->n_nodes, paths, r->mean, r->se);
    hipError_t e = hipGetLastError();
    const Bmap B = to_device(&q.bmap);
    if (e == hipSuccess) e = launch_fill(q.layout, q.k, nullptr, B, r->nodes, r->mean, q.interp, r->vert, r->horiz, st);
    if (e == hipSuccess)
        e = launch_subdomain_solve(to_device(&q.w), B, q.layout, r->vert, r->horiz, 1e-13, 100000, r->mesh, nullptr,
                                   nullptr, r->fd_ws, st);
    char* stage = S->pinned + (size_t)r->slot * S->slot_stride + align_up(sizeof(ServeReq), 256);
    const size_t acc_bytes = align_up((size_t)S->max_nodes * sizeof(NodeAcc), 256);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stage, r->acc, (size_t)r->n_nodes * sizeof(NodeAcc), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stage + acc_bytes, r->se, (size_t)r->n_nodes * 2 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stage + acc_bytes + align_up((size_t)S->max_nodes * 2 * sizeof(double), 256), r->mesh,
                           (size_t)q.layout.nx * q.layout.ny * 2 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(r->ev_done, st);
    if (e != hipSuccess) r->status = SDD_EDEVICE;
}

void complete(sdd_server* S, Request* r)
{
    // called with the lock held, after ev_done
    if (r->status == SDD_OK && !r->cancelled) {
        char* stage = S->pinned + (size_t)r->slot * S->slot_stride + align_up(sizeof(ServeReq), 256);
        const size_t acc_bytes = align_up((size_t)S->max_nodes * sizeof(NodeAcc), 256);
        const NodeAcc* a = (const NodeAcc*)stage;
        const double* se = (const double*)(stage + acc_bytes);
        const double* mesh = (const double*)(stage + acc_bytes + align_up((size_t)S->max_nodes * 2 * sizeof(double), 256));
        long long steps = 0;
        double mse = 0.0;
        for (int64_t g = 0; g < r->n_nodes; ++g) {
            steps += a[g].steps;
            mse = fmax(mse, fmax(se[2 * g], se[2 * g + 1]));
        }
        r->steps = steps;
        r->max_se = mse;
        r->paths = (int64_t)r->nb_total * kBlockPaths;
        memcpy(r->user_mesh, mesh, (size_t)r->spec.layout.nx * r->spec.layout.ny * 2 * sizeof(double));
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
            lk.lock();
            if (!done) continue;
            for (auto& b : Lh.blocks) b.first->nb_done += b.second;
            Lh.blocks.clear();
            Lh.busy = false;
            progress = true;
        }
        // pilots: copy the sums to the host, then decide the paths (the
        // pilot block's launch has retired, so its sums are final)
        for (Request* r : std::vector<Request*>(S->active)) {
            if (r->state == PILOT && !r->cancelled && r->nb_done >= 1 && !r->pilot_copy) {
                if (r->spec.se_target > 0.0) {
                    char* stage = S->pinned + (size_t)r->slot * S->slot_stride + align_up(sizeof(ServeReq), 256);
                    lk.unlock();
                    hipError_t e = hipMemcpyAsync(stage, r->acc, (size_t)r->n_nodes * sizeof(NodeAcc),
                                                  hipMemcpyDeviceToHost, S->finish_stream);
                    if (e == hipSuccess) e = hipEventRecord(r->ev_pilot, S->finish_stream);
                    lk.lock();
                    if (e != hipSuccess) {
                        r->status = SDD_EDEVICE;
                        r->cancelled = true;
                    }
                }
                r->pilot_copy = true;
                progress = true;
            }
            if (r->state == PILOT && r->pilot_copy && !r->cancelled) {
                if (r->spec.se_target > 0.0) {
                    lk.unlock();
                    const bool ready = hipEventQuery(r->ev_pilot) == hipSuccess;
                    lk.lock();
                    if (!ready) continue;
                    decide_paths(S, r);
                } else {
                    r->nb_total = (uint32_t)((r->spec.paths_per_node + kBlockPaths - 1) / kBlockPaths);
                }
                r->state = MAIN;
                progress = true;
            }
        }
        // requests whose blocks are all reduced: finish them
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
    if (launch_paths < kBlockPaths || launch_paths >= kMaxTickets) return SDD_EINVAL;
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
    for (int i = 0; i < 2 && ok; ++i) {
        ok = hipMalloc((void**)&S->pq[i], (size_t)launch_paths * sizeof(float4)) == hipSuccess &&
             hipMalloc((void**)&S->info[i], (size_t)launch_paths * sizeof(uint32_t)) == hipSuccess &&
             hipMalloc((void**)&S->dsegs[i], kMaxSegments * sizeof(ServeSeg)) == hipSuccess &&
             hipMalloc((void**)&S->counter[i], 256) == hipSuccess &&
             hipHostMalloc((void**)&S->hsegs[i], kMaxSegments * sizeof(ServeSeg), hipHostMallocDefault) == hipSuccess &&
             hipStreamCreateWithFlags(&S->walk_stream[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&S->launches[i].ev, hipEventDisableTiming) == hipSuccess;
    }
    ok = ok && hipStreamCreateWithFlags(&S->finish_stream, hipStreamNonBlocking) == hipSuccess &&
         hipStreamCreateWithFlags(&S->setup_stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&S->reduce_done, hipEventDisableTiming) == hipSuccess;
    S->slot_stride = align_up(sizeof(ServeReq), 256) + align_up((size_t)max_nodes * sizeof(NodeAcc), 256) +
                     align_up((size_t)max_nodes * 2 * sizeof(double), 256) +
                     align_up((size_t)max_points * 2 * sizeof(double), 256);
    ok = ok && hipHostMalloc((void**)&S->pinned, S->slot_stride * max_slots, hipHostMallocDefault) == hipSuccess;
    int occ = 0, cus = 0;
    ok = ok && hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, serve_walk_kernel, 256, 0) == hipSuccess &&
         hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess;
    if (!ok) {
        sdd_server_destroy(S);
        return SDD_EDEVICE;
    }
    // Waves per SIMD of each walk launch (blocks of 4 waves per CU;
    // SDD_SERVE_WAVES_PER_SIMD overrides).  Two launches are in flight, and
    // the finish stream's subdomain solves and the reduces need wave slots
    // beside them: measured same-box, 3 waves give 3% more capacity and 4-7%
    // lower p50 and p99 than 4 (which fill every SIMD with the two walks);
    // 2 lose capacity.
    int want = 3;
    if (const char* env = getenv("SDD_SERVE_WAVES_PER_SIMD"))
        if (atoi(env) > 0) want = atoi(env);
    S->walk_blocks = std::max(1, std::min(occ, want)) * cus;
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
        hipEventCreateWithFlags(&r->ev_done, hipEventDisableTiming) != hipSuccess) {
        delete r;
        return SDD_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) {
        (void)hipEventDestroy(r->ev_pilot);
        (void)hipEventDestroy(r->ev_done);
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
    }
    const sdd_status st = r->status;
    S->all.erase(it);
    (void)hipEventDestroy(r->ev_pilot);
    (void)hipEventDestroy(r->ev_done);
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
        (void)hipEventDestroy(kv.second->ev_pilot);
        (void)hipEventDestroy(kv.second->ev_done);
        delete kv.second;
    }
    for (int i = 0; i < 2; ++i) {
        if (S->walk_stream[i]) (void)hipStreamSynchronize(S->walk_stream[i]);
    }
    if (S->finish_stream) (void)hipStreamSynchronize(S->finish_stream);
    if (S->setup_stream) (void)hipStreamSynchronize(S->setup_stream);
    for (int i = 0; i < 2; ++i) {
        if (S->pq[i]) (void)hipFree(S->pq[i]);
        if (S->info[i]) (void)hipFree(S->info[i]);
        if (S->dsegs[i]) (void)hipFree(S->dsegs[i]);
        if (S->counter[i]) (void)hipFree(S->counter[i]);
        if (S->hsegs[i]) (void)hipHostFree(S->hsegs[i]);
        if (S->walk_stream[i]) (void)hipStreamDestroy(S->walk_stream[i]);
        if (S->launches[i].ev) (void)hipEventDestroy(S->launches[i].ev);
    }
    if (S->finish_stream) (void)hipStreamDestroy(S->finish_stream);
    if (S->setup_stream) (void)hipStreamDestroy(S->setup_stream);
    if (S->reduce_done) (void)hipEventDestroy(S->reduce_done);
    if (S->pinned) (void)hipHostFree(S->pinned);
    if (S->arena_base) (void)hipFree(S->arena_base);
    delete S;
    return SDD_OK;
}

}  // extern "C"
