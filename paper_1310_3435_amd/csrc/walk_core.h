// walk_core.h -- the interface walk kernel (gfx950), shared by estimate
// calls (walk.hip) and the request server (serve.hip).
//
// A persistent grid of wavefronts draws pools of consecutive paths of one
// node (64 to 256, per launch) from a device counter.  One lane walks one path; when its
// path exits, the lane takes the wave's next path, whatever node it
// belongs to, so lanes stay busy until the pools run out.  A loop iteration
// is one Philox block, i.e. three Euler-Maruyama steps (Sec. 2.2) with an
// exit test after each; a path always starts a block.  With the Brownian
// bridge the step also exits, with the bridge's conditional probability,
// when both its ends are inside; with exponential time stepping every step
// has an exponentially distributed length and the bridge test (rng.h).
//
// A finished path leaves its last step's ends P, Q and its step count in a
// per-wave queue in LDS.  Once the queue holds 64 entries the wave empties
// it with all lanes at once: each lane projects one path's last step onto
// the boundary in double (first crossing; the nearest boundary point for a
// capped path), evaluates the boundary map there (eq. (7a)) and rounds the
// value and its square to integer contributions to the node's exact sums
// (walk.h); the wave adds them and the step counts up per node into one of
// two node slots it keeps in LDS, and a slot goes to the node's sums in
// device memory with 64-bit atomics when the wave moves on to other nodes.
// The walk keeps no double-precision state, the double work runs on full
// waves, and the sums do not depend on which lane walked which path or when.
#pragma once

#include <cstddef>
#include <type_traits>

#include "common.h"
#include "rng.h"
#include "walk.h"

namespace sdd {

constexpr int kWavesPerBlock = kWalkBlock / kWave;

// ------------------------------------------------------- exit processing

// A finished path's contribution to its node's sums, kept in the lane
// between its exit processing and the per-node reduction.
struct PathValue {
    double x, y;       // boundary value at the exit point
    uint32_t steps;
    NodeAcc* acc;      // the node's sums (the reduction key)
};

// The rounded, scaled j-th of x, y, x^2, y^2 (walk.h): |n| <= 2^54.
__device__ __forceinline__ long long acc_value(const PathValue& v, const AccScale& S, int j)
{
    const double u = j == 0 ? v.x : j == 1 ? v.y : j == 2 ? v.x * v.x : v.y * v.y;
    return (long long)rint(u * S.s[j >> 1]);
}

// Exit point and boundary value of one finished path.  Writes the path's
// record in parity mode and counts a capped path.
template <typename R>
__device__ __forceinline__ PathValue finish_path(const WalkJob& J, const ExitEntry<R>& e)
{
    const double px = e.px, py = e.py, qx = e.qx, qy = e.qy;
    const uint32_t w = e.info;
    const bool capped = (w & kInfoCapped) != 0;
    double ex, ey;
    int side;
    if (w & kInfoBridged) {
        // bridged exit: the end of the step moved onto the wall it crossed
        side = (int)((w >> kInfoSideShift) & 3u);
        ex = side == 0 ? 0.0 : side == 1 ? 1.0 : qx;
        ey = side == 2 ? 0.0 : side == 3 ? 1.0 : qy;
    } else {
        side = capped ? nearest_side(qx, qy, ex, ey) : exit_point(px, py, qx, qy, ex, ey);
    }
    PathValue v;
    bmap_eval(J.bmap, side, ex, ey, v.x, v.y);
    v.steps = w & kInfoSteps;
    v.acc = J.acc + e.g;
    if (capped) atomicAdd(&v.acc->capped, 1ull);
    if (J.per_path) {
        sdd_path_record* rec = J.per_path + (size_t)e.g * J.paths + e.p;
        rec->exit_xi = ex;
        rec->exit_eta = ey;
        rec->steps = w & kInfoSteps;
        rec->side = side;
        rec->capped = capped ? 1 : 0;
    }
    return v;
}

// A wave's exit queue is a ring of kQueue entries in LDS; it is emptied up
// to 64 entries at a time, lane i finishing entry head + i.  The entries'
// contributions are then summed per node across the wave (integer sums:
// exact, in any order), and one lane per node adds them as limbs to one of
// the wave's kSlots node slots in LDS.  A slot goes to the node's sums in
// device memory (nine atomics) only when another node needs it (the least
// recently used slot goes) and at the end of the walk, so a node whose pool
// spans several drains costs nine atomics per pool instead of nine per
// drain.  Paths of a pool finish long after the pool's last path started
// (exit times have an exponential tail), so a wave has two or three nodes
// in flight; four slots keep them all.  The limb totals, and with them the
// results, are the same either way.
constexpr uint32_t kQueue = 2 * kWave;

// A wave's node slots: the node's sums address (0: empty) and the limbs
// lo[4], hi[4] and the step count, as in NodeAcc, and when each was last
// used.  Different lanes of the wave touch them in turn (the leader of each
// node), so every access is a wave-scope atomic: in order, and never kept
// in a lane's registers.
constexpr int kSlots = 4;
struct NodeSlots {
    unsigned long long key[kSlots];
    unsigned long long w[kSlots][9];
    uint32_t stamp[kSlots];
    uint32_t tick;
};

// The calling wave's slots (an address the compiler recomputes where it
// needs it rather than keeping it in a register across the walk).
__device__ __forceinline__ NodeSlots& wave_slots()
{
    __shared__ NodeSlots slots[kWavesPerBlock];
    return slots[threadIdx.x / kWave];
}

__device__ __forceinline__ unsigned long long slot_load(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void slot_store(unsigned long long* p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ uint32_t stamp_load(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void stamp_store(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

static_assert(offsetof(NodeAcc, hi) == offsetof(NodeAcc, lo) + 32 &&
                  offsetof(NodeAcc, steps) == offsetof(NodeAcc, lo) + 64,
              "a node slot's nine words follow NodeAcc's lo, hi, steps");

// Add slot s to its node's sums in device memory and empty it.
__device__ __forceinline__ void flush_slot(NodeSlots& c, uint32_t s)
{
    NodeAcc* a = (NodeAcc*)slot_load(&c.key[s]);
    // lo[4], hi[4], steps: the slot's words in NodeAcc's order
    unsigned long long* dst = &a->lo[0];
    for (int j = 0; j < 9; ++j) {
        atomicAdd(dst + j, slot_load(&c.w[s][j]));
        slot_store(&c.w[s][j], 0ull);
    }
    slot_store(&c.key[s], 0ull);
}

// Lane `lane`'s 64-bit value in scalar registers.  The builtin returns a
// signed 32-bit int: each half is taken unsigned before it is widened.
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((unsigned long long)hi << 32) | lo;
}

template <typename R, bool LANE>
__device__ __forceinline__ void drain_exits(const WalkArgs& A, const ExitEntry<R>* queue, uint32_t head,
                                            uint32_t count)
{
    __builtin_amdgcn_wave_barrier();
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const bool have = lane < count;
    PathValue v{ 0.0, 0.0, 0u, nullptr };
    AccScale S{ { 1.0, 1.0 } };
    if (have) {
        const ExitEntry<R> e = queue[(head + lane) & (kQueue - 1)];
        if constexpr (LANE) {
            const WalkJob& J = *A.segs[e.seg].job;
            v = finish_path(J, e);
            S = *J.scale;
        } else {
            v = finish_path(A.job, e);
            S = *A.job.scale;
        }
    }
    __builtin_amdgcn_wave_barrier();
    long long n[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) n[j] = have ? acc_value(v, S, j) : 0ll;
    uint64_t todo = __ballot(have);
    while (todo != 0) {
        const int leader = (int)__builtin_ctzll(todo);
        const unsigned long long acc = (unsigned long long)v.acc;
        const unsigned long long key = uniform_u64(acc, leader);
        const bool mine = have && acc == key;
        // (the leader's bit goes in any case: every pass retires a lane)
        todo &= ~(__ballot(mine) | (1ull << leader));
        const uint32_t cnt = (uint32_t)__popcll(__ballot(mine));
        // The node's lanes' n and step counts summed across the wave in 32-bit
        // words that cannot carry over 64 lanes, so that no add needs the
        // carry of another and the shuffles of a round all go out together:
        // n = l0 + l1 2^26 + l2 2^52 with l0, l1 26-bit fields and |l2| <= 4
        // (kept as l2 + 4 in 10-bit fields), the step count as its low 26
        // bits and the rest.
        uint32_t w[11];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            w[2 * j] = mine ? (uint32_t)(n[j] & 0x3ffffffll) : 0u;
            w[2 * j + 1] = mine ? (uint32_t)((n[j] >> 26) & 0x3ffffffll) : 0u;
        }
        w[8] = mine ? (v.steps & 0x3ffffffu) : 0u;
        w[9] = mine ? ((uint32_t)((n[0] >> 52) + 4) | (uint32_t)((n[1] >> 52) + 4) << 10 |
                       (uint32_t)((n[2] >> 52) + 4) << 20)
                    : 0u;
        w[10] = mine ? ((uint32_t)((n[3] >> 52) + 4) | (v.steps >> 26) << 10) : 0u;
#pragma unroll
        for (int m = kWave / 2; m >= 1; m >>= 1) {
#pragma unroll
            for (int j = 0; j < 11; ++j) w[j] += (uint32_t)__shfl_xor((int)w[j], m, kWave);
        }
        if ((int)lane == leader) {
            NodeSlots& slots = wave_slots();
            uint32_t s = kSlots;
#pragma unroll
            for (int i = 0; i < kSlots; ++i)
                if (slot_load(&slots.key[i]) == key) s = (uint32_t)i;
            const uint32_t tick = stamp_load(&slots.tick) + 1u;
            if (s == kSlots) {
                // an empty slot, else the least recently used one
                uint32_t oldest = 0xffffffffu;
                s = 0u;
#pragma unroll
                for (int i = 0; i < kSlots; ++i) {
                    const uint32_t t = slot_load(&slots.key[i]) == 0ull ? 0u : stamp_load(&slots.stamp[i]);
                    if (t < oldest) {
                        oldest = t;
                        s = (uint32_t)i;
                    }
                }
                if (slot_load(&slots.key[s]) != 0ull) flush_slot(slots, s);
                slot_store(&slots.key[s], key);
            }
            stamp_store(&slots.stamp[s], tick);
            stamp_store(&slots.tick, tick);
            const uint32_t h[4] = { w[9] & 0x3ffu, (w[9] >> 10) & 0x3ffu, (w[9] >> 20) & 0x3ffu, w[10] & 0x3ffu };
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                // the node's sum of n over these lanes, |t| <= 2^60
                const long long t = (long long)w[2 * j] + ((long long)w[2 * j + 1] << 26) +
                                    (long long)((int)h[j] - 4 * (int)cnt) * (1ll << 52);
                __hip_atomic_fetch_add(&slots.w[s][j], (unsigned long long)(t & 0x7fffffffll), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WAVEFRONT);
                __hip_atomic_fetch_add(&slots.w[s][4 + j], (unsigned long long)(t >> 31), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
            __hip_atomic_fetch_add(&slots.w[s][8], (unsigned long long)w[8] + ((unsigned long long)(w[10] >> 10) << 26),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
    }
}

// ------------------------------------------------------------ the walk

// The drift times `scale`: the float walk with fixed steps takes b dt
// (scale = dt: the constants times dt are loop invariants, and the update
// X + b dt becomes one FMA per coordinate), exponential steps b (scale 1).
// The double walk takes b.
template <int KIND>
__device__ __forceinline__ void drift(const WalkArgs& A, float scale, float x, float y, float& bx, float& by)
{
    if constexpr (KIND == kGaussSum) {
        const GaussParams& G = A.job.gp;
        float m2c[SDD_MAX_TERMS];
#pragma unroll
        for (int q = 0; q < SDD_MAX_TERMS; ++q) m2c[q] = G.m2c[q] * scale;
        gauss_sum_drift(G.n_terms, G.base, G.cx, G.cy, G.k2, G.la, m2c, x, y, bx, by);
    } else {
        drift_f32<KIND>(A.dens, scale, x, y, bx, by);
    }
}
template <int KIND>
__device__ __forceinline__ void drift(const WalkArgs& A, double, double x, double y, double& bx, double& by)
{
    drift_f64<KIND>(A.dens, x, y, bx, by);
}

// Noise factor of one step: sqrt(2 dt) times the normals' scale (rng.h).
__device__ __forceinline__ float noise_scale(const WalkArgs& A, float) { return (float)A.noise_f32; }
__device__ __forceinline__ double noise_scale(const WalkArgs& A, double) { return A.sqrt2dt; }
// Constant of the bridge test: -log2(e)/dt in float, dt in double.
__device__ __forceinline__ float bridge_const(double dt, float) { return (float)(-1.4426950408889634 / dt); }
__device__ __forceinline__ double bridge_const(double dt, double) { return dt; }
// Exponential steps: tau = -log2(u) (dt ln 2) in float, -ln(u) dt in double;
// then the noise factor and the bridge constant of that step.
__device__ __forceinline__ float expo_const(double dt, float) { return (float)(dt * 0.69314718055994530942); }
__device__ __forceinline__ double expo_const(double dt, double) { return dt; }
__device__ __forceinline__ float expo_noise(float tau) { return __builtin_amdgcn_sqrtf(tau * 2.7725887222397812f); }
__device__ __forceinline__ double expo_noise(double tau) { return sqrt(2.0 * tau); }
__device__ __forceinline__ float expo_bridge(float tau) { return -kLog2e * __builtin_amdgcn_rcpf(tau); }
__device__ __forceinline__ double expo_bridge(double tau) { return tau; }

// Wave-uniform reads of data the walk never writes (segments, jobs, node
// coordinates) go through the constant address space, so that they are
// scalar loads through the scalar cache rather than a load per lane.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* uniform_ptr(const T* p)
{
    return (const __attribute__((address_space(4))) T*)p;
}

// Segment of pool q (server): the last segment with pool_base <= q.
__device__ __forceinline__ int find_segment(const WalkSeg* segs, int nseg, uint64_t q)
{
    const auto* cs = uniform_ptr(segs);
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cs[mid].pool_base <= q) lo = mid; else hi = mid;
    }
    return lo;
}

// R: walk precision.  KIND: density kind (common.h).  EXIT: ExitKind.
// PIPE: each iteration also computes the next three steps' Philox block
// (it depends on the counters only), so that waves have independent work
// to overlap with the steps' latency; the random numbers, and hence all
// results, are the same either way.  LANE: per-lane job parameters
// (request server; float Gaussian sums), else wave-uniform ones in A.
template <typename R, int KIND, int EXIT, bool PIPE, bool LANE>
__device__ __forceinline__ void walk_body(const WalkArgs& A)
{
    static_assert(!LANE || (KIND == kGaussSum && EXIT == kExitLane), "the server walks float Gaussian sums");
    __shared__ ExitEntry<R> queues[kWavesPerBlock][kQueue];
    ExitEntry<R>* queue = queues[threadIdx.x / kWave];
    uint32_t qh = 0, qn = 0;  // first entry and entries in the wave's queue (wave-uniform)
    const int lane = threadIdx.x & (kWave - 1);
    if (lane == 0) {
        NodeSlots& slots = wave_slots();
        for (int j = 0; j < kSlots; ++j) {
            slot_store(&slots.key[j], 0ull);
            for (int i = 0; i < 9; ++i) slot_store(&slots.w[j][i], 0ull);
            stamp_store(&slots.stamp[j], 0u);
        }
        stamp_store(&slots.tick, 0u);
    }

    // wave-uniform pool: node, next path, end, and (per-lane jobs) the job
    uint32_t pool_g = 0, pool_p = 0, pool_end = 0, pool_seg = 0;
    double pool_x = 0.0, pool_y = 0.0;  // per-lane jobs: the pool's node (scalar loads)
    // (per-lane jobs only; never the address of the kernel argument, which
    // would put a copy of the whole argument block in per-lane scratch)
    const WalkJob* pool_job = nullptr;
    bool exhausted = false;
    // lane state
    bool live = false;
    uint32_t g = 0, p = 0, seg = 0, pc = 0;  // node, path, segment, path counter word
    uint4 rc = make_uint4(0, 0, 0, 0);      // Philox block of the lane's current steps (PIPE)
    R X = 0, Y = 0;
    uint32_t m = 0;  // Philox block index: steps 3m .. 3m+2
    // step parameters: wave-uniform, or the lane's job
    R dt = (R)A.dt, sd = noise_scale(A, R(0)), bc = bridge_const(A.dt, R(0));
    const R ec = expo_const(A.dt, R(0));
    uint32_t mmax = (uint32_t)(A.kmax / 3);
    uint32_t key0 = A.job.key0, key1 = A.job.key1;
    bool lbridge = false;
    GaussParams lg;
    // Euler-Maruyama step x + b dt + s z: float walks with fixed steps get
    // b dt from the drift (scale dt, one FMA fewer per coordinate), others b
    constexpr bool kDriftDt = std::is_same<R, float>::value && EXIT != kExitExpo;
    const float dscale = kDriftDt ? (float)A.dt : 1.0f;
    auto euler = [](R x, R b, R d, R s, R z) { return kDriftDt ? fmar(s, z, x + b) : fmar(s, z, fmar(b, d, x)); };
    if constexpr (LANE) {
        lg.n_terms = 0;
        lg.base = 1.0f;
#pragma unroll
        for (int q = 0; q < SDD_MAX_TERMS; ++q) lg.cx[q] = lg.cy[q] = lg.k2[q] = lg.la[q] = lg.m2c[q] = 0.0f;
    }

    for (;;) {
        // hand the wave's pools to idle lanes, in lane order
        uint64_t need = __ballot(!live);
        while (need != 0 && !exhausted) {
            if (pool_p == pool_end) {
                unsigned long long q = 0;
                if (lane == 0) q = atomicAdd(A.counter, 1ull);
                q = uniform_u64(q, 0);  // lane 0's ticket, in scalar registers
                if (q >= A.total_pools) {
                    exhausted = true;
                    break;
                }
                int si = 0;
                WalkSeg S;
                if constexpr (LANE) {
                    si = find_segment(A.segs, A.nseg, q);
                    const auto* cs = uniform_ptr(A.segs) + si;
                    S.pool_base = cs->pool_base;
                    S.job = cs->job;
                    S.n_nodes = cs->n_nodes;
                    S.p_lo = cs->p_lo;
                    S.p_hi = cs->p_hi;
                    pool_job = S.job;
                } else {
                    S = A.seg;
                }
                // pools go round the nodes (pool j of node g is local pool
                // j n + g), so that waves working at the same time add into
                // different nodes' sums
                const uint64_t local = q - S.pool_base;
                const uint64_t c = local / S.n_nodes;
                pool_g = (uint32_t)(local - c * S.n_nodes);
                pool_p = S.p_lo + (uint32_t)c * A.pool_paths;
                pool_end = min(S.p_hi, pool_p + A.pool_paths);
                pool_seg = (uint32_t)si;
                if constexpr (LANE) {
                    const double* nodes = uniform_ptr(pool_job)->nodes;
                    pool_x = uniform_ptr(nodes)[2 * (size_t)pool_g];
                    pool_y = uniform_ptr(nodes)[2 * (size_t)pool_g + 1];
                }
            }
            const uint32_t avail = pool_end - pool_p;
            const uint32_t want = (uint32_t)__popcll(need);
            const uint32_t take = want < avail ? want : avail;
            const uint32_t rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
            if (!live && rank < take) {
                g = pool_g;
                p = pool_p + rank;
                seg = pool_seg;
                const WalkJob& J = LANE ? *pool_job : A.job;  // the pool's job: a uniform address
                if constexpr (LANE) {
                    const auto* cj = uniform_ptr(pool_job);
                    lg.n_terms = cj->gp.n_terms;
                    lg.base = cj->gp.base;
                    dt = cj->dt;
#pragma unroll
                    for (int q = 0; q < SDD_MAX_TERMS; ++q) {
                        lg.cx[q] = cj->gp.cx[q];
                        lg.cy[q] = cj->gp.cy[q];
                        lg.k2[q] = cj->gp.k2[q];
                        lg.la[q] = cj->gp.la[q];
                        // the server's steps are fixed: its drift is b dt (see drift)
                        lg.m2c[q] = cj->gp.m2c[q] * dt;
                    }
                    sd = cj->noise;
                    bc = cj->bridge_c;
                    lbridge = cj->exit_test == SDD_EXIT_BRIDGE;
                    mmax = cj->kblocks;
                    key0 = cj->key0;
                    key1 = cj->key1;
                    pc = cj->path0 + p;
                } else {
                    pc = A.job.path0 + p;
                }
                // (an estimate call's kernel keeps its scalar registers for
                // the wave-uniform density: per-lane loads of the node)
                const double nx0 = LANE ? pool_x : A.job.nodes[2 * (size_t)g];
                const double ny0 = LANE ? pool_y : A.job.nodes[2 * (size_t)g + 1];
                if (nx0 > 0.0 && nx0 < 1.0 && ny0 > 0.0 && ny0 < 1.0) {
                    X = (R)nx0;
                    Y = (R)ny0;
                    m = 0;
                    live = true;
                    if constexpr (PIPE) rc = philox(0u, pc, g, 0u, key0, key1);
                } else {
                    // a node off the open square walks nothing: NaN result
                    J.acc[g].invalid = 1u;
                    if (J.per_path) {
                        sdd_path_record* rec = J.per_path + (size_t)g * J.paths + p;
                        rec->exit_xi = rec->exit_eta = __builtin_nan("");
                        rec->steps = 0;
                        rec->side = -1;
                        rec->capped = 0;
                    }
                }
            }
            pool_p += take;
            need = __ballot(!live);
        }
        if (__ballot(live) == 0) break;

        uint4 r;
        if constexpr (PIPE) {
            r = rc;
            rc = philox(m + 1u, pc, g, 0u, key0, key1);
        } else {
            r = philox(m, pc, g, 0u, key0, key1);
        }
        // step lengths, noise factors and bridge constants of the three steps
        R dA = dt, dB = dt, dC = dt, sA = sd, sB = sd, sC = sd, cA = bc, cB = bc, cC = bc;
        if constexpr (EXIT == kExitExpo) {
            const uint4 e = philox(m, pc, g, 2u, key0, key1);
            dA = expo_step(e.x, ec);
            dB = expo_step(e.y, ec);
            dC = expo_step(e.z, ec);
            sA = expo_noise(dA);
            sB = expo_noise(dB);
            sC = expo_noise(dC);
            cA = expo_bridge(dA);
            cB = expo_bridge(dB);
            cC = expo_bridge(dC);
        }
        R bx, by, z0, z1;
        // step 3m
        normals(field_hi(r.x, R(0)), field_hi(r.y, R(0)), z0, z1);
        if constexpr (LANE) gauss_sum_drift(lg.n_terms, lg.base, lg.cx, lg.cy, lg.k2, lg.la, lg.m2c, X, Y, bx, by);
        else drift<KIND>(A, dscale, X, Y, bx, by);
        const R XA = euler(X, bx, dA, sA, z0);
        const R YA = euler(Y, by, dA, sA, z1);
        // step 3m+1
        normals(field_hi(r.z, R(0)), field_hi(r.w, R(0)), z0, z1);
        if constexpr (LANE) gauss_sum_drift(lg.n_terms, lg.base, lg.cx, lg.cy, lg.k2, lg.la, lg.m2c, XA, YA, bx, by);
        else drift<KIND>(A, dscale, XA, YA, bx, by);
        const R XB = euler(XA, bx, dB, sB, z0);
        const R YB = euler(YA, by, dB, sB, z1);
        // step 3m+2
        normals(field_lo(r.x, r.y, R(0)), field_lo(r.z, r.w, R(0)), z0, z1);
        if constexpr (LANE) gauss_sum_drift(lg.n_terms, lg.base, lg.cx, lg.cy, lg.k2, lg.la, lg.m2c, XB, YB, bx, by);
        else drift<KIND>(A, dscale, XB, YB, bx, by);
        const R XC = euler(XB, bx, dC, sC, z0);
        const R YC = euler(YB, by, dC, sC, z1);

        // the step cap is a whole number of blocks, so it can only fall
        // after step 3m+2
        const bool outA = outside(XA, YA);
        const bool outB = outside(XB, YB);
        const bool outC = outside(XC, YC);
        bool exA = outA, exB = outB, exC = outC;
        bool test = EXIT == kExitBridge || EXIT == kExitExpo;
        if constexpr (EXIT == kExitLane) test = __ballot(live && lbridge) != 0;  // some lane's job asks for it
        if (test) {
            const bool mine = EXIT == kExitLane ? lbridge : true;
            const R PA = bridge_prob(X, Y, XA, YA, cA);
            const R PB = bridge_prob(XA, YA, XB, YB, cB);
            const R PC = bridge_prob(XB, YB, XC, YC, cC);
            const bool may = (!outA && bridge_may_exit(PA)) || (!outB && bridge_may_exit(PB)) ||
                             (!outC && bridge_may_exit(PC));
            if (__ballot(live && mine && may) != 0) {
                // some lane is near a wall: draw the bridge block (wave-uniform branch)
                const uint4 q = philox(m, pc, g, 1u, key0, key1);
                exA = outA || (mine && uniform23(q.x, R(0)) < PA);
                exB = outB || (mine && uniform23(q.y, R(0)) < PB);
                exC = outC || (mine && uniform23(q.z, R(0)) < PC);
            }
        }
        const bool fin = live && (exA || exB || exC || (m + 1u >= mmax));
        const uint64_t fm = __ballot(fin);
        if (fm != 0) {
            const uint32_t nf = (uint32_t)__popcll(fm);
            if (fin) {
                // the first exiting step's ends
                const R px = exA ? X : (exB ? XA : XB), py = exA ? Y : (exB ? YA : YB);
                const R qx = exA ? XA : (exB ? XB : XC), qy = exA ? YA : (exB ? YB : YC);
                uint32_t w = 3u * m + (exA ? 1u : (exB ? 2u : 3u));
                if (!(exA || exB || exC))
                    w |= kInfoCapped;
                else if (EXIT != kExitStep && !(exA ? outA : (exB ? outB : outC)))
                    w |= kInfoBridged | (bridge_side(px, py, qx, qy) << kInfoSideShift);
                const uint32_t slot =
                    qh + qn + __builtin_amdgcn_mbcnt_hi((uint32_t)(fm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)fm, 0u));
                ExitEntry<R>& E = queue[slot & (kQueue - 1)];
                E.px = px;
                E.py = py;
                E.qx = qx;
                E.qy = qy;
                E.info = w;
                E.g = g;
                E.p = p;
                E.seg = seg;
                live = false;
            }
            qn += nf;
        }
        // finished and idle lanes carry garbage until their next start
        X = XC;
        Y = YC;
        ++m;
        if (qn >= (uint32_t)kWave) {  // at most 127 entries: room for the next iteration's 64
            drain_exits<R, LANE>(A, queue, qh, kWave);
            qh = (qh + kWave) & (kQueue - 1);
            qn -= kWave;
        }
    }
    while (qn) {
        const uint32_t c = qn < (uint32_t)kWave ? qn : (uint32_t)kWave;
        drain_exits<R, LANE>(A, queue, qh, c);
        qh = (qh + c) & (kQueue - 1);
        qn -= c;
    }
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
        NodeSlots& slots = wave_slots();
        for (uint32_t j = 0; j < (uint32_t)kSlots; ++j)
            if (slot_load(&slots.key[j]) != 0ull) flush_slot(slots, j);
    }
}

template <typename R, int KIND, int EXIT, bool PIPE, bool LANE>
__global__ __launch_bounds__(kWalkBlock) void walk_kernel(const WalkArgs A)
{
    walk_body<R, KIND, EXIT, PIPE, LANE>(A);
}

// The same walk held to 64 VGPRs, so that 8 waves fit on a SIMD; what the
// exit drain's double projection needs beyond that spills to scratch.  The
// general sum of terms, whose loop over the terms leaves latency that more
// waves hide, takes it on short paths (see the launch).
template <typename R, int KIND, int EXIT>
__global__ __launch_bounds__(kWalkBlock) __attribute__((amdgpu_waves_per_eu(8))) void walk_kernel_wide(
    const WalkArgs A)
{
    walk_body<R, KIND, EXIT, false, false>(A);
}

}  // namespace sdd
