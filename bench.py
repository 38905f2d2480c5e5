"""Throughput benchmark of the interface Monte Carlo hot path on one MI355X.

One step = one pass of the whole path over the workload: interface
estimate (walk + finalize), interface fill and the batched subdomain
solves, all on the GPU, inputs already resident in HBM.  Prints one JSON
line.

Default workload (the largest single-GPU one): shear-layer density
w = 1 + 20 sech^2(40 (xi - eta)) on the quarter annulus 1 <= rho <= 2,
8 x 8 subdomains of 129 x 129 nodes (global 1025 x 1025), 32 points per
interface segment placed by equidistributing w (3633 nodes), 1e5 paths per
node, dt = 1e-5, float walk with exact double node sums, monotone cubic
fill.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-cpu-baseline] [--no-ring] [--serve-requests N]
                    [--serve-load RHO] [--serve-bridge-dt DT]

Beside the throughput line it reports the ring workload (4 x 4 of 65 x 65,
1521 nodes x 1e4 paths) with its double-precision walk (equal paths, hence
equal standard error) and its 64-node double-oracle subset, the
Brownian-bridge and exponential-stepping legs on the closed-form workload,
and a serving run: a Poisson stream of mesh requests at RHO x the measured
capacity, with p50/p99 latency from arrival to the mesh in host memory.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 floating-point operations per float Euler-Maruyama step
# (FMA = 2, transcendental = 1), the roofline's unit of work, fixed by the
# method rather than by how the kernel evaluates it: Philox's integer work
# aside, a step converts two uniforms, makes two Box-Muller normals (log,
# sqrt, sin, cos and products), evaluates the drift (one Gaussian term: the
# offsets, r^2, an exp, the gradient products and a reciprocal) and updates
# both coordinates (4 FMA): 34 flops.  The ring adds a square root and a
# reciprocal (36), sin^2 takes a sine and a cosine in place of the exp
# (35), sech^2 an exp and a reciprocal like the Gaussian (34).  The kernel
# executes fewer (31 for sech^2 after its algebra; the counters report
# them), which the issue model below accounts.  The peak is MI355X's
# published FP32 vector rate.
FP32_FLOPS_PER_STEP = {"ring": 36, "gauss": 34, "sech2": 34, "sin2": 35}
FP32_PEAK_TFLOPS = 157.3
# Issue-cycle view, beside the FLOP roofline: SIMD cycles per wave64 step
# from the algorithm's instruction mix weighted by gfx950's measured issue
# cost per instruction class (profiles/valu_rates_gfx950.md: two-operand
# ops 2 cycles, three-operand ops (fma, v_bitop3_b32, v_and_or_b32,
# v_mad_u64_u32) 4, transcendentals 8).  Per step: a third of a
# Philox4x32-10 block (20 v_mad_u64_u32 + 20 v_bitop3_b32 = 160 per block),
# two uniforms (60 per block, 20 a step), Box-Muller 36, the drift (ring 56,
# one Gaussian term 42, sech2 46, sin2 46), the update 16, the exit test 8.
# Capacity: 256 CUs x 4 SIMDs x 2.4 GHz.
_STEP_COMMON = 160 / 3 + 20 + 36 + 16 + 8
CYCLES_PER_WAVE_STEP = {k: _STEP_COMMON + d for k, d in
                        {"ring": 56, "gauss": 42, "sech2": 46, "sin2": 46}.items()}
ISSUE_PEAK_G = 256 * 4 * 2.4e9 / 1e9  # G SIMD-cycles/s
# A float sum of n Gaussian bumps (the request server's densities): per term
# two offsets, a product, two FMAs, the exp, the sum, a product and two
# gradient FMAs (34 cycles); then one rcp (8; the products by 1/w fuse into
# the update).


def gauss_sum_cycles(n_terms: int) -> float:
    return _STEP_COMMON + 34 * n_terms + 8
# HBM bytes the walk must move per launch: the node table (16 B a node) and
# the node sums (96 B a node, zeroed then written back); a path reads and
# writes nothing beyond on-chip memory and the node sums' cache lines.
WALK_BYTES_PER_NODE = 16 + 2 * 96


def kernel_source_hash(src_dir: str = None) -> str:
    """Hash of the walk kernel's code (comments and layout removed) and of
    the compiler flags (without include paths), which ties the committed
    counter figures to the kernel they were taken on."""
    import re

    from paper_1310_3435_amd import build
    src_dir = src_dir or os.path.join(ROOT, "paper_1310_3435_amd", "csrc")
    h = hashlib.sha256()
    h.update(" ".join(f for f in build.FLAGS if not os.path.isabs(f)).encode())
    for f in ("walk.hip", "walk.h", "walk_core.h", "common.h", "rng.h"):
        with open(os.path.join(src_dir, f)) as fh:
            code = fh.read()
        code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(workload: str):
    """HBM bytes per walk launch from the committed counter summary, if it was
    taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"walk_{workload}_traffic.txt")
    if not os.path.exists(p):
        return None
    vals = {}
    for line in open(p):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(cfg, nodes, sample_nodes: int, full_steps: int, gpu_mean=None, single_paths: int = 10000,
                 sample_paths: int = 0):
    """The oracle, untuned, on this host's cores: `sample_nodes` evenly spaced
    nodes of the same workload, `sample_paths` paths each (0: the workload's
    own), double precision; then one node with `single_paths` paths on one
    core.  The full workload's oracle time is extrapolated linearly in steps
    from the all-core rate.  With gpu_mean (the GPU's float estimate of every
    node over the same first paths: the same counters, so the same paths)
    the sample also gives, node by node, |GPU - oracle| / SE."""
    import numpy as np

    import oracle
    oracle.lib()
    n = nodes.shape[0]
    idx = (np.arange(sample_nodes) * (n // sample_nodes)).astype(np.int64)
    threads = host_threads()
    paths = sample_paths or cfg["paths"]
    t0 = time.perf_counter()
    r = oracle.interface_estimate(cfg["density"], cfg["bmap"], nodes[idx], paths, cfg["dt"], cfg["seed"],
                                  "fp64", node_ids=idx, nthreads=threads)
    el = time.perf_counter() - t0
    one = idx[sample_nodes // 2: sample_nodes // 2 + 1]
    t0 = time.perf_counter()
    r1 = oracle.interface_estimate(cfg["density"], cfg["bmap"], nodes[one], single_paths, cfg["dt"], cfg["seed"],
                                   "fp64", node_ids=one, nthreads=1)
    el1 = time.perf_counter() - t0
    rate = r["steps"] / el
    out = {"value": rate, "unit": "walk steps/s", "cores": threads, "kind": "oracle",
           "sample": f"{sample_nodes} of {n} nodes (indices i*{n // sample_nodes}), paths 0..{paths - 1} of each, "
                     f"dt={cfg['dt']}, fp64 walk, {r['steps']} steps in {el:.2f} s",
           "nodes_per_s": sample_nodes / el, "cpu": cpu_model(),
           "single_core": {"value": r1["steps"] / el1, "unit": "walk steps/s",
                           "sample": f"node {int(one[0])}, {single_paths} paths, {r1['steps']} steps in {el1:.2f} s"},
           "full_workload_s_extrapolated": full_steps / rate}
    if gpu_mean is not None:
        z = np.abs(gpu_mean[idx] - r["mean"]) / r["se"]
        out["gpu_vs_oracle"] = {"what": "float GPU walk against this double oracle run, same paths, per node",
                                "abs_diff_over_se": [round(float(v), 5) for v in z.max(1)],
                                "max_abs_diff": float(np.abs(gpu_mean[idx] - r["mean"]).max()),
                                "median_se": float(np.median(r["se"]))}
    return out


def serve_stream(ctx, n_requests: int, load: float, burst: int, seed: int = 4, bridge_dt: float = 0.0,
                 launch_paths: int = 0):
    """Serving stream: a burst of `burst` requests measures capacity
    (requests/s at saturation); then `n_requests` arrive as a Poisson stream
    at `load` x capacity.  Latency = arrival (submit) to the mesh being in
    host memory, on the server's clock.  bridge_dt > 0: every request uses
    the Brownian-bridge exit test at that time step instead."""
    import numpy as np

    import paper_1310_3435_amd as sdd
    import workloads

    reqs = workloads.serving_requests(n_requests + burst, master_seed=seed)
    if bridge_dt > 0:
        reqs = [dict(r, exit_test="bridge", dt=bridge_dt) for r in reqs]
    srv = sdd.Server(ctx, hbm_budget_bytes=4 << 30, max_slots=64, max_nodes=4096, max_points=257 * 257,
                     launch_paths=launch_paths)
    try:
        t0 = srv.clock()
        ids = [srv.submit(r) for r in reqs[:burst]]
        res = [srv.wait(i) for i in ids]
        t_burst = max(r["t_done"] for r in res) - t0
        burst_steps = sum(r["steps"] for r in res if r["status"] >= 0)
        capacity = burst / t_burst
        rate = load * capacity
        arrivals = workloads.poisson_arrivals(n_requests, rate, seed=seed)
        out, pending = [], {}
        start = time.perf_counter()

        def done(r):
            out.append(r)
            if len(out) % 100 == 0:
                print(f"[serve] {len(out)} of {n_requests} requests done, "
                      f"{time.perf_counter() - start:.0f} s", file=sys.stderr, flush=True)

        def shape(r, req):
            L = req["layout"]
            r.update(grid=f"{L['nx']}x{L['ny']}", subdomains=f"{L['sx']}x{L['sy']}", nodes=r["n_nodes"])
            return r

        for req, ta in zip(reqs[burst:], arrivals):
            while True:
                now = time.perf_counter() - start
                for rid in list(pending):
                    r = srv.poll(rid)
                    if r is not None:
                        done(shape(r, pending.pop(rid)))
                if now >= ta:
                    break
                time.sleep(min(ta - now, 0.002))
            pending[srv.submit(req)] = req
        for rid in list(pending):
            done(shape(srv.wait(rid), pending[rid]))
        wall = max(r["t_done"] for r in out) - min(r["t_submit"] for r in out)
    finally:
        srv.close()
    ok = [r for r in out if r["status"] >= 0]   # 0, or 1: done with capped paths
    lat = np.array([r["t_done"] - r["t_submit"] for r in ok]) * 1e3
    steps = sum(r["steps"] for r in ok)
    return {
        "requests": len(out), "completed": len(ok), "load": load,
        "arrival_rate_per_s": rate, "capacity_req_per_s": capacity,
        "p50_latency_ms": float(np.percentile(lat, 50)), "p99_latency_ms": float(np.percentile(lat, 99)),
        "mean_latency_ms": float(lat.mean()), "throughput_req_per_s": len(ok) / wall,
        "walk_steps_per_s": steps / wall, "walk_steps": steps, "burst_walk_steps": burst_steps,
        "median_paths_per_node": float(np.median([r["paths_per_node"] for r in ok])),
        "max_se": float(max(r["max_se"] for r in ok)),
        "capped_paths": int(sum(r["capped"] for r in ok)),
        "stage_ms_median": {k: float(np.median([r[k] for r in ok]))
                            for k in ("t_queue_ms", "t_stoc_ms", "t_fill_ms", "t_sub_ms")},
        "stage_ms_p99": {k: float(np.percentile([r[k] for r in ok], 99))
                         for k in ("t_queue_ms", "t_stoc_ms", "t_fill_ms", "t_sub_ms")},
        "slowest_1pct": slowest(ok, lat),
        "stream": "1-4 Gaussian bumps (amp U[1,20], width U[20,200]), grids {33,65,129,257}^2, 2x2..8x8 "
                  "subdomains, SE 1e-3 per node, float walks, Poisson arrivals, "
                  + (f"bridge exit test at dt {bridge_dt:g}" if bridge_dt > 0 else "end-of-step exit test at dt 1e-4"),
    }


def slowest(ok, lat):
    """The slowest 1% of requests: their shapes and where their time went."""
    import numpy as np
    k = max(1, len(ok) // 100)
    order = np.argsort(lat)[::-1][:k]
    rows = []
    for i in order:
        r = ok[int(i)]
        rows.append({"latency_ms": round(float(lat[i]), 1),
                     **{key: r.get(key) for key in ("grid", "subdomains", "nodes", "paths_per_node")},
                     **{key: round(float(r[key]), 2) for key in ("t_queue_ms", "t_stoc_ms", "t_fill_ms", "t_sub_ms")}})
    return rows


def serve_like(ctx, grid: int = 257, sub: int = 8, paths: int = 65536, dt: float = 1e-4):
    """One request of the serving stream's shape (grid^2, sub x sub
    subdomains, two Gaussian bumps, end-of-step test) through the server and
    through sdd_interface_estimate on the same nodes, paths and seed: the
    same steps (asserted), timed each on its own walk (the server's T_stoc,
    HIP events around the estimate call), with the issue model of a
    two-term Gaussian sum beside each rate."""
    import torch

    import paper_1310_3435_amd as sdd
    import workloads
    terms = [{"kind": "gauss", "amp": 6.0, "coef": 60.0, "cx": 0.4, "cy": 0.55},
             {"kind": "gauss", "amp": 12.0, "coef": 150.0, "cx": 0.7, "cy": 0.3}]
    dens = workloads.density(1.0, terms)
    L = {"nx": grid, "ny": grid, "sx": sub, "sy": sub}
    k = (grid - 1) // sub - 1
    req = {"density": dens, "bmap": {"kind": "identity"}, "layout": L, "k": k, "placement": "uniform",
           "interp": "linear", "dt": dt, "se_target": 0.0, "paths": paths, "seed": 5, "exit_test": "step"}
    srv = sdd.Server(ctx, hbm_budget_bytes=256 << 20, max_slots=4, max_nodes=8192)
    try:
        srv.wait(srv.submit(req))  # loads the kernels
        r = srv.wait(srv.submit(req))
    finally:
        srv.close()
    nodes = sdd.sdd_layout_nodes(ctx, L, k, "uniform", dens)
    e, _ = timed_estimate(ctx, dens, {"kind": "identity"}, nodes, r["paths_per_node"], dt, 5, "fp32")
    e, ms = timed_estimate(ctx, dens, {"kind": "identity"}, nodes, r["paths_per_node"], dt, 5, "fp32", out=e)
    torch.cuda.synchronize()
    steps = int(e["stats"].cpu().numpy()[0])
    assert steps == r["steps"], "the server walked other paths than the estimate call"
    cyc = gauss_sum_cycles(len(terms))
    out = {"workload": f"{grid}^2, {sub}x{sub} subdomains, {int(nodes.shape[0])} nodes x {r['paths_per_node']} "
                       f"paths, two Gaussian bumps, end-of-step test at dt {dt:g}, float walk",
           "steps": steps, "serve_walk_ms": r["t_stoc_ms"], "estimate_walk_ms": ms,
           "serve_steps_per_s": steps / (r["t_stoc_ms"] * 1e-3), "estimate_steps_per_s": steps / (ms * 1e-3)}
    out["serve_over_estimate"] = out["serve_steps_per_s"] / out["estimate_steps_per_s"]
    # the plain double path on the same paths: equal standard error
    sdd.sdd_interface_estimate(ctx, dens, {"kind": "identity"}, nodes, 1024, dt, 5, "fp64")  # loads the kernel
    e64, ms64 = timed_estimate(ctx, dens, {"kind": "identity"}, nodes, r["paths_per_node"], dt, 5, "fp64")
    se32, se64 = float(e["se"].median()), float(e64["se"].median())
    out["fp64_estimate_walk_ms"] = ms64
    out["median_se"] = {"fp32": se32, "fp64": se64}
    out["served_fp32_speedup_over_fp64_at_equal_se"] = ms64 / r["t_stoc_ms"]
    out["issue_model"] = {"cycles_per_wave_step": round(cyc, 2), "peak_G_cycles_per_s": ISSUE_PEAK_G,
                          "serve_frac": out["serve_steps_per_s"] / 64 * cyc / 1e9 / ISSUE_PEAK_G,
                          "estimate_frac": out["estimate_steps_per_s"] / 64 * cyc / 1e9 / ISSUE_PEAK_G}
    return out


def closed_form_sin2(xi):
    """x(xi) = int_0^xi 1/w / int_0^1 1/w for w = 1 + 3 sin^2(2 pi xi): with
    Theta(t) = arctan(2 tan t) continued through the poles, x = Theta(2 pi xi)/(2 pi)."""
    import numpy as np
    t = 2 * np.pi * np.asarray(xi, dtype=np.float64)
    th = np.arctan2(2 * np.sin(t), np.cos(t))
    return np.where(th < 0, th + 2 * np.pi, th) / (2 * np.pi)


def sin2_estimate(ctx, paths: int, dt: float, prec: str, exit_test: str, warm: bool = True):
    """One timed walk of the 64-node sin^2 workload (after an untimed one of
    1024 paths, which loads the kernel); errors against the closed form.
    Returns a row of figures."""
    import numpy as np
    import torch

    import paper_1310_3435_amd as sdd
    import workloads

    cfg = workloads.cfg_sin2_sweep()
    dens = cfg["density"]
    B = sdd.Bmap(cfg["bmap"], ctx, dens)
    nodes_np = np.array(cfg["nodes"])
    nodes = torch.as_tensor(nodes_np).cuda()
    exact = np.stack([closed_form_sin2(nodes_np[:, 0]), np.full(len(nodes_np), 0.5)], 1)
    stream = torch.cuda.current_stream()
    if warm:
        sdd.sdd_interface_estimate(ctx, dens, B, nodes, min(paths, 1024), dt, cfg["seed"], prec, exit_test=exit_test)
        torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    o = sdd.sdd_interface_estimate(ctx, dens, B, nodes, paths, dt, cfg["seed"], prec, exit_test=exit_test)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    m, se = o["mean"].cpu().numpy(), o["se"].cpu().numpy()
    steps = int(o["stats"].cpu().numpy()[0])
    err = m - exact
    return {"dt": dt, "walk": prec, "exit_test": exit_test, "ms": ms, "steps_per_s": steps / (ms / 1e3),
            "mean_steps_per_path": steps / (paths * len(nodes_np)),
            "max_abs_err_x": float(np.abs(err[:, 0]).max()), "mean_err_x": float(err[:, 0].mean()),
            "max_abs_err_y": float(np.abs(err[:, 1]).max()), "median_se": float(np.median(se)),
            "max_err_over_se": float(np.abs(err / se).max()), "_mean": m}


def bias_sweep(paths: int, dts, exit_tests=("step", "bridge")):
    """Bias of the exit point against the closed form of the w(xi) workload,
    float and double walks, for each time step and exit test."""
    import numpy as np

    import paper_1310_3435_amd as sdd
    ctx = sdd.Context(0)
    rows = []
    for et in exit_tests:
        for dt in dts:
            r32 = sin2_estimate(ctx, paths, dt, "fp32", et)
            r64 = sin2_estimate(ctx, paths, dt, "fp64", et)
            r64["max_diff_fp32_fp64"] = float(np.abs(r32["_mean"] - r64["_mean"]).max())
            for r in (r32, r64):
                r.pop("_mean")
                rows.append(r)
                print(json.dumps(r), flush=True)
    return rows


def bridge_legs(ctx, cfg, B, nodes, plain_walk_ms: float, plain_steps: int, plain_mean, sin2_paths: int):
    """The Brownian-bridge exit test: its cost on the throughput workload
    (same paths, fewer steps each) and the time to a given exit bias on the
    closed-form workload, against the end-of-step test at a 100x smaller
    time step."""
    import numpy as np
    import torch

    import paper_1310_3435_amd as sdd
    stream = torch.cuda.current_stream()
    o = sdd.sdd_interface_estimate(ctx, cfg["density"], B, nodes, cfg["paths"], cfg["dt"], cfg["seed"], cfg["prec"],
                                   exit_test="bridge")
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    o = sdd.sdd_interface_estimate(ctx, cfg["density"], B, nodes, cfg["paths"], cfg["dt"], cfg["seed"], cfg["prec"],
                                   exit_test="bridge", out=o)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    steps = int(o["stats"].cpu().numpy()[0])
    paths = int(o["stats"].cpu().numpy()[1])
    out = {"workload": cfg["name"], "walk_ms": ms, "walk_steps_per_s": steps / (ms / 1e3),
           "steps_per_path": steps / paths, "plain_steps_per_path": plain_steps / paths,
           "cost_per_step_vs_plain": (ms / steps) / (plain_walk_ms / plain_steps),
           "max_node_shift_vs_plain": float(np.abs(o["mean"].cpu().numpy() - plain_mean).max())}
    plain = sin2_estimate(ctx, sin2_paths, 1e-6, "fp32", "step")
    bridge = sin2_estimate(ctx, sin2_paths, 1e-4, "fp32", "bridge")
    for r in (plain, bridge):
        r.pop("_mean")
    out["equal_bias"] = {"workload": f"sin2_1d_closed_form, 64 nodes x {sin2_paths} paths, float walk",
                         "step_dt_1e-6": plain, "bridge_dt_1e-4": bridge,
                         "bridge_speedup": plain["ms"] / bridge["ms"],
                         "bridge_err_ratio": bridge["max_abs_err_x"] / plain["max_abs_err_x"]}
    return out


def quality_study(ctx, cfg, B, nodes, est_mean, dd_mesh):
    """Mesh quality of the domain-decomposition mesh against the single-domain
    finite-difference mesh of the same grid (Sec. 3.1-3.3: Q_max, Q_mean,
    R = Q/Q^S, l_inf), with Perona-Malik smoothing of both (Sec. 3.4, eq. (12);
    dt/h^2 as in the paper's 29 x 29 example, k = 1000) and interface
    pre-smoothing (Sec. 4).  Kernel times from HIP events."""
    import numpy as np
    import torch

    import paper_1310_3435_amd as sdd
    dens, L = cfg["density"], cfg["layout"]
    nx, ny = L["nx"], L["ny"]
    stream = torch.cuda.current_stream()

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        r = fn()
        b.record(stream)
        torch.cuda.synchronize()
        return r, a.elapsed_time(b)

    single = {"nx": nx, "ny": ny, "sx": 1, "sy": 1}

    def q(m):
        return sdd.sdd_mesh_quality(ctx, m)["out"].cpu().numpy()

    if nx * ny > 257 * 257:
        # one SOR block per component would need minutes on this grid: the
        # decomposition's own quality only
        qd = q(dd_mesh)
        return {"reference": None, "q_max_dd": float(qd[0]), "q_mean_dd": float(qd[1]), "folded_dd": int(qd[2])}
    ref_sol, ref_ms = timed(lambda: sdd.sdd_subdomain_solve(ctx, dens, B, single, None, None))
    ref = ref_sol["mesh"]

    def row(m_dd, m_ref):
        qd, qr = q(m_dd), q(m_ref)
        cmp = sdd.sdd_mesh_compare(ctx, dens, m_dd, m_ref).cpu().numpy()
        return {"q_max": float(qr[0]), "q_mean": float(qr[1]), "q_max_dd": float(qd[0]), "q_mean_dd": float(qd[1]),
                "r_max": float(qr[0] / qd[0]), "r_mean": float(qr[1] / qd[1]), "linf": float(cmp[0]),
                "max_disp": float(cmp[1]), "folded_dd": int(qd[2])}

    _, q_ms = timed(lambda: sdd.sdd_mesh_quality(ctx, dd_mesh))
    out = {"reference": f"single-domain finite-difference solve {nx}x{ny} (SOR, {int(ref_sol['sweeps'].max())} "
                        f"sweeps, {ref_ms:.1f} ms)",
           "quality_kernel_ms": q_ms, "no_smoothing": row(dd_mesh, ref)}
    dt = 1e-4 * 28**2 / ((nx - 1) ** 2)          # the paper's dt / h^2 on its 29 x 29 grid
    sm = {}
    for m in (1, 2, 5, 10):
        a, b = dd_mesh.clone(), ref.clone()
        _, ms = timed(lambda: sdd.sdd_mesh_smooth(ctx, L, a, dt, 1000.0, m, per_subdomain=True))
        sdd.sdd_mesh_smooth(ctx, single, b, dt, 1000.0, m, per_subdomain=False)
        sm[str(m)] = dict(row(a, b), smooth_ms=ms)
    out["perona_malik_per_subdomain"] = {"dt": dt, "k": 1000.0, "steps": sm}
    # a second cycle on the subdomains shifted by half their size (Sec. 4),
    # and the whole grid, each for 10 steps after 10 per-subdomain steps
    for name, mode in (("then_shifted_subdomains", "shifted"), ("then_whole_grid", False)):
        a, b = dd_mesh.clone(), ref.clone()
        sdd.sdd_mesh_smooth(ctx, L, a, dt, 1000.0, 10, per_subdomain=True)
        _, ms = timed(lambda: sdd.sdd_mesh_smooth(ctx, L, a, dt, 1000.0, 10, per_subdomain=mode))
        sdd.sdd_mesh_smooth(ctx, single, b, dt, 1000.0, 20, per_subdomain=False)
        out["perona_malik_per_subdomain"][name] = dict(row(a, b), smooth_ms=ms)
    vert, horiz = sdd.sdd_fill_interfaces(ctx, L, cfg["k"], B, nodes, est_mean, cfg.get("interp", "linear"))
    _, ls_ms = timed(lambda: sdd.sdd_smooth_interfaces(ctx, L, vert, horiz, 9))
    sol = sdd.sdd_subdomain_solve(ctx, dens, B, L, vert, horiz)
    out["interface_presmoothing_span9"] = dict(row(sol["mesh"], ref), smooth_ms=ls_ms)
    return out


def paper_study(ctx):
    """The kinds of study of the paper's Sec. 3 on a workload shaped like its
    running example (29 x 29 grid, Gaussian monitor function, four square
    subdomains): the mesh by Monte Carlo at every node with N = 1e3 and 1e4
    (Table 1: l_inf, Q^S_max, Q^S_mean, R_max, R_mean), Perona-Malik
    smoothing of the N = 1e3 mesh and of the reference for m = 1, 2, 5, 10
    steps with dt = 1e-4, k = 1000 (Table 2), the decomposition with every
    interface node by Monte Carlo (Sec. 3.5), with seven equidistant
    points per dividing line and with points at the extrema of w_s and w_ss
    (Sec. 3.6), linear fill.  Reference: the single-domain
    finite-difference mesh."""
    import torch

    import paper_1310_3435_amd as sdd
    import workloads

    cfg = workloads.cfg_paper_example()
    dens, L = cfg["density"], cfg["layout"]
    nx, ny = L["nx"], L["ny"]
    single = {"nx": nx, "ny": ny, "sx": 1, "sy": 1}
    B = sdd.Bmap(cfg["bmap"], ctx, dens)
    ref = sdd.sdd_subdomain_solve(ctx, dens, B, single, None, None)["mesh"]

    def row(m, r):
        qs = sdd.sdd_mesh_quality(ctx, m)["out"].cpu().numpy()
        qr = sdd.sdd_mesh_quality(ctx, r)["out"].cpu().numpy()
        c = sdd.sdd_mesh_compare(ctx, dens, m, r).cpu().numpy()
        return {"linf": float(c[0]), "q_max": float(qr[0]), "q_mean": float(qr[1]), "q_max_s": float(qs[0]),
                "q_mean_s": float(qs[1]), "r_max": float(qr[0] / qs[0]), "r_mean": float(qr[1] / qs[1]),
                "folded": int(qs[2])}

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) * 1e3

    out = {"workload": f"{cfg['name']}: {nx}x{ny}, 2x2 subdomains, bridge exits at dt {cfg['dt']:g}, float walks",
           "whole_grid": {}, "smoothing_n1000": {}, "decomposition": {}}
    prob = {}
    for n in (1000, 10000):
        r, ms = timed(lambda: sdd.run_probabilistic(ctx, dict(cfg, paths=n)))
        prob[n] = r["mesh"]
        out["whole_grid"][str(n)] = dict(row(r["mesh"], ref), ms=ms, nodes=int(r["nodes"].shape[0]))
    for m in (1, 2, 5, 10):
        a, b = prob[1000].clone(), ref.clone()
        sdd.sdd_mesh_smooth(ctx, single, a, 1e-4, 1000.0, m, per_subdomain=False)
        sdd.sdd_mesh_smooth(ctx, single, b, 1e-4, 1000.0, m, per_subdomain=False)
        out["smoothing_n1000"][str(m)] = row(a, b)
    r, ms = timed(lambda: sdd.run_pipeline(ctx, cfg))
    out["decomposition"]["all_interface_nodes"] = dict(row(r["mesh"], ref), ms=ms,
                                                       nodes=int(r["nodes"].shape[0]))
    r, ms = timed(lambda: sdd.run_pipeline(ctx, dict(cfg, k=3)))
    out["decomposition"]["seven_points_per_line"] = dict(row(r["mesh"], ref), ms=ms,
                                                         nodes=int(r["nodes"].shape[0]))
    r, ms = timed(lambda: sdd.run_pipeline(ctx, dict(cfg, k=8, placement="extrema")))
    out["decomposition"]["extrema_points"] = dict(row(r["mesh"], ref), ms=ms,
                                                  nodes=int((r["nodes"][:, 0] >= 0).sum().item()),
                                                  counts=r["counts"].cpu().numpy().tolist())
    return out


def walk_kind_name(cfg) -> str:
    terms = cfg["density"]["terms"]
    if all(t["kind"] == "gauss" for t in terms):
        return "gauss"
    return terms[0]["kind"] if len(terms) == 1 else "sum"


def roofline(cfg, steps_per_launch: int, walk_s: float, traffic):
    """The walk kernel against the FP32 vector peak (algorithmic flops per
    step x steps per launch / launch time), with the issue-cycle view and the
    algorithmic bytes beside it."""
    kind = walk_kind_name(cfg)
    n_nodes = cfg.get("_nodes", 0)
    out = {"bound": "alu", "unit": "TFLOP/s", "peak": FP32_PEAK_TFLOPS, "traffic": traffic,
           "kernel": "walk_kernel<%s, %s, end-of-step exit>" % ("float" if cfg["prec"] == "fp32" else "double",
                                                                 kind),
           "flops_per_step": FP32_FLOPS_PER_STEP.get(kind), "steps_per_launch": steps_per_launch,
           "launch_s": walk_s, "algorithmic_bytes_per_launch": n_nodes * WALK_BYTES_PER_NODE}
    if cfg["prec"] == "fp32" and kind in FP32_FLOPS_PER_STEP:
        tf = steps_per_launch * FP32_FLOPS_PER_STEP[kind] / walk_s / 1e12
        out.update(achieved=tf, frac=tf / FP32_PEAK_TFLOPS, frac_of_unpacked_78_6=tf / (FP32_PEAK_TFLOPS / 2))
        cyc = CYCLES_PER_WAVE_STEP[kind]
        g = steps_per_launch / 64 * cyc / walk_s / 1e9
        out["issue_model"] = {"cycles_per_wave_step": round(cyc, 2), "achieved_G_cycles_per_s": g,
                              "peak_G_cycles_per_s": ISSUE_PEAK_G, "frac": g / ISSUE_PEAK_G}
    else:
        out.update(achieved=None, frac=None)
    return out


def timed_estimate(ctx, dens, B, nodes, paths, dt, seed, prec, exit_test="step", out=None):
    """One estimate call timed with HIP events on torch's current stream
    (the stream its kernels run on); returns (result, ms)."""
    import torch

    import paper_1310_3435_amd as sdd
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    o = sdd.sdd_interface_estimate(ctx, dens, B, nodes, paths, dt, seed, prec, exit_test=exit_test, out=out)
    b.record(stream)
    torch.cuda.synchronize()
    return o, a.elapsed_time(b)


def ring_leg(ctx, oracle_paths: int, want_fp64: bool = True):
    """The ring workload (1521 nodes x 1e4 paths, dt = 1e-5): float walk rate
    and roofline, the double walk on the same paths (equal standard error),
    and its 64-node double-oracle subset node by node (oracle_paths paths)."""
    import numpy as np

    import paper_1310_3435_amd as sdd
    import workloads
    cfg = workloads.cfg_ring_fp32()
    dens, L = cfg["density"], cfg["layout"]
    B = sdd.Bmap(cfg["bmap"], ctx, dens)
    nodes = sdd.sdd_layout_nodes(ctx, L, cfg["k"], "uniform", dens)
    n = int(nodes.shape[0])
    cfg["_nodes"] = n
    est, _ = timed_estimate(ctx, dens, B, nodes, cfg["paths"], cfg["dt"], cfg["seed"], "fp32")
    ms = []
    for _ in range(3):
        est, t = timed_estimate(ctx, dens, B, nodes, cfg["paths"], cfg["dt"], cfg["seed"], "fp32", out=est)
        ms.append(t)
    st = sdd.walk_stats(est["stats"])
    walk_ms = float(np.median(ms))
    mean32, se32 = est["mean"].cpu().numpy(), est["se"].cpu().numpy()
    out = {"workload": cfg["name"], "nodes": n, "paths_per_node": cfg["paths"], "dt": cfg["dt"],
           "walk_ms": walk_ms, "walk_steps_per_s": st["steps"] / (walk_ms / 1e3),
           "interface_nodes_per_s": n / (walk_ms / 1e3), "median_se": float(np.median(se32)),
           "t_stoc_ms_device": st["t_stoc_ms"],
           "roofline": roofline(cfg, st["steps"], walk_ms / 1e3, traffic_from_profile(cfg["name"]))}
    if want_fp64:
        e64, _ = timed_estimate(ctx, dens, B, nodes, cfg["paths"], cfg["dt"], cfg["seed"], "fp64")
        e64, ms64 = timed_estimate(ctx, dens, B, nodes, cfg["paths"], cfg["dt"], cfg["seed"], "fp64", out=e64)
        st64 = sdd.walk_stats(e64["stats"])
        d = np.abs(e64["mean"].cpu().numpy() - mean32)
        z = d / np.maximum(e64["se"].cpu().numpy(), 1e-300)
        q = lambda a: {"p50": float(np.percentile(a, 50)), "p99": float(np.percentile(a, 99)), "max": float(a.max())}
        out["fp64_walk"] = {"walk_ms": ms64, "walk_steps_per_s": st64["steps"] / (ms64 / 1e3),
                            "median_se": float(np.median(e64["se"].cpu().numpy())),
                            "fp32_speedup_at_equal_se": ms64 / walk_ms,
                            "node_diff_fp32_vs_fp64": q(d), "node_diff_over_se": q(z)}
    if oracle_paths > 0:
        import oracle
        idx = np.arange(64) * (n // 64)
        g, _ = timed_estimate(ctx, dens, B, nodes, oracle_paths, cfg["dt"], cfg["seed"], "fp32")
        gm = g["mean"].cpu().numpy()[idx]
        t0 = time.perf_counter()
        r = oracle.interface_estimate(dens, cfg["bmap"], nodes.cpu().numpy()[idx], oracle_paths, cfg["dt"],
                                      cfg["seed"], "fp64", node_ids=idx, nthreads=host_threads())
        el = time.perf_counter() - t0
        z = np.abs(gm - r["mean"]) / r["se"]
        out["oracle_subset_64"] = {"nodes": "list indices i*%d, i = 0..63" % (n // 64), "paths_per_node": oracle_paths,
                                   "oracle_s": el, "abs_diff_over_se_max": float(z.max()),
                                   "abs_diff_over_se_p50": float(np.median(z)),
                                   "max_abs_diff": float(np.abs(gm - r["mean"]).max()),
                                   "all_within_3_se": bool(np.all(z <= 3.0))}
    out["_keep"] = (cfg, B, nodes, walk_ms, st["steps"], mean32)
    return out


def expo_legs(ctx, paths: int):
    """Exponential time stepping (mean step dt) against the bridge and the
    end-of-step test at the same dt on the closed-form workload: error
    against the closed form, steps per path and time."""
    rows = []
    for dt in (1e-3, 1e-4):
        for et in ("expo", "bridge", "step"):
            r = sin2_estimate(ctx, paths, dt, "fp32", et)
            r.pop("_mean")
            rows.append(r)
    return {"workload": f"sin2_1d_closed_form, 64 nodes x {paths} paths, float walk", "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="annulus_fp32_8x8x129")
    ap.add_argument("--prec", default=None, help="override the workload's walk precision")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-nodes", type=int, default=8)
    ap.add_argument("--cpu-sample-paths", type=int, default=25000,
                    help="paths per sampled node of the oracle baseline (about 15 s on 16 host cores)")
    ap.add_argument("--no-ring", action="store_true", help="skip the ring workload leg")
    ap.add_argument("--ring-oracle-paths", type=int, default=2000,
                    help="paths per node of the ring workload's 64-node oracle subset (0: skip)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the double-precision comparison walk")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests in the serving stream (0: skip)")
    ap.add_argument("--serve-load", type=float, default=0.8, help="arrival rate / measured capacity")
    ap.add_argument("--serve-burst", type=int, default=32, help="requests of the capacity burst")
    ap.add_argument("--serve-sweep", default="", metavar="LOADS",
                    help="only run the serving stream at each load in LOADS (e.g. 0.5,0.8,1.0), one line each")
    ap.add_argument("--serve-launch-paths", type=int, default=0,
                    help="paths per serving walk launch (0: the server's default)")
    ap.add_argument("--serve-bridge-dt", type=float, default=1e-3,
                    help="> 0: serving requests use the bridge exit test at this time step (0: end of step, 1e-4)")
    ap.add_argument("--serve-like", action="store_true",
                    help="only run one request through the server and through the estimate call (same paths)")
    ap.add_argument("--bias-sweep", action="store_true",
                    help="only run the float/double dt sweep of the closed-form workload")
    ap.add_argument("--sweep-paths", type=int, default=1000000)
    ap.add_argument("--sweep-dts", default="1e-3,1e-4,1e-5,1e-6")
    ap.add_argument("--sweep-exit", default="step,bridge,expo", help="exit tests of the sweep")
    ap.add_argument("--no-quality", action="store_true", help="skip the mesh-quality study")
    ap.add_argument("--bridge-paths", type=int, default=1000000,
                    help="paths per node of the equal-bias comparison (0: skip the bridge legs)")
    ap.add_argument("--expo-paths", type=int, default=200000,
                    help="paths per node of the exponential-stepping legs (0: skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes (counter calibration)")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}), flush=True)
        return

    if args.bias_sweep:
        rows = bias_sweep(args.sweep_paths, [float(v) for v in args.sweep_dts.split(",")],
                          tuple(args.sweep_exit.split(",")))
        print(json.dumps({"bias_sweep": rows, "paths_per_node": args.sweep_paths, "nodes": 64,
                          "workload": "sin2_bias_sweep"}), flush=True)
        return

    if args.serve_like:
        import paper_1310_3435_amd as sdd
        print(json.dumps({"serve_like": serve_like(sdd.Context(0))}), flush=True)
        return

    if args.serve_sweep:
        import paper_1310_3435_amd as sdd
        ctx = sdd.Context(0)
        for load in (float(v) for v in args.serve_sweep.split(",")):
            r = serve_stream(ctx, args.serve_requests, load, args.serve_burst, bridge_dt=args.serve_bridge_dt,
                             launch_paths=args.serve_launch_paths)
            print(json.dumps({"serve": r}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(nodes and requests would shard across GPUs, one process each)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1310_3435_amd as sdd
    import workloads

    cfg = workloads.CONFIGS[args.workload]()
    if args.prec:
        cfg["prec"] = args.prec
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = sdd.Context(0)
    stream = torch.cuda.current_stream()
    dens, L = cfg["density"], cfg["layout"]
    B = sdd.Bmap(cfg["bmap"], ctx, dens)
    nodes = sdd.sdd_layout_nodes(ctx, L, cfg["k"], cfg.get("placement", "uniform"), dens)
    n = nodes.shape[0]
    cfg["_nodes"] = n
    est = None
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    interp = cfg.get("interp", "linear")

    def step(i=None):
        nonlocal est
        if i is not None:
            ev[i][0].record(stream)
        est = sdd.sdd_interface_estimate(ctx, dens, B, nodes, cfg["paths"], cfg["dt"], cfg["seed"], cfg["prec"],
                                         out=est)
        if i is not None:
            ev[i][1].record(stream)
        vert, horiz = sdd.sdd_fill_interfaces(ctx, L, cfg["k"], B, nodes, est["mean"], interp)
        return sdd.sdd_subdomain_solve(ctx, dens, B, L, vert, horiz)

    print(f"[bench] {cfg['name']}: {n} nodes x {cfg['paths']} paths, {args.warmup} warmup + {args.steps} timed passes",
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        sol = step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    st = sdd.walk_stats(est["stats"])
    steps_per_pass = int(st["steps"])
    walk_ms = [a.elapsed_time(b) for a, b in ev]
    walk_avg_s = float(np.mean(walk_ms)) / 1e3
    se = est["se"].cpu().numpy()
    sweeps = sol["sweeps"].cpu().numpy()
    mesh = sol["mesh"].cpu().numpy()
    assert np.all(np.isfinite(mesh)), "non-finite mesh"

    total_steps = steps_per_pass * args.steps
    value = total_steps / elapsed
    line = {
        "metric": "walk steps/s + interface nodes/s at fixed std error; serve p50/p99 latency",
        "value": value,
        "unit": "walk steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if cfg["prec"] == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": cfg["name"], "nodes": int(n), "paths_per_node": cfg["paths"], "dt": cfg["dt"],
            "layout": f"{L['nx']}x{L['ny']} nodes, {L['sx']}x{L['sy']} subdomains",
            "walk_precision": cfg["prec"] + " steps, f64 exit projection, exact node sums",
            "parallelism": "single GPU",
        },
        "interface_nodes_per_s": n * args.steps / elapsed,
        "median_se": float(np.median(se)),
        "walk_steps_per_pass": steps_per_pass,
        "walk_ms": float(np.mean(walk_ms)),
        "stage_ms": {"t_stoc_device_clock": st["t_stoc_ms"],
                     "t_fill_plus_sub": elapsed / args.steps * 1e3 - float(np.mean(walk_ms))},
        "fd_sweeps_max": int(sweeps.max()),
        "roofline": roofline(cfg, steps_per_pass, walk_avg_s, traffic_from_profile(args.workload)),
    }
    print(f"[bench] timed: {value:.3e} walk steps/s, {line['ms_per_step']:.1f} ms/pass", file=sys.stderr, flush=True)
    ring = None
    if not args.no_ring:
        print("[bench] ring workload leg", file=sys.stderr, flush=True)
        ring = ring_leg(ctx, args.ring_oracle_paths, not args.no_fp64)
        line["ring"] = {k: v for k, v in ring.items() if not k.startswith("_")}
    if not args.no_quality:
        print("[bench] quality studies", file=sys.stderr, flush=True)
        line["quality"] = quality_study(ctx, cfg, B, nodes, est["mean"], sol["mesh"])
        line["paper_example"] = paper_study(ctx)
    if args.bridge_paths > 0 and ring is not None:
        print("[bench] bridge legs", file=sys.stderr, flush=True)
        rc, rB, rnodes, rms, rsteps, rmean = ring["_keep"]
        line["bridge"] = bridge_legs(ctx, rc, rB, rnodes, rms, rsteps, rmean, args.bridge_paths)
    if args.expo_paths > 0:
        print("[bench] exponential stepping legs", file=sys.stderr, flush=True)
        line["expo"] = expo_legs(ctx, args.expo_paths)
    if args.serve_requests > 0:
        print(f"[bench] serving stream of {args.serve_requests} requests", file=sys.stderr, flush=True)
        line["serve"] = serve_stream(ctx, args.serve_requests, args.serve_load, args.serve_burst,
                                     bridge_dt=args.serve_bridge_dt, launch_paths=args.serve_launch_paths)
        line["serve"]["like_for_like"] = serve_like(ctx)
    if not args.no_cpu_baseline:
        # the same first paths of every node on the GPU, for the per-node comparison
        sp = min(args.cpu_sample_paths, cfg["paths"])
        g, _ = timed_estimate(ctx, dens, B, nodes, sp, cfg["dt"], cfg["seed"], cfg["prec"])
        print("[bench] oracle baseline on the host", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(cfg, nodes.cpu().numpy(), args.cpu_sample_nodes, steps_per_pass,
                                            gpu_mean=g["mean"].cpu().numpy(), sample_paths=sp)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
