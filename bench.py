"""Throughput benchmark of the interface Monte Carlo hot path on one MI355X.

One step = one pass of the whole path over the workload: interface
estimate (walk + finalize), interface fill and the batched subdomain
solves, all on the GPU, inputs already resident in HBM.  Prints one JSON
line.

Default workload: ring density w = 1 + 10 exp(-200 (r - 0.3)^2), identity
boundary map, 4 x 4 subdomains of 65 x 65 nodes (global 257 x 257), every
interior interface node estimated (1521 nodes), 1e4 paths per node,
dt = 1e-5, float walk with compensated double accumulation.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU issue model of one float Euler-Maruyama step with the ring density
# (lane-slots; an op of the transcendental unit or a 32x32-bit integer
# multiply occupies 4 slots, every other VALU op 1).  Derivation in the
# design notes; the peak is 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
SLOTS_PER_STEP = {"ring": 115, "gauss": 98, "sech2": 108, "sin2": 106}
VALU_PEAK_TSLOTS = 256 * 4 * 16 * 2.4e9 / 1e12  # 39.3 T lane-slots/s
FP32_FLOPS_PER_STEP = {"ring": 38, "gauss": 34, "sech2": 40, "sin2": 36}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("walk.hip", "common.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_1310_3435_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
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


def cpu_baseline(cfg, nodes, sample_nodes: int):
    """The oracle, untuned, on this host's cores: `sample_nodes` evenly spaced
    nodes of the same workload at its full paths per node, double precision."""
    import numpy as np

    import oracle
    oracle.lib()
    n = nodes.shape[0]
    idx = (np.arange(sample_nodes) * (n // sample_nodes)).astype(np.int64)
    threads = os.cpu_count() or 1
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    t0 = time.perf_counter()
    r = oracle.interface_estimate(cfg["density"], cfg["bmap"], nodes[idx], cfg["paths"], cfg["dt"], cfg["seed"],
                                  "fp64", node_ids=idx, nthreads=threads)
    el = time.perf_counter() - t0
    return {"value": r["steps"] / el, "unit": "walk steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample_nodes} of {n} nodes (indices i*{n // sample_nodes}), {cfg['paths']} paths/node, "
                      f"dt={cfg['dt']}, fp64 walk, {r['steps']} steps in {el:.2f} s",
            "nodes_per_s": sample_nodes / el}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ring_fp32_4x4x65")
    ap.add_argument("--prec", default=None, help="override the workload's walk precision")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-nodes", type=int, default=64)
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

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(see the sharding notes in DESIGN.md)", file=sys.stderr)
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
    est = None
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]

    def step(i=None):
        nonlocal est
        if i is not None:
            ev[i][0].record(stream)
        est = sdd.sdd_interface_estimate(ctx, dens, B, nodes, cfg["paths"], cfg["dt"], cfg["seed"], cfg["prec"],
                                         out=est)
        if i is not None:
            ev[i][1].record(stream)
        vert, horiz = sdd.sdd_fill_interfaces(ctx, L, cfg["k"], B, nodes, est["mean"], cfg.get("interp", "linear"))
        return sdd.sdd_subdomain_solve(ctx, dens, B, L, vert, horiz)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        sol = step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    stats = est["stats"].cpu().numpy()
    steps_per_pass = int(stats[0])
    walk_ms = [a.elapsed_time(b) for a, b in ev]
    walk_avg_s = float(np.mean(walk_ms)) / 1e3
    se = est["se"].cpu().numpy()
    sweeps = sol["sweeps"].cpu().numpy()
    mesh = sol["mesh"].cpu().numpy()
    assert np.all(np.isfinite(mesh)), "non-finite mesh"

    total_steps = steps_per_pass * args.steps
    value = total_steps / elapsed
    kind = dens["terms"][0]["kind"] if dens["terms"] else "gauss"
    slots = SLOTS_PER_STEP.get(kind, 100)
    achieved = steps_per_pass * slots / walk_avg_s / 1e12
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
            "workload": cfg["name"], "nodes": n, "paths_per_node": cfg["paths"], "dt": cfg["dt"],
            "layout": f"{L['nx']}x{L['ny']} nodes, {L['sx']}x{L['sy']} subdomains",
            "walk_precision": cfg["prec"] + " steps, f64 exit projection and sums",
            "parallelism": "single GPU",
        },
        "interface_nodes_per_s": n * args.steps / elapsed,
        "median_se": float(np.median(se)),
        "walk_steps_per_pass": steps_per_pass,
        "walk_ms": float(np.mean(walk_ms)),
        "fd_sweeps_max": int(sweeps.max()),
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": VALU_PEAK_TSLOTS,
            "unit": "T VALU lane-slots/s",
            "frac": achieved / VALU_PEAK_TSLOTS,
            "traffic": traffic_from_profile(args.workload),
            "kernel": "walk_kernel<float>" if cfg["prec"] == "fp32" else "walk_kernel<double>",
            "slots_per_step": slots,
            "fp32_tflops": steps_per_pass * FP32_FLOPS_PER_STEP.get(kind, 34) / walk_avg_s / 1e12,
        },
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, nodes.cpu().numpy(), args.cpu_sample_nodes)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
