"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
bring results to the host; compare per-path records with the oracle's."""
import sys

import numpy as np


def say(msg: str):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def gpu_estimate(ctx, density, bmap, nodes, paths, dt, seed, prec="fp64", per_path=False, **kw):
    import torch

    import paper_1310_3435_amd as sdd
    nodes = np.ascontiguousarray(nodes, dtype=np.float64).reshape(-1, 2)
    say(f"interface_estimate n={nodes.shape[0]} N={paths} dt={dt} seed={seed} prec={prec} per_path={per_path}")
    t = torch.as_tensor(nodes).cuda()
    o = sdd.sdd_interface_estimate(ctx, density, bmap, t, paths, dt, seed, prec, per_path=per_path,
                                   want_sums=True, **kw)
    torch.cuda.synchronize()
    out = {"mean": o["mean"].cpu().numpy(), "se": o["se"].cpu().numpy(), "sums": o["sums"].cpu().numpy()}
    st = o["stats"].cpu().numpy()
    out.update(steps=int(st[0]), paths=int(st[1]), capped=int(st[2]))
    if per_path:
        out["per_path"] = sdd.path_records(o["per_path"])
    return out


def compare_paths(gpu_rec, ref_rec, tol):
    """Per-path comparison.  Returns (flip_mask, max exit-point difference on
    paths whose exit step agrees)."""
    same = gpu_rec["steps"] == ref_rec["steps"]
    dx = np.abs(gpu_rec["exit_xi"] - ref_rec["exit_xi"])
    dy = np.abs(gpu_rec["exit_eta"] - ref_rec["exit_eta"])
    d = np.where(same, np.maximum(dx, dy), 0.0)
    return ~same, float(d.max()) if d.size else 0.0
