"""GPU parity of the float walks the workloads run, against the oracle.

* The closed-form workload's kernel (w = 1 + 3 sin^2(2 pi xi), 1D edge data):
  the float walk at small steps (the pipelined Philox loop, dt < 2e-5) and at
  dt = 1e-4 (the plain loop), with and without the bridge, path by path
  against the oracle's float walk; and a sample of its 64 nodes at
  dt = 1e-5 and 1e-6 within 3 standard errors of the double oracle.
* The general sum of terms (every kind mixed), uncapped, path by path.
* The ring workload's 64-node subset (node indices i * floor(1521/64)),
  node by node against the double oracle.
* The curved workload's interface fill (14 224 points) and its 64 subdomain
  solves of 129 x 129 at full size, fed the same node values on both sides.

Bars: float per-path exit points p99 <= 1e-5 with a flip rate (paths whose
exit step differs) below 2e-3, max <= 1e-3 on the rest; node estimates within 3 SE of the
double oracle (common random numbers: the same uniforms drive both walks).
"""
import math

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import compare_paths, gpu_estimate, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1310_3435_amd as sdd
    return sdd.Context(0)


def _float_paths_agree(g, r, what):
    gp, rp = g["per_path"], r["per_path"]
    flips, dmax = compare_paths(gp, rp, 1e-5)
    same = ~flips
    d = np.maximum(np.abs(gp["exit_xi"] - rp["exit_xi"]), np.abs(gp["exit_eta"] - rp["exit_eta"]))[same]
    q = np.percentile(d, [50, 99]) if d.size else np.zeros(2)
    say(f"{what}: flips {int(flips.sum())} of {flips.size}; exit diff p50 {q[0]:.2e} p99 {q[1]:.2e} "
        f"max {dmax:.2e}")
    assert flips.mean() < 2e-3
    assert q[1] <= 1e-5 and dmax <= 1e-3
    return flips


def _sin2():
    c = W.cfg_sin2_sweep()
    return c, np.array(c["nodes"])


@pytest.mark.parametrize("exit_test", ["step", "bridge"])
@pytest.mark.parametrize("dt", [1e-5, 1e-4])
def test_sin2_float_walk_paths_match_oracle(ctx, ref, dt, exit_test):
    """Nodes across the closed-form workload (both ends and the middle) with
    a cap of 501 steps at dt = 1e-5 and uncapped at 1e-4."""
    c, allnodes = _sin2()
    nodes = allnodes[[0, 5, 20, 31, 44, 63]]
    t_max = 5.01e-3 if dt < 2e-5 else 8.0
    N = 400
    g = gpu_estimate(ctx, c["density"], c["bmap"], nodes, N, dt, c["seed"], "fp32", per_path=True, t_max=t_max,
                     exit_test=exit_test)
    r = ref.interface_estimate(c["density"], ref.Bmap(c["bmap"], c["density"]), nodes, N, dt, c["seed"], "fp32",
                               per_path=True, t_max=t_max, exit_test=exit_test)
    flips = _float_paths_agree(g, r, f"sin2 fp32 dt={dt:g} {exit_test}")
    assert g["capped"] == r["capped"] and (dt < 2e-5) == (g["capped"] > 0)
    if dt >= 2e-5:
        r64 = ref.interface_estimate(c["density"], ref.Bmap(c["bmap"], c["density"]), nodes, N, dt, c["seed"],
                                     per_path=False, exit_test=exit_test)
        z = np.abs(g["mean"] - r64["mean"]) / np.maximum(r64["se"], 1e-300)
        say(f"  vs fp64 oracle: max |diff|/SE {z.max():.3f}")
        assert np.all(z <= 3.0)


@pytest.mark.parametrize("dt,N", [(1e-5, 2000), (1e-6, 400)])
def test_sin2_sample_nodes_within_3se_of_double_oracle(ctx, ref, dt, N):
    """Eight of the closed-form workload's 64 nodes at its small steps,
    uncapped, the float walk in the launch configuration its sweep uses,
    against the double oracle on the same paths."""
    c, allnodes = _sin2()
    idx = np.arange(0, 64, 8)
    nodes = allnodes[idx]
    g = gpu_estimate(ctx, c["density"], c["bmap"], nodes, N, dt, c["seed"], "fp32")
    say(f"oracle fp64 on 8 nodes x {N} paths at dt={dt:g}")
    r = ref.interface_estimate(c["density"], ref.Bmap(c["bmap"], c["density"]), nodes, N, dt, c["seed"],
                               node_ids=None)
    z = np.abs(g["mean"] - r["mean"]) / r["se"]
    say(f"sin2 fp32 dt={dt:g}: max |diff|/SE {z.max():.4f}, max |diff| {np.abs(g['mean'] - r['mean']).max():.2e}")
    assert np.all(z <= 3.0)
    assert g["capped"] == r["capped"] == 0


@pytest.mark.parametrize("dseed", [3, 6, 9])
def test_general_sum_float_walk_uncapped(ctx, ref, dseed):
    d = W.random_density(dseed, 4)
    nodes = W.random_nodes(24, dseed + 200)
    g = gpu_estimate(ctx, d, {"kind": "identity"}, nodes, 300, 1e-3, 500 + dseed, "fp32", per_path=True)
    r = ref.interface_estimate(d, {"kind": "identity"}, nodes, 300, 1e-3, 500 + dseed, "fp32", per_path=True)
    _float_paths_agree(g, r, f"sum of 4 terms d{dseed} fp32")
    assert g["capped"] == 0
    r64 = ref.interface_estimate(d, {"kind": "identity"}, nodes, 300, 1e-3, 500 + dseed)
    z = np.abs(g["mean"] - r64["mean"]) / np.maximum(r64["se"], 1e-300)
    assert np.all(z <= 3.0)


def test_ring_workload_64_node_subset_against_double_oracle(ctx, ref):
    """The ring workload's double-oracle subset (64 nodes at list indices
    i * floor(1521/64)), node by node, at dt = 1e-5 with 1000 paths per
    node (the full 1e4 in the benchmark's baseline leg)."""
    c = W.cfg_ring_fp32()
    allnodes = ref.layout_nodes(c["layout"], c["k"])
    n = allnodes.shape[0]
    idx = np.arange(64) * (n // 64)
    N = 1000
    g = gpu_estimate(ctx, c["density"], c["bmap"], allnodes, N, c["dt"], c["seed"], "fp32")
    say(f"oracle fp64 on the 64-node subset x {N} paths")
    r = ref.interface_estimate(c["density"], c["bmap"], allnodes[idx], N, c["dt"], c["seed"], node_ids=idx)
    z = np.abs(g["mean"][idx] - r["mean"]) / r["se"]
    say(f"ring subset: |diff|/SE p50 {np.median(z):.4f} max {z.max():.4f}")
    assert np.all(z <= 3.0)
    # common random numbers: the float and double estimates differ far less than their SE
    assert np.median(z) < 0.05


def test_curved_workload_fill_and_solves_at_full_size(ctx, ref):
    """The 1025 x 1025 layout (8 x 8 subdomains of 129 x 129, 3633
    equidistributed points, monotone cubic fill of 14 224 interface points):
    the GPU's fill and 64 subdomain solves against the oracle's fill and
    direct solves, both fed the same node values (a short float walk)."""
    import torch

    import paper_1310_3435_amd as sdd
    c = W.cfg_annulus_fp32()
    L = c["layout"]
    B = sdd.Bmap(c["bmap"], ctx, c["density"])
    nodes = sdd.sdd_layout_nodes(ctx, L, c["k"], c["placement"], c["density"])
    assert nodes.shape[0] == 3633
    est = sdd.sdd_interface_estimate(ctx, c["density"], B, nodes, 256, 1e-4, c["seed"], "fp32")
    vert, horiz = sdd.sdd_fill_interfaces(ctx, L, c["k"], B, nodes, est["mean"], "pchip")
    sol = sdd.sdd_subdomain_solve(ctx, c["density"], B, L, vert, horiz)
    torch.cuda.synchronize()
    mean = est["mean"].cpu().numpy()
    nodes_h = nodes.cpu().numpy()
    say("oracle fill and 64 direct solves at 1025 x 1025")
    rv, rh = ref.fill_interfaces(L, c["k"], ref.Bmap(c["bmap"], c["density"]), nodes_h, mean, "pchip")
    dv = max(np.abs(vert.cpu().numpy() - rv).max(), np.abs(horiz.cpu().numpy() - rh).max())
    say(f"fill: max |diff| {dv:.2e} over {rv.shape[0] * rv.shape[1] + rh.shape[0] * rh.shape[1]} points")
    assert dv <= 1e-13
    mesh = ref.subdomain_solve(c["density"], ref.Bmap(c["bmap"], c["density"]), L, vert.cpu().numpy(),
                               horiz.cpu().numpy())
    dm = np.abs(sol["mesh"].cpu().numpy() - mesh).max()
    say(f"solves: max |diff| {dm:.2e}, sweeps {int(sol['sweeps'].max())}")
    assert dm <= 1e-9
