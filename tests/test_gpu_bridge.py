"""GPU parity of the walk with the Brownian-bridge exit test (Sec. 2.2, the
conditional exit probability within a step) against the oracle's bridge
walk, under the same Philox counters.

Bars as for the end-of-step walk: double precision per path (equal exit
steps and sides up to counted roundoff flips, exit points within 1e-12);
float per path up to rare flips, and node estimates within 3 standard errors
of the double-precision oracle.
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


@pytest.mark.parametrize("dt", [1e-3, 1e-4])
def test_fp64_bridge_paths_match_oracle(ctx, ref, dt):
    c = W.cfg_plain_fp64()
    nodes = ref.layout_nodes(c["layout"], c["k"])
    g = gpu_estimate(ctx, c["density"], c["bmap"], nodes, c["paths"], dt, c["seed"], "fp64", per_path=True,
                     exit_test="bridge")
    r = ref.interface_estimate(c["density"], c["bmap"], nodes, c["paths"], dt, c["seed"], per_path=True,
                               bridge=True)
    plain = ref.interface_estimate(c["density"], c["bmap"], nodes, c["paths"], dt, c["seed"], per_path=True)
    flips, dmax = compare_paths(g["per_path"], r["per_path"], 1e-12)
    shorter = (r["per_path"]["steps"] < plain["per_path"]["steps"]).mean()
    say(f"bridge fp64 dt={dt}: flips {int(flips.sum())} of {flips.size}, max exit diff {dmax:.3e}, "
        f"paths the bridge shortened {shorter:.3f}")
    assert shorter > 0.1          # the bridge decided many exits here
    assert flips.sum() <= max(1, flips.size // 10000)
    assert dmax <= 1e-12
    assert np.array_equal(g["per_path"]["side"][~flips], r["per_path"]["side"][~flips])
    ok = ~flips.any(axis=1)
    assert ok.sum() >= len(ok) - 1
    assert np.max(np.abs(g["mean"][ok] - r["mean"][ok])) <= 1e-10
    assert np.max(np.abs(g["se"][ok] - r["se"][ok])) <= 1e-10
    assert g["paths"] == r["paths"] and g["capped"] == r["capped"] == 0


@pytest.mark.parametrize("bm", [
    {"kind": "identity"},
    {"kind": "annulus", "p": [1.0, 2.0, 0.0, 0.5 * math.pi]},
    {"kind": "edge1d", "n_per_edge": 1025},
], ids=["identity", "annulus", "edge1d"])
def test_fp64_bridge_all_terms_and_maps(ctx, ref, bm):
    d = W.random_density(6, 4)
    nodes = W.random_nodes(24, 106)
    g = gpu_estimate(ctx, d, bm, nodes, 300, 2e-3, 1006, "fp64", per_path=True, exit_test="bridge")
    r = ref.interface_estimate(d, bm, nodes, 300, 2e-3, 1006, per_path=True, bridge=True)
    flips, dmax = compare_paths(g["per_path"], r["per_path"], 1e-12)
    say(f"bridge {bm['kind']}: flips {int(flips.sum())}, max exit diff {dmax:.3e}")
    assert flips.sum() <= 1
    assert dmax <= 1e-12
    ok = ~flips.any(axis=1)
    assert np.max(np.abs(g["mean"][ok] - r["mean"][ok])) <= 1e-10


def test_fp32_bridge_matches_oracle_float_and_double(ctx, ref):
    c = W.cfg_plain_fp64()
    nodes = ref.layout_nodes(c["layout"], c["k"])
    dt = 1e-3
    g = gpu_estimate(ctx, c["density"], c["bmap"], nodes, c["paths"], dt, c["seed"], "fp32", per_path=True,
                     exit_test="bridge")
    r32 = ref.interface_estimate(c["density"], c["bmap"], nodes, c["paths"], dt, c["seed"], "fp32",
                                 per_path=True, bridge=True)
    r64 = ref.interface_estimate(c["density"], c["bmap"], nodes, c["paths"], dt, c["seed"], bridge=True)
    flips, dmax = compare_paths(g["per_path"], r32["per_path"], 1e-5)
    gp, rp = g["per_path"], r32["per_path"]
    d = np.maximum(np.abs(gp["exit_xi"] - rp["exit_xi"]), np.abs(gp["exit_eta"] - rp["exit_eta"]))[~flips]
    q = np.percentile(d, [50, 99])
    say(f"bridge fp32 vs oracle fp32: flips {int(flips.sum())} of {flips.size}; p50 {q[0]:.2e} p99 {q[1]:.2e} "
        f"max {dmax:.2e}")
    assert flips.mean() < 2e-3
    assert q[1] < 1e-5 and dmax < 1e-2
    z = np.abs(g["mean"] - r64["mean"]) / r64["se"]
    say(f"bridge fp32 vs fp64 oracle: max z {z.max():.3f}")
    assert np.all(z <= 3.0)
    assert np.all(np.abs(g["mean"] - r32["mean"]) <= 0.5 * r32["se"])


def test_bridge_with_step_cap(ctx, ref):
    d = {"base": 1.0, "terms": []}
    nodes = np.array([[0.5, 0.5], [0.3, 0.6]])
    for prec in ("fp64", "fp32"):
        g = gpu_estimate(ctx, d, {"kind": "identity"}, nodes, 500, 1e-3, 4, prec, per_path=True, t_max=0.005,
                         exit_test="bridge")
        r = ref.interface_estimate(d, {"kind": "identity"}, nodes, 500, 1e-3, 4, prec, t_max=0.005, per_path=True,
                                   bridge=True)
        say(f"bridge cap {prec}: capped {g['capped']} oracle {r['capped']}")
        assert g["capped"] == r["capped"] > 0
        assert np.array_equal(g["per_path"]["capped"], r["per_path"]["capped"])
        assert np.all(g["per_path"]["steps"] <= 6)


def test_full_size_ring_with_bridge_sampled_nodes(ctx, ref):
    """The ring workload at full size (1521 nodes x 1e4 paths, dt=1e-5, float)
    with the bridge test; sampled nodes against the double oracle."""
    c = W.cfg_ring_fp32()
    nodes = ref.layout_nodes(c["layout"], c["k"])
    g = gpu_estimate(ctx, c["density"], c["bmap"], nodes, c["paths"], c["dt"], c["seed"], "fp32",
                     exit_test="bridge")
    assert np.all(np.isfinite(g["mean"])) and g["capped"] == 0
    sample = np.array([0, 400, 1100, 1520])
    say(f"oracle fp64 bridge on {len(sample)} sampled nodes")
    r = ref.interface_estimate(c["density"], c["bmap"], nodes[sample], c["paths"], c["dt"], c["seed"],
                               node_ids=sample, bridge=True)
    z = np.abs(g["mean"][sample] - r["mean"]) / r["se"]
    say(f"ring bridge fp32 vs fp64 oracle: max z {z.max():.3f}")
    assert np.all(z <= 3.0)


def test_bad_exit_test_is_rejected(ctx):
    import ctypes as C

    import torch

    import paper_1310_3435_amd as sdd
    nodes = torch.tensor([[0.5, 0.5]], dtype=torch.float64, device="cuda")
    D = sdd.make_density({"base": 1.0, "terms": []})
    B = sdd.Bmap({"kind": "identity"}, ctx)
    mean = torch.empty((1, 2), dtype=torch.float64, device="cuda")
    ws = ctx.workspace(sdd.sdd_workspace_bytes(1, 4, "fp64"))
    for bad in (3, -1):   # 0, 1, 2: end of step, bridge, exponential stepping
        rc = sdd.lib().sdd_interface_estimate(ctx.h, C.byref(D), C.byref(B.s), nodes.data_ptr(), 1, 4, 0, 1e-3,
                                              C.c_uint64(1), 0, 8.0, bad, mean.data_ptr(), None, None, None, None,
                                              ws.data_ptr(), ws.numel(), None)
        assert rc == sdd.SDD_EINVAL
