"""GPU parity of the interface walk against the CPU oracle (same Philox
counters, so individual paths are compared).

Bars:
* double precision: per-path exit points within 1e-12, equal exit steps
  except roundoff flips (counted; expected ~0), node means and standard
  errors within 1e-10 on flip-free nodes;
* float stepping: per-path agreement with the oracle's float walk except
  rare flips, and node estimates within 3 standard errors of the
  double-precision oracle (they share the uniforms, so the difference
  isolates precision effects).
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


def _flip_free_nodes(flips):
    return ~flips.any(axis=1)


def test_fp64_paths_match_oracle_on_the_small_workload(ctx, ref):
    c = W.cfg_plain_fp64()
    nodes = ref.layout_nodes(c["layout"], c["k"])
    g = gpu_estimate(ctx, c["density"], c["bmap"], nodes, c["paths"], c["dt"], c["seed"], "fp64", per_path=True)
    r = ref.interface_estimate(c["density"], c["bmap"], nodes, c["paths"], c["dt"], c["seed"], per_path=True)
    flips, dmax = compare_paths(g["per_path"], r["per_path"], 1e-12)
    say(f"fp64 flips {int(flips.sum())} of {flips.size}, max exit diff {dmax:.3e}")
    assert flips.sum() <= max(1, flips.size // 10000)
    assert dmax <= 1e-12
    ok = _flip_free_nodes(flips)
    assert ok.sum() >= len(ok) - 1
    assert np.max(np.abs(g["mean"][ok] - r["mean"][ok])) <= 1e-10
    assert np.max(np.abs(g["se"][ok] - r["se"][ok])) <= 1e-10
    assert np.array_equal(g["per_path"]["side"][~flips], r["per_path"]["side"][~flips])
    assert abs(g["steps"] - r["steps"]) <= int(flips.sum()) * 2 * 10**5
    assert g["paths"] == r["paths"] and g["capped"] == r["capped"] == 0


@pytest.mark.parametrize("bm", [
    {"kind": "identity"},
    {"kind": "affine", "p": [0.3, 2.0, -0.5, -1.0, 0.25, 3.0]},
    {"kind": "annulus", "p": [1.0, 2.0, 0.0, 0.5 * math.pi]},
    {"kind": "edge1d", "n_per_edge": 1025},
], ids=["identity", "affine", "annulus", "edge1d"])
@pytest.mark.parametrize("dseed", [3, 6])
def test_fp64_paths_match_oracle_all_terms_and_maps(ctx, ref, bm, dseed):
    d = W.random_density(dseed, 4)
    nodes = W.random_nodes(24, dseed + 100)
    g = gpu_estimate(ctx, d, bm, nodes, 300, 1e-3, 1000 + dseed, "fp64", per_path=True)
    r = ref.interface_estimate(d, bm, nodes, 300, 1e-3, 1000 + dseed, per_path=True)
    flips, dmax = compare_paths(g["per_path"], r["per_path"], 1e-12)
    say(f"{bm['kind']} d{dseed}: flips {int(flips.sum())}, max exit diff {dmax:.3e}")
    assert flips.sum() <= 1
    assert dmax <= 1e-12
    ok = _flip_free_nodes(flips)
    assert np.max(np.abs(g["mean"][ok] - r["mean"][ok])) <= 1e-10
    assert np.max(np.abs(g["se"][ok] - r["se"][ok])) <= 1e-10


def test_fp32_walk_matches_oracle_float_walk_and_double_estimates(ctx, ref):
    c = W.cfg_plain_fp64()
    nodes = ref.layout_nodes(c["layout"], c["k"])
    g = gpu_estimate(ctx, c["density"], c["bmap"], nodes, c["paths"], c["dt"], c["seed"], "fp32", per_path=True)
    r32 = ref.interface_estimate(c["density"], c["bmap"], nodes, c["paths"], c["dt"], c["seed"], "fp32",
                                 per_path=True)
    r64 = ref.interface_estimate(c["density"], c["bmap"], nodes, c["paths"], c["dt"], c["seed"], "fp64")
    flips, dmax = compare_paths(g["per_path"], r32["per_path"], 1e-5)
    gp, rp = g["per_path"], r32["per_path"]
    same = ~flips
    d = np.maximum(np.abs(gp["exit_xi"] - rp["exit_xi"]), np.abs(gp["exit_eta"] - rp["exit_eta"]))[same]
    q = np.percentile(d, [50, 99, 99.9])
    say(f"fp32 vs oracle fp32: flips {int(flips.sum())} of {flips.size}; exit diff p50 {q[0]:.2e} "
        f"p99 {q[1]:.2e} p99.9 {q[2]:.2e} max {dmax:.2e}")
    # the float walks differ only through the transcendental approximations
    # (hardware sin/cos/log/exp against libm), so paths agree to float
    # rounding amplified along the path; rare paths drift further
    assert flips.mean() < 2e-3
    assert q[1] < 1e-5 and dmax < 1e-2
    assert g["capped"] == 0 and np.all(np.isfinite(gp["exit_xi"]))
    # the stated accuracy bar: within 3 standard errors of the double oracle
    z64 = np.abs(g["mean"] - r64["mean"]) / r64["se"]
    say(f"fp32 vs fp64 oracle: max |diff|/SE = {z64.max():.3f}, max |diff| = {np.abs(g['mean'] - r64['mean']).max():.3e}")
    assert np.all(z64 <= 3.0)
    assert np.all(np.abs(g["mean"] - r32["mean"]) <= 0.5 * r32["se"])


def test_full_size_ring_workload_sampled_nodes(ctx, ref):
    """The throughput workload at full size (1521 nodes x 1e4 paths, dt=1e-5,
    float walk) in the benchmark's launch configuration; sampled nodes
    against the double-precision oracle, every node against symmetry."""
    c = W.cfg_ring_fp32()
    nodes = ref.layout_nodes(c["layout"], c["k"])
    g = gpu_estimate(ctx, c["density"], c["bmap"], nodes, c["paths"], c["dt"], c["seed"], "fp32")
    n = nodes.shape[0]
    assert np.all(np.isfinite(g["mean"])) and np.all((g["mean"] > 0) & (g["mean"] < 1))
    assert g["paths"] == n * c["paths"] and g["capped"] == 0
    sample = np.array([0, 5, 400, 800, 1100, 1520])
    say(f"oracle fp64 on {len(sample)} sampled nodes")
    r = ref.interface_estimate(c["density"], c["bmap"], nodes[sample], c["paths"], c["dt"], c["seed"],
                               node_ids=sample)
    z = np.abs(g["mean"][sample] - r["mean"]) / r["se"]
    say(f"ring fp32 vs fp64 oracle sampled: max z {z.max():.3f}, max |diff| {np.abs(g['mean'][sample] - r['mean']).max():.3e}")
    assert np.all(z <= 3.0)
    # mirror symmetry of the ring about xi = 1/2: x(1-xi, eta) = 1 - x(xi, eta)
    key = {tuple(np.rint(p * 256).astype(int)): i for i, p in enumerate(nodes)}
    zs = []
    for i, p in enumerate(nodes):
        j = key[(256 - int(round(p[0] * 256)), int(round(p[1] * 256)))]
        if j > i:
            s = math.hypot(g["se"][i, 0], g["se"][j, 0])
            zs.append((g["mean"][i, 0] + g["mean"][j, 0] - 1.0) / s)
    zs = np.array(zs)
    say(f"mirror pairs {len(zs)}: max |z| {np.abs(zs).max():.2f}, mean z^2 {np.mean(zs**2):.3f}")
    assert np.abs(zs).max() < 5.5
    assert np.mean(zs**2) < 1.3


@pytest.mark.parametrize("exit_test", ["step", "bridge"])
@pytest.mark.parametrize("kind", ["ring", "sech2"])
def test_small_step_float_walk_paths_match_oracle(ctx, ref, kind, exit_test):
    """Float walks at dt = 1e-5, where the loop that computes the next Philox
    block beside the current steps runs for sech^2 without the bridge and
    for the ring with it, and the plain loop otherwise.  Nodes near the
    walls and a cap of 501 steps (167 blocks), so that exits at every step
    of a block and capped paths are both present; per path against the
    oracle's float walk."""
    c = {"density": (W.cfg_ring_fp32() if kind == "ring" else W.cfg_annulus_fp32())["density"],
         "bmap": {"kind": "identity"}}
    rng = np.random.default_rng(31)
    near = rng.uniform(0.005, 0.03, 6)
    nodes = np.array([[near[0], 0.5], [1 - near[1], 0.4], [0.3, near[2]], [0.6, 1 - near[3]],
                      [near[4], near[5]], [0.5, 0.5]])
    dt, t_max, N = 1e-5, 5e-3, 300
    g = gpu_estimate(ctx, c["density"], c["bmap"], nodes, N, dt, 41, "fp32", per_path=True, t_max=t_max,
                     exit_test=exit_test)
    r = ref.interface_estimate(c["density"], c["bmap"], nodes, N, dt, 41, "fp32", per_path=True, t_max=t_max,
                               bridge=exit_test == "bridge")
    gp, rp = g["per_path"], r["per_path"]
    flips, dmax = compare_paths(gp, rp, 1e-5)
    same = ~flips
    d = np.maximum(np.abs(gp["exit_xi"] - rp["exit_xi"]), np.abs(gp["exit_eta"] - rp["exit_eta"]))[same]
    q = np.percentile(d, [50, 99])
    mod = np.bincount(rp["steps"][rp["capped"] == 0] % 3, minlength=3)
    say(f"small-step fp32 {kind} {exit_test}: flips {int(flips.sum())} of {flips.size}; capped {g['capped']} "
        f"(oracle {r['capped']}); exit steps mod 3 {mod.tolist()}; diff p50 {q[0]:.2e} p99 {q[1]:.2e} max {dmax:.2e}")
    assert g["capped"] > 0 and np.all(mod > 0)
    assert flips.mean() < 2e-3
    assert q[1] < 1e-5 and dmax < 1e-2
    cap_same = (gp["capped"] == rp["capped"])
    assert cap_same.mean() > 1 - 2e-3
    assert np.all(gp["steps"][gp["capped"] == 1] == 501)


def test_calls_on_side_streams_overlap_safely(ctx):
    """Two estimates on two side streams through one context run at the same
    time: each stream gets its own workspace, and each result is bitwise the
    one its call gives alone on the default stream."""
    import torch

    import paper_1310_3435_amd as sdd
    d = W.random_density(19, 2)
    bm = {"kind": "identity"}
    na = torch.as_tensor(W.random_nodes(40, 3)).cuda()
    nb = torch.as_tensor(W.random_nodes(70, 4)).cuda()
    ref_a = sdd.sdd_interface_estimate(ctx, d, bm, na, 3000, 1e-3, 5, "fp64", want_sums=True)
    ref_b = sdd.sdd_interface_estimate(ctx, d, bm, nb, 5000, 1e-3, 6, "fp32", want_sums=True)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    say("two estimates on two side streams")
    a = sdd.sdd_interface_estimate(ctx, d, bm, na, 3000, 1e-3, 5, "fp64", want_sums=True, stream=s1)
    b = sdd.sdd_interface_estimate(ctx, d, bm, nb, 5000, 1e-3, 6, "fp32", want_sums=True, stream=s2)
    torch.cuda.synchronize()
    for got, want in ((a, ref_a), (b, ref_b)):
        assert torch.equal(got["mean"], want["mean"]) and torch.equal(got["sums"], want["sums"])
        assert torch.equal(got["stats"][:3], want["stats"][:3])   # word 3 is the walk time


def test_full_size_annulus_workload_sampled_nodes(ctx, ref):
    """The curved workload at full size (3633 equidistributed nodes x 1e5
    paths, dt = 1e-5, float walk, shear-layer density, quarter-annulus map)
    in the benchmark's launch configuration; eight sampled nodes against the
    double-precision oracle."""
    c = W.cfg_annulus_fp32()
    nodes = ref.layout_nodes(c["layout"], c["k"], c["placement"], c["density"])
    g = gpu_estimate(ctx, c["density"], c["bmap"], nodes, c["paths"], c["dt"], c["seed"], "fp32")
    n = nodes.shape[0]
    assert n == 3633 and g["paths"] == n * c["paths"] and g["capped"] == 0
    assert np.all(np.isfinite(g["mean"]))
    # maximum principle per component: the sector's boundary lies in [0, 2]^2
    assert np.all((g["mean"] >= 0.0) & (g["mean"] <= 2.0))
    sample = np.linspace(0, n - 1, 8).astype(int)
    say(f"oracle fp64 on {len(sample)} sampled annulus nodes")
    r = ref.interface_estimate(c["density"], c["bmap"], nodes[sample], c["paths"], c["dt"], c["seed"],
                               node_ids=sample)
    z = np.abs(g["mean"][sample] - r["mean"]) / r["se"]
    say(f"annulus fp32 vs fp64 oracle sampled: max z {z.max():.3f}, max |diff| "
        f"{np.abs(g['mean'][sample] - r['mean']).max():.3e}")
    assert np.all(z <= 3.0)


def test_bias_sweep_workload_full_paths_fp64(ctx, ref):
    """The closed-form workload at its full 1e6 paths per node (dt = 1e-3,
    1D edge data as the boundary map), double walk, three of its nodes:
    path by path against the oracle."""
    c = W.cfg_sin2_sweep()
    nodes = np.array(c["nodes"])[[0, 31, 63]]
    N = c["paths"]
    g = gpu_estimate(ctx, c["density"], c["bmap"], nodes, N, 1e-3, c["seed"], "fp64", per_path=True)
    r = ref.interface_estimate(c["density"], c["bmap"], nodes, N, 1e-3, c["seed"], per_path=True)
    flips, dmax = compare_paths(g["per_path"], r["per_path"], 1e-12)
    say(f"sin2 fp64, 3 x 1e6 paths: flips {int(flips.sum())}, max exit diff {dmax:.3e}, "
        f"max mean diff {np.abs(g['mean'] - r['mean']).max():.3e}")
    assert flips.mean() < 1e-5 and dmax <= 1e-12
    # a flipped path moves its node's mean by at most 1/N of the map's range
    bound = np.maximum(1e-10, flips.sum(axis=1)[:, None] / N)
    assert np.all(np.abs(g["mean"] - r["mean"]) <= bound)


def test_edge_cases(ctx, ref):
    import torch

    import paper_1310_3435_amd as sdd
    d = W.random_density(11, 3)
    bm = {"kind": "identity"}
    # one path: SE is 0, the mean is that path's value
    nodes = W.random_nodes(3, 5)
    g = gpu_estimate(ctx, d, bm, nodes, 1, 1e-3, 9, "fp64", per_path=True)
    r = ref.interface_estimate(d, bm, nodes, 1, 1e-3, 9, per_path=True)
    assert np.all(g["se"] == 0)
    assert np.max(np.abs(g["mean"] - r["mean"])) <= 1e-12
    # ragged: paths not a multiple of the wave, a single node
    for N in (63, 65, 130, 4097):
        g = gpu_estimate(ctx, d, bm, nodes[:1], N, 1e-3, 10, "fp64", per_path=True)
        r = ref.interface_estimate(d, bm, nodes[:1], N, 1e-3, 10, per_path=True)
        flips, dmax = compare_paths(g["per_path"], r["per_path"], 1e-12)
        assert flips.sum() == 0 and dmax <= 1e-12
        assert abs(g["mean"] - r["mean"]).max() <= 1e-10
    # path ranges: counters follow the path index
    g = gpu_estimate(ctx, d, bm, nodes, 100, 1e-3, 12, "fp64", per_path=True, path_begin=1000)
    r = ref.interface_estimate(d, bm, nodes, 100, 1e-3, 12, path_begin=1000, per_path=True)
    flips, dmax = compare_paths(g["per_path"], r["per_path"], 1e-12)
    assert flips.sum() == 0 and dmax <= 1e-12
    # step cap: tiny t_max caps most paths, identically on both sides
    g = gpu_estimate(ctx, d, bm, nodes, 200, 1e-3, 13, "fp64", per_path=True, t_max=4.5e-3)
    r = ref.interface_estimate(d, bm, nodes, 200, 1e-3, 13, t_max=4.5e-3, per_path=True)
    assert g["capped"] == r["capped"] > 0
    assert np.array_equal(g["per_path"]["capped"], r["per_path"]["capped"])
    flips, dmax = compare_paths(g["per_path"], r["per_path"], 1e-12)
    assert flips.sum() == 0 and dmax <= 1e-12
    # a node on the boundary gives NaN, the others are unaffected
    bad = np.array([[0.5, 0.5], [0.0, 0.3], [0.25, 0.75]])
    g = gpu_estimate(ctx, d, bm, bad, 64, 1e-3, 14, "fp64")
    assert np.all(np.isnan(g["mean"][1])) and np.all(np.isfinite(g["mean"][[0, 2]]))
    r = ref.interface_estimate(d, bm, bad[[0, 2]], 64, 1e-3, 14, node_ids=[0, 2])
    assert np.max(np.abs(g["mean"][[0, 2]] - r["mean"])) <= 1e-10
    # determinism: two runs are bitwise equal
    a = gpu_estimate(ctx, d, bm, nodes, 5000, 1e-3, 15, "fp32")
    b = gpu_estimate(ctx, d, bm, nodes, 5000, 1e-3, 15, "fp32")
    assert np.array_equal(a["mean"], b["mean"]) and np.array_equal(a["sums"], b["sums"])
    # invalid arguments are rejected before any launch
    t = torch.as_tensor(nodes).cuda()
    for kw in ({"dt": 0.0}, {"dt": 1.5}, {"prec": "bf16"}):
        args = dict(dt=1e-3, prec="fp64")
        args.update(kw)
        with pytest.raises((sdd.SddError, KeyError)):
            sdd.sdd_interface_estimate(ctx, d, bm, t, 10, args["dt"], 1, args["prec"])
    with pytest.raises(sdd.SddError):
        sdd.sdd_interface_estimate(ctx, {"base": -1.0, "terms": []}, bm, t, 10, 1e-3, 1)
    # a step cap beyond the 28-bit step count, and path counters beyond 32 bits
    with pytest.raises(sdd.SddError, match="invalid"):
        sdd.sdd_interface_estimate(ctx, d, bm, t, 10, 1e-6, 1, t_max=300.0)
    with pytest.raises(sdd.SddError, match="invalid"):
        sdd.sdd_interface_estimate(ctx, d, bm, t, 10, 1e-3, 1, path_begin=2**32 - 5)
    # the largest accepted cap: ceil(t_max/dt) = 2^28 - 4 rounds up to a whole block
    g = gpu_estimate(ctx, d, bm, nodes, 64, 1e-3, 16, "fp32", t_max=(2**28 - 4) * 1e-3 * (1 - 1e-12))
    assert g["capped"] == 0 and np.all(np.isfinite(g["mean"]))


def test_many_nodes_per_drain(ctx, ref):
    """A few paths per node: every pool is a handful of paths, so a wave's
    exit queue holds many nodes at once and its node slots in LDS are evicted
    to the node sums over and over.  The sums are exact, so the double walk's
    means, sums and step totals must still match the oracle path for path,
    and the float walk must give the same sums with and without per-path
    records (a different schedule) and across repeated calls."""
    d = W.random_density(5, 3)
    bm = {"kind": "affine", "p": [0.3, 2.0, -0.5, -1.0, 0.25, 3.0]}
    nodes = W.random_nodes(500, 21)
    for N in (1, 5, 37):
        g = gpu_estimate(ctx, d, bm, nodes, N, 1e-3, 22, "fp64", per_path=True)
        r = ref.interface_estimate(d, bm, nodes, N, 1e-3, 22, per_path=True)
        flips, dmax = compare_paths(g["per_path"], r["per_path"], 1e-12)
        assert flips.sum() == 0 and dmax <= 1e-12
        assert np.max(np.abs(g["mean"] - r["mean"])) <= 1e-10
        assert np.max(np.abs(g["sums"] - r["sums"]) / np.maximum(1.0, np.abs(r["sums"]))) <= 1e-12
        assert g["steps"] == r["steps"] and g["paths"] == r["paths"] == 500 * N
    a = gpu_estimate(ctx, d, bm, nodes, 37, 1e-3, 23, "fp32")
    b = gpu_estimate(ctx, d, bm, nodes, 37, 1e-3, 23, "fp32", per_path=True)
    c = gpu_estimate(ctx, d, bm, nodes, 37, 1e-3, 23, "fp32")
    for o in (b, c):
        assert np.array_equal(a["sums"], o["sums"]) and np.array_equal(a["mean"], o["mean"])
        assert a["steps"] == o["steps"]
    assert int(b["per_path"]["steps"].sum()) == b["steps"]


def test_more_paths_than_32_bits_and_empty_inputs(ctx, ref):
    """n * N above 2^32 (70 000 nodes x 65 536 paths = 4.59e9 paths; the
    walk's workspace is the 6.7 MB of node sums), every path capped at three
    steps (one Philox block); sampled nodes against the oracle's float walk.
    Then empty node lists, zero paths, 2^32 paths and path counters past 32
    bits are rejected."""
    import ctypes as C

    import torch

    import paper_1310_3435_amd as sdd
    n, N = 70000, 65536
    assert n * N > 2**32
    d = W.random_density(21, 2)
    nodes = W.random_nodes(n, 22)
    t = torch.as_tensor(nodes).cuda()
    wsb = sdd.sdd_workspace_bytes(n, N, "fp32")
    say(f"{n} x {N} = {n * N} paths, workspace {wsb / 2**20:.1f} MiB")
    assert wsb < n * 100 + 4096
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    D = sdd.make_density(d)
    B = sdd.Bmap({"kind": "identity"}, ctx)
    mean = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    se = torch.empty_like(mean)
    stats = torch.empty(4, dtype=torch.int64, device="cuda")

    def call(nn, NN, work, work_bytes, begin=0):
        return sdd.lib().sdd_interface_estimate(ctx.h, C.byref(D), C.byref(B.s), t.data_ptr(), nn, NN, begin, 1e-3,
                                                C.c_uint64(23), sdd.SDD_FP32, 1e-3, 0, mean.data_ptr(),
                                                se.data_ptr(), None, stats.data_ptr(), None, work.data_ptr(),
                                                work_bytes, None)

    assert call(n, N, ws, wsb) == 0
    torch.cuda.synchronize()
    st = sdd.walk_stats(stats, warn=False)
    m, s = mean.cpu().numpy(), se.cpu().numpy()
    say(f"stats: steps {st['steps']}, paths {st['paths']}, capped {st['capped']}, {st['t_stoc_ms']:.1f} ms")
    assert st["paths"] == n * N and st["steps"] <= 3 * n * N and np.all(np.isfinite(m))
    assert st["capped"] > 0 and st["t_stoc_ms"] > 0
    sample = np.array([0, 1234, n // 2, n - 1])
    r = ref.interface_estimate(d, {"kind": "identity"}, nodes[sample], N, 1e-3, 23, "fp32", t_max=1e-3,
                               node_ids=sample)
    diff = np.abs(m[sample] - r["mean"]).max()
    say(f"sampled nodes vs oracle float walk: max |diff| {diff:.3e}")
    assert diff <= 1e-6 and np.abs(s[sample] - r["se"]).max() <= 1e-6
    # rejected before any launch
    assert sdd.sdd_workspace_bytes(n, 2**32, "fp32") == 0
    assert call(n, 2**32, ws, wsb) == sdd.SDD_EINVAL
    assert call(0, 16, ws, wsb) == sdd.SDD_EINVAL
    assert call(16, 0, ws, wsb) == sdd.SDD_EINVAL
    assert call(16, 100, ws, wsb, begin=2**32 - 50) == sdd.SDD_EINVAL
    assert call(n, N, ws, wsb - 256) == -2   # SDD_ENOSPC
