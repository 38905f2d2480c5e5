"""GPU parity of exponential time stepping (Sec. 2.2) against the oracle
(same Philox counters: the step lengths come from the blocks with counter
word 3 = 2, so paths are compared one by one).

Bars.  Single-term densities, as for the other exit tests: double per-path
exit points within 1e-12 and equal exit steps, node means within 1e-10.
Float: per path p99 <= 1e-5 with rare flips, node estimates within 3 SE of
the double oracle.  Steep sums of four terms in double: exponential steps
are unbounded (P(tau > 10 dt) = e^-10), and a long step on a steep density
multiplies a last-ulp difference by tau |grad b| >> 1, so paths spread out
of the 1e-12 band.  The oracle alone shows the size of it: moving every
tau by one ulp (what two libraries' log may differ by) moves this
workload's exit points by p97 7e-12, p99 1e-9, flips 4 of 6000 exit steps
and shifts node means by up to 0.1 SE.  The bar for those densities is
that band: flips below 2e-3, p90 <= 1e-12, p99 <= 1e-8, node means within
0.25 SE.  Then the closed form of the first passage through an exponential
clock (w = 1) on the GPU itself.
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


@pytest.mark.parametrize("bm", [
    {"kind": "identity"},
    {"kind": "annulus", "p": [1.0, 2.0, 0.0, 0.5 * math.pi]},
    {"kind": "edge1d", "n_per_edge": 1025},
], ids=["identity", "annulus", "edge1d"])
@pytest.mark.parametrize("terms", [1, 4])
def test_fp64_expo_paths_match_oracle(ctx, ref, bm, terms):
    d = W.random_density(7 + terms, terms)
    nodes = W.random_nodes(20, 300 + terms)
    g = gpu_estimate(ctx, d, bm, nodes, 300, 1e-3, 77, "fp64", per_path=True, exit_test="expo")
    r = ref.interface_estimate(d, bm, nodes, 300, 1e-3, 77, per_path=True, exit_test="expo")
    gp, rp = g["per_path"], r["per_path"]
    d = np.maximum(np.abs(gp["exit_xi"] - rp["exit_xi"]), np.abs(gp["exit_eta"] - rp["exit_eta"]))
    flips = gp["steps"] != rp["steps"]
    q = np.percentile(d[~flips], [90, 99])
    say(f"expo fp64 {bm['kind']} {terms} terms: flips {int(flips.sum())} of {flips.size}, exit diff p90 {q[0]:.2e} "
        f"p99 {q[1]:.2e}, paths beyond 1e-12 {int((d > 1e-12).sum())}")
    if terms == 1:
        assert flips.sum() == 0 and d.max() <= 1e-12
        assert np.max(np.abs(g["mean"] - r["mean"])) <= 1e-10
        assert np.max(np.abs(g["se"] - r["se"])) <= 1e-10
        assert np.array_equal(gp["side"], rp["side"])
    else:
        assert flips.mean() < 2e-3 and q[0] <= 1e-12 and q[1] <= 1e-8
        assert np.all(np.abs(g["mean"] - r["mean"]) <= 0.25 * r["se"])


@pytest.mark.parametrize("kind", ["gauss", "ring", "sech2", "sin2"])
def test_fp32_expo_paths_match_oracle(ctx, ref, kind):
    cfgs = {"gauss": W.cfg_plain_fp64, "ring": W.cfg_ring_fp32, "sech2": W.cfg_annulus_fp32,
            "sin2": W.cfg_sin2_sweep}
    d = cfgs[kind]()["density"]
    nodes = W.random_nodes(16, 41)
    g = gpu_estimate(ctx, d, {"kind": "identity"}, nodes, 400, 1e-4, 88, "fp32", per_path=True, exit_test="expo")
    r = ref.interface_estimate(d, {"kind": "identity"}, nodes, 400, 1e-4, 88, "fp32", per_path=True,
                               exit_test="expo")
    gp, rp = g["per_path"], r["per_path"]
    flips, dmax = compare_paths(gp, rp, 1e-5)
    d_ = np.maximum(np.abs(gp["exit_xi"] - rp["exit_xi"]), np.abs(gp["exit_eta"] - rp["exit_eta"]))[~flips]
    q99 = np.percentile(d_, 99)
    say(f"expo fp32 {kind}: flips {int(flips.sum())} of {flips.size}, p99 {q99:.2e}, max {dmax:.2e}")
    assert flips.mean() < 2e-3 and q99 <= 1e-5 and dmax <= 1e-3
    r64 = ref.interface_estimate(d, {"kind": "identity"}, nodes, 400, 1e-4, 88, exit_test="expo")
    z = np.abs(g["mean"] - r64["mean"]) / np.maximum(r64["se"], 1e-300)
    assert np.all(z <= 3.0)


def test_expo_first_passage_closed_form_on_gpu(ctx):
    """w = 1, three steps at most: the GPU's exit fractions by steps 1, 2, 3
    against e^{-c}, e^{-c}(1 + c/2), e^{-c}(1 + 5c/8 + c^2/8), c = a/sqrt(dt)."""
    flat = {"base": 1.0, "terms": []}
    a = np.array([0.01, 0.03, 0.06])
    nodes = np.stack([a, np.full_like(a, 0.5)], 1)
    N, dt = 1 << 20, 1e-3
    for prec in ("fp64", "fp32"):
        g = gpu_estimate(ctx, flat, {"kind": "identity"}, nodes, N, dt, 29, prec, per_path=True, t_max=3 * dt,
                         exit_test="expo")
        pp = g["per_path"]
        exited = pp["capped"] == 0
        for i, ai in enumerate(a):
            c = ai / math.sqrt(dt)
            F = [math.exp(-c), math.exp(-c) * (1 + c / 2), math.exp(-c) * (1 + 5 * c / 8 + c * c / 8)]
            for k in (1, 2, 3):
                f = float((exited[i] & (pp["steps"][i] <= k)).mean())
                assert abs(f - F[k - 1]) <= 4.5 * math.sqrt(F[k - 1] * (1 - F[k - 1]) / N), (prec, ai, k, f)
        say(f"expo {prec}: exit fractions match the first-passage closed form")
