"""GPU tests of the request server (continuous batching).

* a request's mesh is bitwise the same alone and in a mix of other requests
  (paths depend only on their counters; node sums are exact integers);
* a served request agrees with the oracle's pipeline under common random
  numbers (within 3 standard errors of the double-precision walk);
* admission by device memory: a budget that holds one request runs the
  stream one at a time, first come first served;
* cancellation and shutdown with work in flight end cleanly;
* bridge and capped requests against the oracle, and served requests (with
  an SE target, or with a fixed path count and no pilot) bitwise equal to
  the estimate call followed by the fill and the solves.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1310_3435_amd as sdd
    return sdd.Context(0)


def small_request(seed=77, n=33, s=2, paths=0, se=1e-3, bumps=None):
    terms = bumps or [{"kind": "gauss", "amp": 6.0, "coef": 60.0, "cx": 0.4, "cy": 0.55}]
    return {"density": W.density(1.0, terms), "bmap": {"kind": "identity"},
            "layout": {"nx": n, "ny": n, "sx": s, "sy": s}, "k": (n - 1) // s - 1, "placement": "uniform",
            "interp": "linear", "dt": 1e-4, "se_target": se, "paths": paths, "seed": seed}


def test_result_is_the_same_alone_and_in_a_mix(ctx):
    import paper_1310_3435_amd as sdd
    target = small_request()
    srv = sdd.Server(ctx, hbm_budget_bytes=256 << 20, max_slots=16)
    try:
        say("serve: target alone")
        alone = srv.wait(srv.submit(target))
        assert alone["status"] == 0
        mix = W.serving_requests(50, master_seed=9, grids=(33, 65), splits=(2, 4))
        ids = [srv.submit(r) for r in mix[:25]]
        tid = srv.submit(target)
        ids += [srv.submit(r) for r in mix[25:]]
        say(f"serve: target in a mix of {len(mix)}")
        res = [srv.wait(i) for i in ids]
        mixed = srv.wait(tid)
    finally:
        srv.close()
    assert mixed["status"] == 0 and all(r["status"] == 0 for r in res)
    assert mixed["paths_per_node"] == alone["paths_per_node"] >= 1024
    assert mixed["steps"] == alone["steps"]
    assert np.array_equal(mixed["mesh"], alone["mesh"])
    say(f"paths/node {alone['paths_per_node']}, max SE {alone['max_se']:.2e}, bitwise equal")
    # the requested standard error was met
    assert alone["max_se"] <= 1e-3 * 1.05
    for r in res:
        assert np.all(np.isfinite(r["mesh"])) and r["max_se"] <= 1e-3 * 1.05


def test_served_mesh_matches_the_oracle_pipeline(ctx, ref):
    import paper_1310_3435_amd as sdd
    req = small_request(seed=5, paths=2048, se=0.0,
                        bumps=[{"kind": "gauss", "amp": 6.0, "coef": 60.0, "cx": 0.4, "cy": 0.55},
                               {"kind": "gauss", "amp": 3.0, "coef": 150.0, "cx": 0.7, "cy": 0.3}])
    srv = sdd.Server(ctx, hbm_budget_bytes=64 << 20, max_slots=4)
    try:
        say("serve: parity request")
        out = srv.wait(srv.submit(req))
    finally:
        srv.close()
    assert out["status"] == 0 and out["paths_per_node"] == 2048
    cfg = dict(req, paths=2048, prec="fp64")
    r64 = ref.pipeline(cfg)
    se = r64["est"]["se"].max()
    diff = np.abs(out["mesh"] - r64["mesh"]).max()
    say(f"served vs oracle double pipeline: max |diff| {diff:.3e}, node SE <= {se:.3e}")
    assert diff <= 3 * se
    r32 = ref.pipeline(dict(cfg, prec="fp32"))
    d32 = np.abs(out["mesh"] - r32["mesh"]).max()
    say(f"served vs oracle float pipeline: max |diff| {d32:.3e}")
    assert d32 <= 0.5 * se


def test_admission_by_device_memory_is_first_come_first_served(ctx):
    import paper_1310_3435_amd as sdd
    reqs = [small_request(seed=100 + i, n=65, s=4, paths=1024, se=0.0) for i in range(4)]
    # one 65^2 request with 4x4 subdomains needs ~187 KB of arena: 250 KB holds one
    srv = sdd.Server(ctx, hbm_budget_bytes=250 << 10, max_slots=8)
    try:
        say("serve: tiny arena, 4 requests")
        ids = [srv.submit(r) for r in reqs]
        res = [srv.wait(i) for i in ids]
    finally:
        srv.close()
    assert all(r["status"] == 0 for r in res)
    for a, b in zip(res, res[1:]):
        assert b["t_admit"] >= a["t_done"] - 1e-3   # admitted only after the previous one freed its memory
    assert all(np.all(np.isfinite(r["mesh"])) for r in res)


def test_cancel_and_shutdown(ctx):
    import paper_1310_3435_amd as sdd
    srv = sdd.Server(ctx, hbm_budget_bytes=250 << 10, max_slots=2)
    big = small_request(seed=3, n=65, s=4, se=2e-4)
    a = srv.submit(big)
    b = srv.submit(small_request(seed=4, n=65, s=4, se=2e-4))   # queued behind a (arena)
    srv.cancel(b)
    rb = srv.wait(b)
    assert rb["status"] == sdd.SDD_ECANCELED and np.all(rb["mesh"] == 0)
    srv.cancel(a)
    ra = srv.wait(a)
    assert ra["status"] == sdd.SDD_ECANCELED
    # shutdown with requests still running drains and returns
    for i in range(3):
        srv.submit(small_request(seed=10 + i, n=65, s=4, se=2e-4))
    say("serve: destroy with work in flight")
    srv.close()


def test_rejected_requests(ctx):
    import paper_1310_3435_amd as sdd
    srv = sdd.Server(ctx, hbm_budget_bytes=8 << 20, max_slots=2, max_nodes=100, max_points=65 * 65)
    try:
        ring = small_request()
        ring["density"] = W.density(1.0, [{"kind": "ring", "amp": 1.0, "coef": 10.0, "cx": 0.5, "cy": 0.5,
                                          "r0": 0.2}])
        with pytest.raises(sdd.SddError, match="unsupported"):
            srv.submit(ring)
        with pytest.raises(sdd.SddError, match="unsupported"):   # exponential stepping: estimate calls only
            srv.submit(dict(small_request(), exit_test="expo"))
        with pytest.raises(sdd.SddError, match="invalid"):
            srv.submit(small_request(n=129, s=2))     # more points than max_points
        with pytest.raises(sdd.SddError, match="invalid"):
            srv.submit(dict(small_request(), dt=0.0))
        ok = srv.wait(srv.submit(small_request(paths=1024, se=0.0)))
        assert ok["status"] == 0
    finally:
        srv.close()


def test_bridge_request_alone_in_a_mix_and_against_the_oracle(ctx, ref):
    import paper_1310_3435_amd as sdd
    req = dict(small_request(seed=21, paths=2048, se=0.0), dt=1e-3, exit_test="bridge")
    srv = sdd.Server(ctx, hbm_budget_bytes=256 << 20, max_slots=16)
    try:
        say("serve: bridge request alone")
        alone = srv.wait(srv.submit(req))
        mix = W.serving_requests(12, master_seed=13, grids=(33, 65), splits=(2, 4))
        ids = [srv.submit(dict(r, exit_test="bridge" if i % 2 else "step")) for i, r in enumerate(mix[:6])]
        tid = srv.submit(req)
        ids += [srv.submit(r) for r in mix[6:]]
        say("serve: bridge request in a mix of step and bridge requests")
        res = [srv.wait(i) for i in ids]
        mixed = srv.wait(tid)
    finally:
        srv.close()
    assert alone["status"] == 0 and mixed["status"] == 0 and all(r["status"] == 0 for r in res)
    assert np.array_equal(mixed["mesh"], alone["mesh"]) and mixed["steps"] == alone["steps"]
    cfg = dict(req, paths=2048, prec="fp64")
    r64 = ref.pipeline(cfg)
    se = r64["est"]["se"].max()
    diff = np.abs(alone["mesh"] - r64["mesh"]).max()
    r32 = ref.pipeline(dict(cfg, prec="fp32"))
    d32 = np.abs(alone["mesh"] - r32["mesh"]).max()
    plain = ref.pipeline(dict(cfg, exit_test="step"))
    shift = np.abs(plain["mesh"] - r64["mesh"]).max()
    say(f"served bridge vs oracle: double {diff:.3e}, float {d32:.3e} (SE {se:.3e}); bridge moved the mesh {shift:.3e}")
    assert diff <= 3 * se and d32 <= 0.5 * se
    assert shift > 3 * se          # at this dt the bridge changes the mesh well beyond the noise


def test_capped_request_matches_the_oracle(ctx, ref):
    """A step cap of 0.01 time units (102 steps at dt = 1e-4) stops most
    paths: the serving walk's cap (whole Philox blocks) and the reduction's
    nearest-boundary value for capped paths against the oracle's pipeline."""
    import paper_1310_3435_amd as sdd
    req = dict(small_request(seed=8, paths=2048, se=0.0), t_max=0.01)
    srv = sdd.Server(ctx, hbm_budget_bytes=64 << 20, max_slots=4)
    try:
        say("serve: capped request")
        out = srv.wait(srv.submit(req))
    finally:
        srv.close()
    # done, with a warning: some paths stopped at the cap
    assert out["status"] == sdd.SDD_WARN_CAPPED and out["paths_per_node"] == 2048
    cfg = dict(req, prec="fp32")
    r32 = ref.pipeline(cfg)
    est = r32["est"]
    assert est["capped"] > 0.3 * est["paths"]
    assert out["capped"] == pytest.approx(est["capped"], rel=1e-3)
    r64 = ref.pipeline(dict(cfg, prec="fp64"))
    se = r64["est"]["se"].max()
    d32 = np.abs(out["mesh"] - r32["mesh"]).max()
    say(f"capped request: {est['capped']} of {est['paths']} oracle paths capped; steps {out['steps']} "
        f"(oracle {est['steps']}); served vs oracle float pipeline {d32:.3e} (SE {se:.3e})")
    assert out["steps"] == pytest.approx(est["steps"], rel=1e-4)
    assert d32 <= 0.05 * se
    assert np.abs(out["mesh"] - r64["mesh"]).max() <= 3 * se


def test_served_request_equals_the_estimate_call_bitwise(ctx):
    """One walk implementation: a served float request walks exactly the
    paths of an sdd_interface_estimate call with the same inputs (path 0 at
    counter 0, N = the request's paths per node), its node sums are exact,
    so the fill and solves downstream give the same mesh bit for bit.  The
    request reports its stage times."""
    import torch

    import paper_1310_3435_amd as sdd
    for exit_test in ("step", "bridge"):
        req = dict(small_request(seed=61, n=65, s=4,
                                 bumps=[{"kind": "gauss", "amp": 6.0, "coef": 60.0, "cx": 0.4, "cy": 0.55},
                                        {"kind": "gauss", "amp": 12.0, "coef": 150.0, "cx": 0.7, "cy": 0.3}]),
                   exit_test=exit_test)
        srv = sdd.Server(ctx, hbm_budget_bytes=64 << 20, max_slots=4)
        try:
            say(f"serve: one {exit_test} request")
            out = srv.wait(srv.submit(req))
        finally:
            srv.close()
        assert out["status"] == 0
        N = out["paths_per_node"]
        assert N % 1024 == 0 and N > 1024
        assert out["t_stoc_ms"] > 0 and out["t_fill_ms"] > 0 and out["t_sub_ms"] > 0 and out["t_queue_ms"] >= 0
        say(f"  N {N}, T_stoc {out['t_stoc_ms']:.1f} ms, T_fill {out['t_fill_ms']:.2f} ms, "
            f"T_sub {out['t_sub_ms']:.2f} ms")
        L = req["layout"]
        nodes = sdd.sdd_layout_nodes(ctx, L, req["k"], "uniform", req["density"])
        est = sdd.sdd_interface_estimate(ctx, req["density"], req["bmap"], nodes, N, req["dt"], req["seed"], "fp32",
                                         exit_test=exit_test)
        vert, horiz = sdd.sdd_fill_interfaces(ctx, L, req["k"], req["bmap"], nodes, est["mean"], "linear")
        mesh = sdd.sdd_subdomain_solve(ctx, req["density"], req["bmap"], L, vert, horiz)["mesh"]
        torch.cuda.synchronize()
        st = sdd.walk_stats(est["stats"])
        assert st["steps"] == out["steps"]
        assert np.array_equal(mesh.cpu().numpy(), out["mesh"])
        say(f"  served mesh == estimate + fill + solve, bitwise ({st['steps']} steps)")


def test_fixed_path_request_equals_the_estimate_call_bitwise(ctx):
    """A request that gives its path count (no SE target) has no pilot: all
    of its blocks may go into the first launch.  Its paths per node are the
    count rounded up to whole blocks of 1024, and, alone or behind other
    requests, it walks exactly the paths of the estimate call."""
    import torch

    import paper_1310_3435_amd as sdd
    req = small_request(seed=23, n=65, s=2, paths=5000, se=0.0)
    srv = sdd.Server(ctx, hbm_budget_bytes=256 << 20, max_slots=8)
    try:
        say("serve: a fixed-path request alone, then behind six others")
        alone = srv.wait(srv.submit(req))
        others = [srv.submit(r) for r in W.serving_requests(6, master_seed=4, grids=(33, 65), splits=(2, 4))]
        mixed = srv.wait(srv.submit(req))
        rest = [srv.wait(i) for i in others]
    finally:
        srv.close()
    assert alone["status"] == mixed["status"] == 0 and all(r["status"] >= 0 for r in rest)
    assert alone["paths_per_node"] == mixed["paths_per_node"] == 5120
    assert np.array_equal(alone["mesh"], mixed["mesh"]) and alone["steps"] == mixed["steps"]
    L = req["layout"]
    nodes = sdd.sdd_layout_nodes(ctx, L, req["k"], "uniform", req["density"])
    est = sdd.sdd_interface_estimate(ctx, req["density"], req["bmap"], nodes, 5120, req["dt"], req["seed"], "fp32")
    vert, horiz = sdd.sdd_fill_interfaces(ctx, L, req["k"], req["bmap"], nodes, est["mean"], "linear")
    mesh = sdd.sdd_subdomain_solve(ctx, req["density"], req["bmap"], L, vert, horiz)["mesh"]
    torch.cuda.synchronize()
    assert sdd.walk_stats(est["stats"])["steps"] == alone["steps"]
    assert np.array_equal(mesh.cpu().numpy(), alone["mesh"])
    say(f"  5000 -> 5120 paths per node, alone == in a mix == estimate + fill + solve, bitwise")


def test_walks_on_fewer_cus_give_the_same_result(ctx, monkeypatch):
    """SDD_SERVE_RESERVED_CUS keeps the walk launches off some CUs (their
    streams carry a CU mask), so that subdomain solves find free CUs.  Where
    the walks run does not change what they compute: same mesh, bitwise."""
    import paper_1310_3435_amd as sdd
    req = small_request(seed=29, n=65, s=4, paths=3000, se=0.0)
    got = []
    for reserve in ("0", "16"):
        monkeypatch.setenv("SDD_SERVE_RESERVED_CUS", reserve)
        srv = sdd.Server(ctx, hbm_budget_bytes=256 << 20, max_slots=8)
        try:
            say(f"serve: a fixed-path request with {reserve} CUs left to the solves")
            got.append(srv.wait(srv.submit(req)))
        finally:
            srv.close()
    a, b = got
    assert a["status"] == b["status"] == 0
    assert a["steps"] == b["steps"] and np.array_equal(a["mesh"], b["mesh"])
