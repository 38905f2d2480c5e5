"""Pins of the oracle's Brownian-bridge exit test (Sec. 2.2: the conditional
probability that the process left the square during a step whose ends are
both inside).

* the probability and side of one step against brute-force simulated
  Brownian bridges (fine substeps with the continuity correction for
  discrete monitoring), near each kind of wall and in a corner;
* the bridge uniform comes from its own Philox block (counter word 3 = 1);
* with the bridge, the mean exit time of Brownian motion (w = 1) matches the
  torsion function to O(dt) with no correction, where the plain end-of-step
  test is off by O(sqrt dt);
* with the bridge, the 1-D closed form is met to O(dt), where the plain test
  is off by O(sqrt dt);
* under common random numbers a bridged path never takes more steps than
  the plain one and agrees with it until it leaves.
"""
import math

import numpy as np
import pytest

from tests.test_oracle_walk import closed_form_sin2, torsion

BETA = 0.5825971579390106   # -zeta(1/2)/sqrt(2 pi), discrete-monitoring shift


def brute_force_bridges(P, Q, dt, n=20000, n_sub=2000, seed=0, chunk=2000):
    """Fraction of 2-D Brownian bridges (diffusion coefficient 2) from P to Q
    over time dt that leave the unit square, and the wall each hits first.
    The bridge is watched at n_sub substeps with the walls moved in by
    BETA sqrt(2 h): watching at discrete times is, to first order, watching
    continuously a wall that far further out (Broadie-Glasserman-Kou)."""
    rng = np.random.default_rng(seed)
    h = dt / n_sub
    c = BETA * math.sqrt(2.0 * h)
    t = np.arange(1, n_sub + 1) * h
    first = np.full(n, -1)
    for i0 in range(0, n, chunk):
        m = min(chunk, n - i0)
        walls = []
        for d in range(2):
            W = np.cumsum(rng.standard_normal((m, n_sub)) * math.sqrt(2.0 * h), axis=1)
            B = P[d] + (Q[d] - P[d]) * t / dt + W - (t / dt) * W[:, -1:]
            lo = np.where((B <= c).any(1), (B <= c).argmax(1), n_sub + 1)
            hi = np.where((B >= 1 - c).any(1), (B >= 1 - c).argmax(1), n_sub + 1)
            walls += [lo, hi]
        walls = np.stack(walls, 1)                      # first substep at each wall
        hit = walls.min(1) <= n_sub
        first[i0:i0 + m] = np.where(hit, walls.argmin(1), -1)
    return float((first >= 0).mean()), np.bincount(first[first >= 0], minlength=4)


CASES = [  # P, Q, dt: near xi=0, near xi=1, near eta=0, a corner, far from every wall
    ((0.02, 0.5), (0.03, 0.52), 1e-3),
    ((0.985, 0.4), (0.97, 0.41), 1e-3),
    ((0.4, 0.01), (0.45, 0.05), 1e-3),
    ((0.03, 0.96), (0.025, 0.97), 1e-3),
    ((0.5, 0.5), (0.52, 0.49), 1e-3),
]


@pytest.mark.parametrize("P,Q,dt", CASES)
def test_step_exit_probability_matches_brute_force_bridges(ref, P, Q, dt):
    p, side = ref.bridge_exit_prob(P, Q, dt)
    n = 20000
    f, first = brute_force_bridges(np.array(P), np.array(Q), dt, n=n)
    tol = 4.0 * math.sqrt(max(p * (1 - p), 1e-4) / n) + 0.01
    assert abs(f - p) <= tol, (f, p)
    if p > 0.05:
        assert side == int(np.argmax(first))


def test_bridge_probability_symmetries(ref):
    # reversing the step, reflecting the square and swapping the axes leave it unchanged
    P, Q, dt = (0.03, 0.2), (0.05, 0.31), 2e-3
    p, s = ref.bridge_exit_prob(P, Q, dt)
    assert ref.bridge_exit_prob(Q, P, dt)[0] == p
    pr, sr = ref.bridge_exit_prob((1 - P[0], P[1]), (1 - Q[0], Q[1]), dt)
    assert pr == pytest.approx(p, rel=1e-13) and (s, sr) == (0, 1)
    pt, st = ref.bridge_exit_prob((P[1], P[0]), (Q[1], Q[0]), dt)
    assert pt == pytest.approx(p, rel=1e-13) and st == 2
    # a step ending on the wall's far side of the probability scale
    assert ref.bridge_exit_prob((0.5, 0.5), (0.5, 0.5), 1e-4)[0] == 0.0
    assert ref.bridge_exit_prob((1e-12, 0.5), (0.3, 0.5), 1e-3)[0] == pytest.approx(1.0, abs=1e-9)


def test_bridge_uniform_from_its_own_block(ref):
    # value: u = ((q mod 2^23) + 1/2) 2^-23 of a word of the counter-word-3 = 1 block
    w = np.array([0xFF800000, 0, 0xFFFFFFFF, 0x007FFFFF, 12345678], dtype=np.uint32)
    u = ref.bridge_uniforms(w)
    f = 2.0**-23
    assert list(u) == [0.5 * f, 0.5 * f, (2**23 - 0.5) * f, (2**23 - 0.5) * f, ((12345678 % 2**23) + 0.5) * f]
    # its blocks are not the normals' blocks: word 3 of the counter differs
    ctr = np.array([[5, 7, 9, 0], [5, 7, 9, 1]], dtype=np.uint32)
    blk = ref.philox(ctr, [3, 0])
    assert not np.any(blk[0] == blk[1])
    # uniform on (0, 1), exact in float
    rng = np.random.default_rng(3)
    u = ref.bridge_uniforms(rng.integers(0, 2**32, size=200000, dtype=np.uint64).astype(np.uint32))
    assert np.all((u > 0) & (u < 1)) and np.array_equal(u.astype(np.float32).astype(np.float64), u)
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 2e-3


def test_mean_exit_time_matches_torsion_without_correction(ref):
    # w = 1: dX = sqrt(2) dW, whose mean exit time solves Laplace v = -1.  A
    # bridged exit falls inside its step, so (k - 1/2) dt estimates tau.
    flat = {"base": 1.0, "terms": []}
    nodes = np.array([[0.5, 0.5], [0.1, 0.3], [0.05, 0.05], [0.8, 0.6]])
    T = np.array([torsion(*p) for p in nodes])
    dt = 1e-3
    z = {}
    for bridge in (True, False):
        r = ref.interface_estimate(flat, {"kind": "identity"}, nodes, 20000, dt, 11, per_path=True, bridge=bridge)
        tau = (r["per_path"]["steps"] - 0.5) * dt
        m, s = tau.mean(1), tau.std(1) / math.sqrt(tau.shape[1])
        z[bridge] = np.abs(m - T) / (4 * s + 2 * dt)
    assert np.all(z[True] <= 1.0), z[True]
    assert np.any(z[False] > 1.0)    # the plain test's overshoot is visible at this dt


def test_closed_form_to_first_order(ref):
    import workloads as W
    c = W.cfg_sin2_sweep()
    d = c["density"]
    B = ref.Bmap(c["bmap"], d)
    xi = np.array([1, 8, 16, 32, 40, 64]) / 65.0
    nodes = np.stack([xi, np.full_like(xi, 0.5)], 1)
    exact = closed_form_sin2(xi)
    dt = 1e-3
    ok = {}
    for bridge in (True, False):
        r = ref.interface_estimate(d, B, nodes, 40000, dt, 7, bridge=bridge)
        ok[bridge] = np.abs(r["mean"][:, 0] - exact) <= 4 * r["se"][:, 0] + 8 * dt
    assert ok[True].all()
    assert not ok[False].all()


def test_bridge_only_shortens_paths(ref):
    import workloads as W
    c = W.cfg_plain_fp64()
    nodes = np.array([[0.2, 0.3], [0.5, 0.5], [0.9, 0.85]])
    for prec in ("fp64", "fp32"):
        a = ref.interface_estimate(c["density"], c["bmap"], nodes, 500, 1e-3, 5, prec=prec, per_path=True)
        b = ref.interface_estimate(c["density"], c["bmap"], nodes, 500, 1e-3, 5, prec=prec, per_path=True,
                                   bridge=True)
        ra, rb = a["per_path"], b["per_path"]
        assert np.all(rb["steps"] <= ra["steps"])
        same = rb["steps"] == ra["steps"]
        # where the bridge did not fire first the path and its exit are the same
        assert np.array_equal(rb["exit_xi"][same & (ra["side"] == rb["side"])],
                              ra["exit_xi"][same & (ra["side"] == rb["side"])])
        assert (rb["steps"] < ra["steps"]).mean() > 0.2
        # a bridged exit lies on its side
        for s, col, v in ((0, "exit_xi", 0.0), (1, "exit_xi", 1.0), (2, "exit_eta", 0.0), (3, "exit_eta", 1.0)):
            assert np.all(rb[col][rb["side"] == s] == v)


def test_float_bridge_agrees_with_double(ref):
    import workloads as W
    c = W.cfg_plain_fp64()
    nodes = np.array([[0.25, 0.5], [0.6, 0.4]])
    a = ref.interface_estimate(c["density"], c["bmap"], nodes, 4000, 1e-4, 9, per_path=True, bridge=True)
    b = ref.interface_estimate(c["density"], c["bmap"], nodes, 4000, 1e-4, 9, prec="fp32", per_path=True,
                               bridge=True)
    flips = (a["per_path"]["steps"] != b["per_path"]["steps"]).mean()
    assert flips < 5e-3
    assert np.abs(a["mean"] - b["mean"]).max() < 0.25 * a["se"].max()


def test_bridge_capped_paths(ref):
    c = {"base": 1.0, "terms": []}
    r = ref.interface_estimate(c, {"kind": "identity"}, np.array([[0.5, 0.5]]), 200, 1e-3, 1, t_max=0.005,
                               per_path=True, bridge=True)
    pp = r["per_path"]
    assert r["capped"] == int(pp["capped"].sum()) > 100
    assert np.all(pp["steps"][pp["capped"] == 1] == 6)
    assert np.all(pp["steps"] <= 6)
