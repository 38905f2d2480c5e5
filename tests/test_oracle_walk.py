"""Statistical pins of the oracle's walk against what the mathematics fixes.

Every check is a z-test of the Monte Carlo estimate (standard error from the
paths themselves) against an exact value, with a Bonferroni bound |z| <= 4.3
per component (family error ~1e-3 over the ~60 components of one test) and,
where many components are tested together, a chi-square bound on sum z^2.

* martingale: for constant w the Euler-Maruyama walk has no drift, so the
  unprojected overshoot point has expectation equal to the start point at
  any dt (discrete optional stopping) -- pins the stepping and stopping;
* symmetry: reflections that map w and the boundary data onto themselves fix
  the solution at every dt;
* closed form: w = w(xi) with the one-dimensional edge data of Sec. 3.2 makes
  x = int_0^xi 1/w / int_0^1 1/w exact; Richardson extrapolation in sqrt(dt)
  removes the O(sqrt(dt)) exit-monitoring bias -- pins drift sign and the
  sqrt(2) diffusion of eq. (6)/(7b);
* brute force: a direct finite-difference solve of eq. (5) on fine grids;
* mean exit time: for w = 1 the expected exit time is the torsion function
  (Laplace v = -1), so the mean step count pins the noise scale.
"""
import math

import numpy as np
import pytest
from scipy import stats

import workloads as W

ZMAX = 4.3
CONST = {"base": 2.5, "terms": []}


def _chi2_ok(z):
    z = np.asarray(z).ravel()
    return (z**2).sum() <= stats.chi2.ppf(1 - 1e-3, z.size)


def torsion(x, y, terms=400):
    """Solution of Laplace v = -1 on the unit square, v = 0 on the boundary."""
    m = np.arange(1, 2 * terms, 2)[:, None]
    n = np.arange(1, 2 * terms, 2)[None, :]
    c = 16.0 / (math.pi**4 * m * n * (m**2 + n**2))
    return float((c * np.sin(m * math.pi * x) * np.sin(n * math.pi * y)).sum())


def closed_form_sin2(xi):
    """int_0^xi 1/w / int_0^1 1/w for w = 1 + 3 sin^2(2 pi xi): Theta(2 pi xi)/(2 pi)
    with Theta(t) = arctan(2 tan t), continued through the poles of tan."""
    t = 2 * math.pi * np.asarray(xi, dtype=np.float64)
    th = np.arctan2(2 * np.sin(t), np.cos(t))
    th = np.where(th < 0, th + 2 * math.pi, th)
    return th / (2 * math.pi)


def test_torsion_series_value():
    # the centre value quoted in the literature for -Laplace v = 1
    assert torsion(0.5, 0.5) == pytest.approx(0.0736713, abs=2e-7)


def test_martingale_overshoot_is_unbiased_at_any_dt(ref):
    aff = {"kind": "affine", "p": [0.3, 2.0, -0.5, -1.0, 0.25, 3.0]}
    nodes = np.array([[0.1, 0.2], [0.7, 0.9], [0.33, 0.5], [0.95, 0.05]])
    exact = np.stack([0.3 + 2 * nodes[:, 0] - 0.5 * nodes[:, 1], -1 + 0.25 * nodes[:, 0] + 3 * nodes[:, 1]], 1)
    zs = []
    for dt, seed in ((2e-2, 21), (1e-2, 22), (1e-3, 23)):
        r = ref.interface_estimate(CONST, aff, nodes, 40000, dt, seed, proj_mode=1)
        z = (r["mean"] - exact) / r["se"]
        assert np.all(np.abs(z) <= ZMAX), z
        zs.append(z)
    assert _chi2_ok(zs)


def test_projection_bias_shrinks_like_sqrt_dt(ref):
    """The projected estimate is biased by the late exit detection, and the
    bias falls by ~sqrt(10) per decade of dt (Sec. 2.2)."""
    nodes = np.array([[0.08, 0.5]])
    b = []
    for dt in (1e-2, 1e-3):
        r = ref.interface_estimate(CONST, {"kind": "identity"}, nodes, 40000, dt, 31)
        b.append(r["mean"][0, 0] - 0.08)
    ratio = b[0] / b[1]
    assert 2.2 < ratio < 4.5, ratio


def test_symmetry_lines_are_exact(ref):
    """w = 1 and the identity map are symmetric under xi -> 1-xi and
    eta -> 1-eta, so x(1/2, eta) = 1/2 and y(xi, 1/2) = 1/2 at every dt."""
    nodes = np.array([[0.5, 0.1], [0.5, 0.37], [0.2, 0.5], [0.93, 0.5]])
    r = ref.interface_estimate({"base": 1.0, "terms": []}, {"kind": "identity"}, nodes, 20000, 1e-3, 41)
    z = np.concatenate([(r["mean"][:2, 0] - 0.5) / r["se"][:2, 0], (r["mean"][2:, 1] - 0.5) / r["se"][2:, 1]])
    assert np.all(np.abs(z) <= ZMAX), z


def test_symmetry_of_the_gaussian_workload(ref):
    """Gaussian bump at the centre, identity map: x(1/2, eta) = 1/2,
    y(1/2, eta) + y(1/2, 1-eta) = 1 and y(1/2, 1/2) = 1/2."""
    c = W.cfg_plain_fp64()
    nodes = ref.layout_nodes(c["layout"], c["k"])
    r = ref.interface_estimate(c["density"], c["bmap"], nodes, c["paths"], c["dt"], c["seed"])
    m, se = r["mean"], r["se"]
    zx = (m[:, 0] - 0.5) / se[:, 0]
    j = np.arange(7)
    zy = (m[j, 1] + m[14 - j, 1] - 1.0) / np.hypot(se[j, 1], se[14 - j, 1])
    zc = (m[7, 1] - 0.5) / se[7, 1]
    z = np.concatenate([zx, zy, [zc]])
    assert np.all(np.abs(z) <= ZMAX), z
    assert _chi2_ok(z)
    assert r["capped"] == 0


@pytest.mark.slow
def test_closed_form_when_w_depends_on_xi_only(ref):
    c = W.cfg_sin2_sweep()
    d = c["density"]
    B = ref.Bmap(c["bmap"], d)
    xi = np.array([1, 8, 16, 32, 40, 64]) / 65.0
    nodes = np.stack([xi, np.full_like(xi, 0.5)], 1)
    exact = closed_form_sin2(xi)
    runs = {}
    for dt, seed in ((1e-3, 51), (1e-4, 52)):
        runs[dt] = ref.interface_estimate(d, B, nodes, 20000, dt, seed)
    q = math.sqrt(10.0)
    m1, m2 = runs[1e-3]["mean"][:, 0], runs[1e-4]["mean"][:, 0]
    s1, s2 = runs[1e-3]["se"][:, 0], runs[1e-4]["se"][:, 0]
    extrap = (q * m2 - m1) / (q - 1)
    se_ex = np.sqrt(q * q * s2**2 + s1**2) / (q - 1)
    z = (extrap - exact) / se_ex
    assert np.all(np.abs(z) <= ZMAX), z
    # the fitted bias coefficient c in m(dt) = X + c sqrt(dt) is O(1)
    c_fit = (m2 - extrap) / math.sqrt(1e-4)
    assert np.all(np.abs(c_fit) < 3.0), c_fit
    # y = eta exactly (the density does not depend on eta)
    zy = (runs[1e-4]["mean"][:, 1] - 0.5) / runs[1e-4]["se"][:, 1]
    assert np.all(np.abs(zy) <= ZMAX), zy
    # the other orientation, int w / int w, is rejected by a wide margin
    wrong = (xi * 2.5 - 3 * np.sin(4 * math.pi * xi) / (8 * math.pi)) / 2.5
    far = np.abs(extrap - wrong) / se_ex
    assert np.max(far) > 20


@pytest.mark.slow
def test_brute_force_finite_differences(ref):
    """MC (Richardson in sqrt(dt)) against the direct FD solve of eq. (5)
    (Richardson in h^2 over 129^2 and 257^2 grids) for the Gaussian density."""
    c = W.cfg_plain_fp64()
    d = c["density"]
    B = ref.Bmap(c["bmap"], d)
    fine = ref.global_solve(d, B, 257, 257)
    coarse = ref.global_solve(d, B, 129, 129)
    jj = np.array([2, 5, 8, 11, 13])
    eta = jj / 16.0
    nodes = np.stack([np.full_like(eta, 0.5), eta], 1)
    fd = (4 * fine[16 * jj, 128] - coarse[8 * jj, 64]) / 3
    assert np.max(np.abs(fine[16 * jj, 128] - coarse[8 * jj, 64])) < 2e-3
    runs = {dt: ref.interface_estimate(d, B, nodes, 20000, dt, s) for dt, s in ((1e-3, 61), (1e-4, 62))}
    q = math.sqrt(10.0)
    m1, m2 = runs[1e-3]["mean"], runs[1e-4]["mean"]
    s1, s2 = runs[1e-3]["se"], runs[1e-4]["se"]
    extrap = (q * m2 - m1) / (q - 1)
    se_ex = np.sqrt(q * q * s2**2 + s1**2) / (q - 1)
    z = (extrap - fd) / se_ex
    assert np.all(np.abs(z) <= ZMAX), z
    assert _chi2_ok(z)


def test_mean_exit_steps_match_torsion(ref):
    """w = 1: E[tau] = v(x0) with Laplace v = -1 (generator Laplace, i.e.
    diffusion sqrt(2)).  Late detection widens the square by
    beta sqrt(2 dt) per side, beta = -zeta(1/2)/sqrt(2 pi) = 0.5826
    (Broadie-Glasserman-Kou continuity correction), and v scales with the
    side squared."""
    dt = 1e-4
    beta = 0.5825971579390106
    delta = beta * math.sqrt(2 * dt)
    side = 1 + 2 * delta

    def predicted_steps(x, y):
        return side**2 * torsion((x + delta) / side, (y + delta) / side) / dt

    for (x, y), seed in (((0.5, 0.5), 71), ((0.2, 0.3), 72), ((0.1, 0.85), 73)):
        r = ref.interface_estimate({"base": 1.0, "terms": []}, {"kind": "identity"}, np.array([[x, y]]),
                                   20000, dt, seed)
        assert r["steps"] / r["paths"] == pytest.approx(predicted_steps(x, y), rel=0.02), (x, y)


def test_maximum_principle_per_path(ref):
    """Every path value lies in the image of the boundary (eq. (7a) averages
    boundary values), for the identity square and the annulus sector."""
    nodes = W.random_nodes(6, 5)
    d = W.random_density(3)
    r = ref.interface_estimate(d, {"kind": "identity"}, nodes, 500, 1e-3, 81, per_path=True)
    pp = r["per_path"]
    e = np.stack([pp["exit_xi"], pp["exit_eta"]], -1)
    assert np.all(e >= 0) and np.all(e <= 1)
    on = (e[..., 0] == 0) | (e[..., 0] == 1) | (e[..., 1] == 0) | (e[..., 1] == 1)
    assert np.all(on)
    assert np.all((r["mean"] > 0) & (r["mean"] < 1))
    ann = {"kind": "annulus", "p": [1.0, 2.0, 0.0, 0.5 * math.pi]}
    r = ref.interface_estimate(d, ann, nodes, 500, 1e-3, 81, per_path=True)
    B = ref.Bmap(ann)
    vals = B.eval(np.stack([r["per_path"]["exit_xi"].ravel(), r["per_path"]["exit_eta"].ravel()], 1),
                  r["per_path"]["side"].ravel())
    rho = np.hypot(vals[:, 0], vals[:, 1])
    assert np.all((rho >= 1 - 1e-14) & (rho <= 2 + 1e-14))
    assert np.all(vals >= -1e-14)
    # per-path values average to the reported mean
    assert np.allclose(vals.reshape(6, 500, 2).mean(1), r["mean"], atol=1e-14)


def test_step_cap_counts_and_projects(ref):
    nodes = np.array([[0.5, 0.5], [0.1, 0.6]])
    dt = 1e-4
    # ceil(2.5) = 3 steps, a whole Philox block: the cap stays 3
    r = ref.interface_estimate({"base": 1.0, "terms": []}, {"kind": "identity"}, nodes, 200, dt, 91,
                               t_max=2.5 * dt, per_path=True)
    pp = r["per_path"]
    assert np.all(pp["steps"] <= 3)
    assert r["capped"] == int(pp["capped"].sum()) > 0
    cap = pp["capped"] == 1
    assert np.all(pp["steps"][cap] == 3)
    # ceil(3.5) = 4 and ceil(4.5) = 5 are rounded up to 6 (blocks of three steps)
    for t in (3.5, 4.5):
        r5 = ref.interface_estimate({"base": 1.0, "terms": []}, {"kind": "identity"}, nodes, 200, dt, 91,
                                    t_max=t * dt, per_path=True)
        assert np.all(r5["per_path"]["steps"][r5["per_path"]["capped"] == 1] == 6)
    # capped paths take the nearest side: from the centre region it is the
    # first side in the order xi=0, xi=1, eta=0, eta=1 only on exact ties
    assert np.all(pp["exit_xi"][1][cap[1]] == 0.0)


def test_path_ranges_and_node_ids_are_additive(ref):
    """Path p always uses counter p, so a run splits into path ranges and node
    subsets without changing any path (Sec. 6: additivity of the expected
    value makes a running estimate resumable)."""
    d = W.random_density(2)
    nodes = W.random_nodes(5, 9)
    full = ref.interface_estimate(d, {"kind": "identity"}, nodes, 300, 1e-3, 7, per_path=True)
    a = ref.interface_estimate(d, {"kind": "identity"}, nodes, 120, 1e-3, 7, per_path=True)
    b = ref.interface_estimate(d, {"kind": "identity"}, nodes, 180, 1e-3, 7, path_begin=120, per_path=True)
    assert np.array_equal(np.concatenate([a["per_path"], b["per_path"]], 1), full["per_path"])
    assert np.allclose(a["sums"] + b["sums"], full["sums"], rtol=1e-14, atol=1e-12)
    sub = ref.interface_estimate(d, {"kind": "identity"}, nodes[[1, 3]], 300, 1e-3, 7,
                                 node_ids=[1, 3], per_path=True)
    assert np.array_equal(sub["per_path"], full["per_path"][[1, 3]])
    assert np.array_equal(sub["mean"], full["mean"][[1, 3]])


def test_float_stepping_agrees_with_double_under_common_numbers(ref):
    """The float walk sees the same uniforms as the double walk; its node
    estimates differ by far less than one standard error."""
    c = W.cfg_plain_fp64()
    nodes = ref.layout_nodes(c["layout"], c["k"])
    r64 = ref.interface_estimate(c["density"], c["bmap"], nodes, 2000, 1e-4, 1, per_path=True)
    r32 = ref.interface_estimate(c["density"], c["bmap"], nodes, 2000, 1e-4, 1, prec="fp32", per_path=True)
    assert np.all(np.abs(r32["mean"] - r64["mean"]) <= 0.5 * r64["se"])
    same = r32["per_path"]["steps"] == r64["per_path"]["steps"]
    assert same.mean() > 0.9


def test_invalid_arguments_are_rejected(ref):
    d = {"base": 1.0, "terms": []}
    with pytest.raises(ValueError):
        ref.interface_estimate(d, {"kind": "identity"}, np.array([[0.0, 0.5]]), 10, 1e-3, 1)
    with pytest.raises(ValueError):
        ref.interface_estimate(d, {"kind": "identity"}, np.array([[0.5, 0.5]]), 10, 0.0, 1)
    with pytest.raises(ValueError):
        ref.interface_estimate(d, {"kind": "identity"}, np.array([[0.5, 1.0]]), 10, 1e-3, 1)
