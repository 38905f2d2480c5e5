"""Pins of the oracle's density terms, boundary maps and exit projection.

The drift of eq. (7b) is grad w / w; the oracle's analytic gradients are
checked against central differences of w itself (an independent route), and
the term values against the points where each term is known in closed form.
The exit point is the first crossing of the last Euler-Maruyama step with
the boundary (Sec. 2.2 tests for exit at the end of each step); hand cases.
"""
import math

import numpy as np
import pytest

import workloads as W

KINDS = [
    {"kind": "gauss", "amp": 5.0, "coef": 50.0, "cx": 0.5, "cy": 0.4},
    {"kind": "ring", "amp": 10.0, "coef": 200.0, "cx": 0.5, "cy": 0.5, "r0": 0.3},
    {"kind": "sech2", "amp": 20.0, "coef": 40.0, "cx": 0.1, "cy": 0.0, "nx": 1.0, "ny": -1.0},
    {"kind": "sin2", "amp": 3.0, "coef": 2 * math.pi, "nx": 1.0, "ny": 0.0},
    {"kind": "sin2", "amp": 2.0, "coef": 5.0, "cx": 0.2, "cy": 0.3, "nx": 0.6, "ny": 0.8},
]


@pytest.mark.parametrize("term", KINDS, ids=[t["kind"] for t in KINDS])
def test_gradient_matches_central_differences(ref, term):
    d = W.density(1.0, [dict({"cx": 0, "cy": 0, "r0": 0, "nx": 0, "ny": 0}, **term)])
    pts = W.random_nodes(2000, 11)
    # keep away from the ring centre, where r is not differentiable
    pts = pts[np.hypot(pts[:, 0] - 0.5, pts[:, 1] - 0.5) > 1e-3]
    w, g = ref.density_eval(d, pts)
    h = 1e-6
    for c in range(2):
        e = np.zeros(2)
        e[c] = h
        wp, _ = ref.density_eval(d, pts + e)
        wm, _ = ref.density_eval(d, pts - e)
        fd = (wp - wm) / (2 * h)
        scale = np.maximum(1.0, np.abs(g[:, c]))
        assert np.max(np.abs(fd - g[:, c]) / scale) < 1e-5


def test_term_values_at_known_points(ref):
    g = W.density(1.0, [KINDS[0]])
    w, grad = ref.density_eval(g, np.array([[0.5, 0.4]]))
    assert w[0] == 6.0 and np.all(grad == 0)
    w, _ = ref.density_eval(g, np.array([[0.6, 0.4]]))
    assert w[0] == pytest.approx(1 + 5 * math.exp(-0.5), rel=1e-15)
    r = W.density(1.0, [KINDS[1]])
    w, grad = ref.density_eval(r, np.array([[0.8, 0.5], [0.5, 0.5]]))
    assert w[0] == pytest.approx(11.0, rel=1e-15)
    assert np.all(grad[1] == 0)          # centre: grad r undefined, taken as 0
    assert w[1] == pytest.approx(1 + 10 * math.exp(-200 * 0.09), rel=1e-13)
    s = W.density(1.0, [KINDS[2]])
    w, _ = ref.density_eval(s, np.array([[0.4, 0.3], [0.4, 0.3 + math.atanh(0.5) / 40]]))
    assert w[0] == pytest.approx(21.0, rel=1e-15)
    assert w[1] == pytest.approx(1 + 20 * 0.75, rel=1e-12)  # sech^2(atanh 1/2) = 3/4
    q = W.density(1.0, [KINDS[3]])
    w, _ = ref.density_eval(q, np.array([[0.25, 0.9], [0.5, 0.1]]))
    assert w[0] == pytest.approx(4.0, rel=1e-15)
    assert w[1] == pytest.approx(1.0, abs=1e-14)


def test_density_is_sum_of_terms(ref):
    d = W.random_density(5, 4)
    pts = W.random_nodes(50, 2)
    w, g = ref.density_eval(d, pts)
    acc_w = np.full(pts.shape[0], -(len(d["terms"]) - 1) * d["base"])
    acc_g = np.zeros_like(pts)
    for t in d["terms"]:
        wt, gt = ref.density_eval(W.density(d["base"], [t]), pts)
        acc_w += wt
        acc_g += gt
    assert np.allclose(w, acc_w, rtol=1e-14, atol=1e-14)
    assert np.allclose(g, acc_g, rtol=1e-13, atol=1e-12)
    assert np.all(w >= d["base"])


@pytest.mark.parametrize("p,q,side,e", [
    ((0.5, 0.5), (-0.5, 0.5), 0, (0.0, 0.5)),
    ((0.5, 0.5), (1.5, 0.7), 1, (1.0, 0.6)),
    ((0.2, 0.1), (0.3, -0.1), 2, (0.25, 0.0)),
    ((0.2, 0.9), (0.4, 1.1), 3, (0.3, 1.0)),
    ((0.1, 0.1), (-0.1, -0.1), 0, (0.0, 0.0)),       # exact corner: tie -> xi=0 first
    ((0.9, 0.9), (1.1, 1.1), 1, (1.0, 1.0)),         # corner tie -> xi=1 before eta=1
    ((0.1, 0.2), (-0.1, -0.6), 2, (0.05, 0.0)),      # eta=0 is crossed first
    ((0.3, 0.4), (0.0, 0.4), 0, (0.0, 0.4)),         # lands exactly on the boundary
    ((0.3, 0.4), (0.3, 1.0), 3, (0.3, 1.0)),
])
def test_exit_point_hand_cases(ref, p, q, side, e):
    s, (ex, ey) = ref.exit_point(p, q)
    assert s == side
    assert ex == pytest.approx(e[0], abs=1e-15) and ey == pytest.approx(e[1], abs=1e-15)
    assert (ex in (0.0, 1.0)) or (ey in (0.0, 1.0))


def test_exit_point_is_on_segment_and_boundary(ref):
    rng = np.random.default_rng(4)
    for _ in range(2000):
        p = rng.uniform(0.01, 0.99, 2)
        q = p + rng.normal(0, 0.3, 2)
        if np.all((q > 0) & (q < 1)):
            continue
        s, (ex, ey) = ref.exit_point(p, q)
        e = np.array([ex, ey])
        assert np.all(e >= 0) and np.all(e <= 1)
        assert [ex == 0, ex == 1, ey == 0, ey == 1][s]
        # collinear with P and Q, and the first boundary crossing
        t = np.dot(e - p, q - p) / np.dot(q - p, q - p)
        assert 0 < t <= 1 + 1e-12
        assert np.linalg.norm(p + t * (q - p) - e) < 1e-12
        for tt in np.linspace(0, t, 20)[:-1]:
            z = p + tt * (q - p)
            assert np.all(z > -1e-12) and np.all(z < 1 + 1e-12)


def test_boundary_maps(ref):
    pts = np.array([[0.0, 0.3], [1.0, 0.6], [0.25, 0.0], [0.75, 1.0], [0.0, 0.0], [1.0, 1.0]])
    side = np.array([0, 1, 2, 3, 0, 1], dtype=np.int32)
    ident = ref.Bmap({"kind": "identity"})
    assert np.array_equal(ident.eval(pts, side), pts)
    aff = ref.Bmap({"kind": "affine", "p": [0.3, 2.0, -0.5, -1.0, 0.25, 3.0]})
    want = np.stack([0.3 + 2 * pts[:, 0] - 0.5 * pts[:, 1], -1 + 0.25 * pts[:, 0] + 3 * pts[:, 1]], 1)
    assert np.allclose(aff.eval(pts, side), want, atol=1e-15)
    ann = ref.Bmap({"kind": "annulus", "p": [1.0, 2.0, 0.0, 0.5 * math.pi]})
    out = ann.eval(pts, side)
    rho = np.hypot(out[:, 0], out[:, 1])
    th = np.arctan2(out[:, 1], out[:, 0])
    assert np.allclose(rho, 1 + pts[:, 0], atol=1e-15)
    assert np.allclose(th, 0.5 * math.pi * pts[:, 1], atol=1e-15)
    # table maps interpolate linearly and agree with the closed-form sides
    n = 9
    tab = np.zeros((4, n, 2))
    s = np.arange(n) / (n - 1)
    tab[0] = np.stack([np.zeros(n), s**2], 1)
    tab[1] = np.stack([np.ones(n), s], 1)
    tab[2] = np.stack([s, np.zeros(n)], 1)
    tab[3] = np.stack([s**2, np.ones(n)], 1)
    T = ref.Bmap({"kind": "table", "table": tab})
    out = T.eval(np.array([[0.0, 0.5], [0.0, 0.5625], [0.5, 1.0], [0.5625, 1.0]]), np.array([0, 0, 3, 3], np.int32))
    assert np.allclose(out[:, 1][:2], [0.25, (0.25 + 0.390625) / 2], atol=1e-15)
    assert np.allclose(out[:, 0][2:], [0.25, (0.25 + 0.390625) / 2], atol=1e-15)
