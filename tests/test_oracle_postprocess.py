"""Pins of the oracle's mesh quality measure (eq. (11), Sec. 3.1 and 3.3),
Perona-Malik smoothing (eq. (12), Sec. 3.4-3.5) and interface pre-smoothing
by local quadratic regression (Sec. 4).

Quality: a hand-worked cell, closed forms for affine maps (stretch, shear,
rotation), the bound Q >= 1 with equality exactly for conformal cells,
O(h^2) convergence to the analytic Q of a smooth map, folds, invariances.
Smoothing: with c = 1 the scheme is the FTCS heat step, whose sine modes
decay by a known factor per step; affine meshes are fixed points; no flux
crosses a sharp jump under a small k while a large k diffuses it; the maximum
principle under the stability bound; per-subdomain smoothing equals
smoothing each subdomain cut out on its own.
Local regression: quadratics reproduced exactly, agreement with numpy's
independent weighted polynomial fit, fixed points kept, reversal symmetry,
noise reduction.
"""
import math

import numpy as np
import pytest


def grid(nx, ny):
    xi, eta = np.meshgrid(np.linspace(0, 1, nx), np.linspace(0, 1, ny))
    return np.stack([xi, eta], -1)


def affine(A, b, nx, ny):
    g = grid(nx, ny)
    return g @ np.asarray(A, dtype=float).T + np.asarray(b, dtype=float)


# ---------------------------------------------------------------- quality

def test_quality_hand_worked_cell(ref):
    # one cell, corners (0,0), (2,0), (0,1), (2,1) on a 2 x 2 grid (h = 1):
    # J = diag(2, 1), tr(J^T J) = 5, det(J^T J) = 4, Q = 5 / (2 * 2) = 1.25
    mesh = np.array([[[0.0, 0.0], [2.0, 0.0]], [[0.0, 1.0], [2.0, 1.0]]])
    r = ref.mesh_quality(mesh)
    assert r["q"].shape == (1, 1)
    assert r["q_max"] == pytest.approx(1.25, abs=1e-15) and r["folded"] == 0


@pytest.mark.parametrize("A,Q", [
    ([[1, 0], [0, 1]], 1.0),
    ([[3, 0], [0, 0.5]], (9 + 0.25) / (2 * 1.5)),          # stretch (a^2 + b^2) / (2ab)
    ([[1, 0.7], [0, 1]], (2 + 0.49) / 2),                   # shear (2 + s^2) / 2
    ([[0.8, -0.6], [0.6, 0.8]], 1.0),                       # rotation
    ([[2 * 0.8, -2 * 0.6], [2 * 0.6, 2 * 0.8]], 1.0),       # rotation and scale
])
def test_quality_of_affine_maps(ref, A, Q):
    # non-square grid, so that a swapped h_xi / h_eta or a transposed J shows
    r = ref.mesh_quality(affine(A, [0.3, -0.2], 9, 5))
    assert np.allclose(r["q"], Q, rtol=1e-13, atol=0)
    assert r["folded"] == 0


def test_quality_bound_and_equality(ref):
    rng = np.random.default_rng(0)
    m = grid(17, 13)
    m[1:-1, 1:-1] += rng.normal(0, 0.01, size=m[1:-1, 1:-1].shape)
    r = ref.mesh_quality(m)
    assert np.all(r["q"] >= 1.0 - 1e-14) and r["q_max"] > 1.0
    # conformal cells (J a multiple of a rotation) and only those give Q = 1
    J = ref.cell_jacobians(m)
    conformal = np.isclose(J[..., 0, 0], J[..., 1, 1], rtol=0, atol=1e-12) & \
        np.isclose(J[..., 0, 1], -J[..., 1, 0], rtol=0, atol=1e-12)
    assert not conformal.any() and np.all(r["q"] > 1.0)


def test_quality_converges_to_the_smooth_map_at_second_order(ref):
    def smooth_map(n):
        g = grid(n, n)
        xi, eta = g[..., 0], g[..., 1]
        return np.stack([xi + 0.05 * np.sin(np.pi * xi) * np.sin(2 * np.pi * eta),
                         eta + 0.04 * np.sin(2 * np.pi * xi) * np.sin(np.pi * eta)], -1)

    def analytic_q(n):
        c = (np.arange(n - 1) + 0.5) / (n - 1)
        xi, eta = np.meshgrid(c, c)
        J = np.empty(xi.shape + (2, 2))
        J[..., 0, 0] = 1 + 0.05 * np.pi * np.cos(np.pi * xi) * np.sin(2 * np.pi * eta)
        J[..., 0, 1] = 0.05 * 2 * np.pi * np.sin(np.pi * xi) * np.cos(2 * np.pi * eta)
        J[..., 1, 0] = 0.04 * 2 * np.pi * np.cos(2 * np.pi * xi) * np.sin(np.pi * eta)
        J[..., 1, 1] = 1 + 0.04 * np.pi * np.sin(2 * np.pi * xi) * np.cos(np.pi * eta)
        fro = (J**2).sum((-1, -2))
        det = J[..., 0, 0] * J[..., 1, 1] - J[..., 0, 1] * J[..., 1, 0]
        return 0.5 * fro / np.abs(det)

    err = [np.abs(ref.mesh_quality(smooth_map(n))["q"] - analytic_q(n)).max() for n in (33, 65, 129)]
    ratios = [err[0] / err[1], err[1] / err[2]]
    assert all(3.6 < q < 4.4 for q in ratios), (err, ratios)


def test_quality_invariances_and_folds(ref):
    rng = np.random.default_rng(1)
    m = grid(11, 11)
    m[1:-1, 1:-1] += rng.normal(0, 0.01, size=m[1:-1, 1:-1].shape)
    q = ref.mesh_quality(m)["q"]
    R = np.array([[math.cos(0.7), -math.sin(0.7)], [math.sin(0.7), math.cos(0.7)]])
    assert np.allclose(ref.mesh_quality(3.0 * m @ R.T + 1.0)["q"], q, rtol=1e-12)
    mirrored = m * np.array([-1.0, 1.0])
    r = ref.mesh_quality(mirrored)
    assert np.allclose(r["q"], q, rtol=1e-12) and r["folded"] == q.size
    # a node pushed across its neighbour folds the cells around it
    f = m.copy()
    f[5, 5, 0] = f[5, 7, 0] + 0.05
    assert ref.mesh_quality(f)["folded"] >= 1
    # a cell whose Jacobian columns are parallel is degenerate: Q = inf, folded
    c = np.array([[[0.0, 0.0], [1.0, 0.0]], [[1.0, 0.0], [2.0, 0.0]]])
    r = ref.mesh_quality(c)
    assert r["q_max"] == np.inf and r["folded"] == 1
    # a cell collapsed to a point (J = 0, Q = 0/0) is degenerate too
    p = np.full((2, 2, 2), 0.3)
    r = ref.mesh_quality(p)
    assert r["q"][0, 0] == np.inf and r["q_max"] == np.inf and r["folded"] == 1


def test_compare(ref):
    d = {"base": 1.0, "terms": [{"kind": "gauss", "amp": 4.0, "coef": 30.0, "cx": 0.4, "cy": 0.6}]}
    m = grid(9, 9)
    r = ref.mesh_compare(m, m, d)
    assert r["linf"] == 0.0 and r["max_disp"] == 0.0
    n = m.copy()
    n[3, 4] += np.array([0.03, -0.04])
    r = ref.mesh_compare(n, m, d)
    w, _ = ref.density_eval(d, np.array([n[3, 4], m[3, 4]]))
    assert r["max_disp"] == pytest.approx(0.05, rel=1e-12)
    assert r["linf"] == pytest.approx(abs(w[0] - w[1]), rel=1e-12)


# ------------------------------------------------------------ Perona-Malik

@pytest.mark.parametrize("nx,ny,m,n", [(33, 17, 1, 1), (33, 17, 3, 2), (21, 41, 2, 5)])
def test_smoothing_with_unit_coefficient_is_the_discrete_heat_step(ref, nx, ny, m, n):
    g = grid(nx, ny)
    eps = 1e-3
    mode = np.sin(m * np.pi * g[..., 0]) * np.sin(n * np.pi * g[..., 1])
    mesh = g.copy()
    mesh[..., 0] += eps * mode
    mesh[..., 1] -= 0.5 * eps * mode
    hx, hy = 1.0 / (nx - 1), 1.0 / (ny - 1)
    dt = 0.2 / (1 / hx**2 + 1 / hy**2)
    steps = 7
    out = ref.perona_malik(mesh, dt, 1e12, steps)
    gain = 1 - 4 * dt * (math.sin(m * math.pi * hx / 2) ** 2 / hx**2 + math.sin(n * math.pi * hy / 2) ** 2 / hy**2)
    assert np.allclose(out[..., 0] - g[..., 0], eps * gain**steps * mode, rtol=0, atol=1e-15)
    assert np.allclose(out[..., 1] - g[..., 1], -0.5 * eps * gain**steps * mode, rtol=0, atol=1e-15)


def test_affine_meshes_are_fixed_points(ref):
    m = affine([[1.3, 0.2], [-0.1, 0.9]], [0.1, 0.2], 17, 25)
    for k in (0.5, 3.0, 1000.0):
        out = ref.perona_malik(m, 1e-5, k, 10)
        assert np.abs(out - m).max() < 1e-14


def test_no_flux_across_a_sharp_jump_under_small_k(ref):
    # a jump of H between columns 16 and 17: with k = 1 the face coefficient
    # across it is exp(-(H/h)^2) < 1e-17, so the left half evolves as if the
    # right half were not there (changing H changes nothing on the left);
    # with k = 1000 the jump diffuses and the left half feels H.
    nx = ny = 33
    dt = 0.2 / (2 * (nx - 1) ** 2)

    def run(H, k):
        m = grid(nx, ny)
        m[:, 17:, 0] += H
        return ref.perona_malik(m, dt, k, 20)

    left = (slice(None), slice(0, 17), 0)
    assert np.abs(run(0.2, 1.0)[left] - run(0.3, 1.0)[left]).max() < 1e-15
    assert np.abs(run(0.2, 1000.0)[left] - run(0.3, 1000.0)[left]).max() > 1e-3


def test_homogeneity_in_the_mesh_scale_and_k(ref):
    # c depends on |grad u| / k only: scaling the mesh and k by alpha scales the
    # result by alpha, in the nonlinear regime (c between 0.1 and 0.9 here)
    rng = np.random.default_rng(7)
    m = grid(21, 21)
    m[1:-1, 1:-1] += rng.normal(0, 0.03, size=m[1:-1, 1:-1].shape)
    a = ref.perona_malik(m, 2e-4, 1.5, 4)
    b = ref.perona_malik(3.0 * m, 2e-4, 4.5, 4)
    assert np.allclose(b, 3.0 * a, rtol=0, atol=1e-13)
    assert np.abs(a - ref.perona_malik(m, 2e-4, 1e9, 4)).max() > 1e-3    # and c matters at k = 1.5


def test_maximum_principle_and_fixed_nodes(ref):
    rng = np.random.default_rng(2)
    nx, ny = 25, 19
    m = grid(nx, ny)
    m[1:-1, 1:-1] += rng.normal(0, 0.02, size=m[1:-1, 1:-1].shape)
    dt = 1.0 / (2 * (nx - 1) ** 2 + 2 * (ny - 1) ** 2)
    assert ref.ftcs_stable(nx, ny, dt) and not ref.ftcs_stable(nx, ny, 1.01 * dt)
    out = ref.perona_malik(m, dt, 2.0, 1)
    P = m[1:-1, 1:-1]
    nb = np.stack([m[1:-1, 2:], m[1:-1, :-2], m[2:, 1:-1], m[:-2, 1:-1], P])
    assert np.all(out[1:-1, 1:-1] <= nb.max(0) + 1e-15) and np.all(out[1:-1, 1:-1] >= nb.min(0) - 1e-15)
    f = ref.fixed_nodes(nx, ny)
    assert np.array_equal(out[f], m[f])


def test_per_subdomain_smoothing_is_each_subdomain_alone(ref):
    # 33 x 33 nodes in 4 x 4 subdomains of 9 x 9: a cut-out has h = 1/8, the
    # full grid h = 1/32.  Smoothing a cut-out on its own with dt x 16 and
    # k / 4 performs the same arithmetic (powers of two), so every subdomain
    # of the per-subdomain result must equal its cut-out smoothed alone.
    rng = np.random.default_rng(3)
    L = {"nx": 33, "ny": 33, "sx": 4, "sy": 4}
    m = grid(33, 33)
    m[1:-1, 1:-1] += rng.normal(0, 0.01, size=m[1:-1, 1:-1].shape)
    dt, k, steps = 1e-4 / 16, 5.0, 6
    out = ref.perona_malik(m, dt, k, steps, L)
    for b in range(4):
        for a in range(4):
            sub = m[8 * b:8 * b + 9, 8 * a:8 * a + 9]
            alone = ref.perona_malik(sub, dt * 16, k / 4, steps)
            assert np.array_equal(out[8 * b:8 * b + 9, 8 * a:8 * a + 9], alone)
    f = ref.fixed_nodes(33, 33, L)
    assert np.array_equal(out[f], m[f])
    glob = ref.perona_malik(m, dt, k, steps)
    assert not np.array_equal(glob[f], m[f])      # smoothing the whole grid moves the interfaces


def test_smoothing_commutes_with_transposition(ref):
    rng = np.random.default_rng(4)
    m = grid(21, 21)
    m[1:-1, 1:-1] += rng.normal(0, 0.01, size=m[1:-1, 1:-1].shape)
    t = np.transpose(m, (1, 0, 2))[..., ::-1]
    a = ref.perona_malik(m, 2e-4, 3.0, 5)
    b = ref.perona_malik(t, 2e-4, 3.0, 5)
    assert np.allclose(np.transpose(b, (1, 0, 2))[..., ::-1], a, rtol=0, atol=1e-15)


# ------------------------------------------------------ local regression

def test_local_regression_reproduces_quadratics(ref):
    n = 41
    s = np.arange(n) / (n - 1)
    v = np.stack([0.3 + 0.2 * s - 0.7 * s**2, 1 - 2 * s + 0.1 * s**2], 1)
    fixed = np.zeros(n, dtype=bool)
    fixed[[0, 20, 40]] = True
    for span in (5, 7, 11):
        assert np.abs(ref.loess_line(v, s, fixed, span) - v).max() < 1e-13


def test_local_regression_against_numpy_weighted_polyfit(ref):
    rng = np.random.default_rng(5)
    n, span = 33, 9
    s = np.arange(n) / (n - 1)
    v = rng.normal(size=(n, 2))
    fixed = np.zeros(n, dtype=bool)
    out = ref.loess_line(v, s, fixed, span)
    for i in (0, 2, 16, 30, 32):
        a = min(max(i - span // 2, 0), n - span)
        t = s[a:a + span] - s[i]
        d = np.abs(t).max()
        w = (1 - (np.abs(t) / d) ** 3) ** 3
        for c in range(2):
            p = np.polyfit(t, v[a:a + span, c], 2, w=np.sqrt(w))
            assert out[i, c] == pytest.approx(np.polyval(p, 0.0), abs=1e-12)


def test_local_regression_fixed_points_symmetry_and_noise(ref):
    rng = np.random.default_rng(6)
    L = {"nx": 65, "ny": 49, "sx": 4, "sy": 3}
    ny, nx = 49, 65
    sv, sh = np.arange(ny) / (ny - 1), np.arange(nx) / (nx - 1)
    clean_v = np.stack([np.full(ny, 0.25), sv + 0.1 * np.sin(np.pi * sv)], 1)
    vert = np.stack([clean_v + rng.normal(0, 0.01, size=(ny, 2)) for _ in range(3)])
    horiz = np.stack([np.stack([sh, np.full(nx, 1 / 3)], 1) + rng.normal(0, 0.01, size=(nx, 2)) for _ in range(2)])
    v2, h2 = ref.smooth_interfaces(L, vert, horiz, 9)
    for a in range(3):
        assert np.array_equal(v2[a, ::16], vert[a, ::16])       # ends and crosspoints
    for b in range(2):
        assert np.array_equal(h2[b, ::16], horiz[b, ::16])
    rough = lambda u: np.sum(np.diff(u, 2, axis=0) ** 2)
    assert rough(v2[0]) < 0.1 * rough(vert[0])
    assert np.abs(v2[0] - clean_v)[1:-1].mean() < 0.8 * np.abs(vert[0] - clean_v)[1:-1].mean()
    # reversing the line commutes with smoothing (odd span)
    fixed = np.zeros(ny, dtype=bool)
    fixed[::16] = True
    fwd = ref.loess_line(vert[1], sv, fixed, 9)
    bwd = ref.loess_line(vert[1][::-1], sv, fixed[::-1], 9)[::-1]
    assert np.allclose(fwd, bwd, rtol=0, atol=1e-13)


def test_shifted_cycle_moves_the_original_interfaces(ref):
    # the shifted cycle fixes the lines half a subdomain away, so the original
    # interface lines are smoothed; a cut-out shifted subdomain smoothed alone
    # (dt x 16, k / 4 as above) equals its part of the result
    rng = np.random.default_rng(8)
    L = {"nx": 33, "ny": 33, "sx": 4, "sy": 4}
    m = grid(33, 33)
    m[1:-1, 1:-1] += rng.normal(0, 0.01, size=m[1:-1, 1:-1].shape)
    dt, k, steps = 1e-4 / 16, 5.0, 4
    out = ref.perona_malik(m, dt, k, steps, L, shifted=True)
    f = ref.fixed_nodes(33, 33, L, shifted=True)
    assert np.array_equal(out[f], m[f])
    orig = ref.fixed_nodes(33, 33, L) & ~ref.fixed_nodes(33, 33)
    assert not np.array_equal(out[orig], m[orig])
    sub = m[4:13, 12:21]                     # the shifted subdomain around the crosspoint (8, 16)
    alone = ref.perona_malik(sub, dt * 16, k / 4, steps)
    assert np.array_equal(out[4:13, 12:21], alone)
