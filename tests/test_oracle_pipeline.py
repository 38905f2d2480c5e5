"""Pins of the oracle's deterministic parts: edge data, node placement,
interface fill and the finite-difference subdomain solves (Sec. 2.1 Fig. 1,
Sec. 3.2, Sec. 3.6).
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.interpolate import PchipInterpolator

import workloads as W
from tests.test_oracle_walk import closed_form_sin2

ONE = {"base": 1.0, "terms": []}


def test_edge1d_table_closed_form(ref):
    d = W.cfg_sin2_sweep()["density"]
    n = 4097
    tab = ref.edge1d_table(d, n)
    s = np.arange(n) / (n - 1)
    # eta = 0 and eta = 1 sides: x = int_0^xi 1/w / int_0^1 1/w
    assert np.max(np.abs(tab[2, :, 0] - closed_form_sin2(s))) < 1e-12
    assert np.max(np.abs(tab[3, :, 0] - closed_form_sin2(s))) < 1e-12
    assert np.all(tab[2, :, 1] == 0) and np.all(tab[3, :, 1] == 1)
    # xi = 0 and xi = 1 sides: w is constant along them, so y = eta
    assert np.max(np.abs(tab[0, :, 1] - s)) < 1e-14 and np.all(tab[0, :, 0] == 0)
    assert np.max(np.abs(tab[1, :, 1] - s)) < 1e-14 and np.all(tab[1, :, 0] == 1)


def test_edge1d_table_general_density_is_monotone_and_continuous(ref):
    d = W.random_density(8)
    tab = ref.edge1d_table(d, 257)
    for side in range(4):
        c = 1 if side < 2 else 0
        assert np.all(np.diff(tab[side, :, c]) > 0)
        assert tab[side, 0, c] == 0 and tab[side, -1, c] == 1
    # corners agree between the two sides that meet there
    assert np.allclose(tab[0, 0], tab[2, 0]) and np.allclose(tab[0, -1], tab[3, 0])
    assert np.allclose(tab[1, 0], tab[2, -1]) and np.allclose(tab[1, -1], tab[3, -1])
    # against adaptive quadrature on one side
    s = 0.37
    f = lambda t: 1.0 / ref.density_eval(d, np.array([[t, 0.0]]))[0][0]
    num = integrate.quad(f, 0, s, epsabs=1e-13)[0] / integrate.quad(f, 0, 1, epsabs=1e-13)[0]
    B = ref.Bmap({"kind": "table", "table": ref.edge1d_table(d, 4097)})
    got = B.eval(np.array([[s, 0.0]]), np.array([2], np.int32))[0, 0]
    assert got == pytest.approx(num, abs=1e-6)


@pytest.mark.parametrize("seed", range(6))
def test_pchip_matches_scipy(ref, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 40))
    t = np.sort(rng.uniform(0, 1, n))
    t[0], t[-1] = 0.0, 1.0
    v = rng.normal(size=n).cumsum() if seed % 2 else rng.normal(size=n)
    if seed == 4:
        v[3:7] = v[3]                   # flat run
    if seed == 5:
        v = np.tanh(10 * (t - 0.5))     # monotone data
    te = np.sort(rng.uniform(0, 1, 500))
    got = ref.interp_segment(t, v, te, "pchip")
    want = PchipInterpolator(t, v)(te)
    assert np.max(np.abs(got - want)) < 1e-12 * max(1.0, np.abs(v).max())
    if seed == 5:
        assert np.all(np.diff(got) >= -1e-15)   # monotone data stays monotone


def test_pchip_two_points_is_linear_and_reproduces_knots(ref):
    t = np.array([0.0, 0.3, 0.5, 1.0])
    v = np.array([0.0, 1.0, 0.2, 0.4])
    assert np.array_equal(ref.interp_segment(t, v, t, "pchip"), v)
    assert np.array_equal(ref.interp_segment(t, v, t, "linear"), v)
    te = np.linspace(0, 1, 11)
    assert np.allclose(ref.interp_segment(t[[0, 3]], v[[0, 3]], te, "pchip"), 0.4 * te, atol=1e-16)
    assert np.allclose(ref.interp_segment(t, v, te, "linear"), np.interp(te, t, v), atol=1e-16)


def test_layout_node_counts(ref):
    assert ref.node_count(W.cfg_plain_fp64()["layout"], 15) == 15
    assert ref.node_count(W.cfg_ring_fp32()["layout"], 63) == 1521
    assert ref.node_count(W.cfg_annulus_fp32()["layout"], 32) == 3633
    nodes = ref.layout_nodes(W.cfg_ring_fp32()["layout"], 63)
    assert nodes.shape == (1521, 2)
    # every interior interface node of the 257^2 grid, each once
    ij = np.rint(nodes * 256).astype(int)
    assert np.array_equal(ij / 256.0, nodes)
    assert len({tuple(p) for p in ij}) == 1521
    assert np.all((ij[:, 0] % 64 == 0) | (ij[:, 1] % 64 == 0))


def test_uniform_placement_is_the_paper_layout(ref):
    nodes = ref.layout_nodes(W.cfg_plain_fp64()["layout"], 15)
    assert np.array_equal(nodes[:, 0], np.full(15, 0.5))
    assert np.array_equal(nodes[:, 1], np.arange(1, 16) / 16.0)


def test_equidistributed_placement(ref):
    L = {"nx": 17, "ny": 17, "sx": 2, "sy": 2}
    # constant w: uniform points
    eq = ref.layout_nodes(L, 5, "equidistributed", {"base": 3.0, "terms": []})
    un = ref.layout_nodes(L, 5, "uniform")
    assert np.max(np.abs(eq - un)) < 1e-13
    # shear layer: equal integral of w between consecutive points
    d = W.cfg_annulus_fp32()["density"]
    eq = ref.layout_nodes(L, 6, "equidistributed", d)
    seg = eq[1:1 + 6]                      # first vertical segment, xi = 1/2, eta in (0, 1/2)
    assert np.all(seg[:, 0] == 0.5)
    t = np.concatenate([[0.0], seg[:, 1], [0.5]])
    assert np.all(np.diff(t) > 0)
    w = lambda e: ref.density_eval(d, np.array([[0.5, e]]))[0][0]
    parts = [integrate.quad(w, a, b, epsabs=1e-12, limit=200)[0] for a, b in zip(t[:-1], t[1:])]
    # the inversion is linear inside a panel of width 1/8192: O(h^2 |w'|) error
    assert np.max(np.abs(np.array(parts) / np.mean(parts) - 1)) < 2e-5
    # points crowd where w is large (near eta = xi = 1/2)
    assert np.diff(t)[-1] < np.diff(t)[0]


@pytest.mark.parametrize("interp", ["linear", "pchip"])
def test_fill_with_exact_linear_data_is_exact(ref, interp):
    """Identity map and exact estimates: every interface value equals its
    mesh position (both interpolants reproduce linear data)."""
    for L, k, place in (({"nx": 65, "ny": 33, "sx": 2, "sy": 1}, 15, "uniform"),
                        ({"nx": 41, "ny": 41, "sx": 4, "sy": 4}, 3, "uniform"),
                        ({"nx": 33, "ny": 25, "sx": 2, "sy": 3}, 4, "equidistributed")):
        nodes = ref.layout_nodes(L, k, place, W.cfg_annulus_fp32()["density"])
        vert, horiz = ref.fill_interfaces(L, k, {"kind": "identity"}, nodes, nodes, interp)
        nx, ny, sx, sy = L["nx"], L["ny"], L["sx"], L["sy"]
        for a in range(1, sx):
            want = np.stack([np.full(ny, a / sx), np.arange(ny) / (ny - 1)], 1)
            assert np.max(np.abs(vert[a - 1] - want)) < 1e-15
        for b in range(1, sy):
            want = np.stack([np.arange(nx) / (nx - 1), np.full(nx, b / sy)], 1)
            assert np.max(np.abs(horiz[b - 1] - want)) < 1e-15


def test_fd_is_exact_for_affine_data_and_constant_w(ref):
    for bm in ({"kind": "identity"}, {"kind": "affine", "p": [0.3, 2.0, -0.5, -1.0, 0.25, 3.0]}):
        mesh = ref.global_solve({"base": 2.0, "terms": []}, bm, 23, 17)
        xi, eta = np.meshgrid(np.arange(23) / 22, np.arange(17) / 16, indexing="xy")
        want = ref.Bmap(bm).eval(np.stack([xi.ravel(), eta.ravel()], 1), np.zeros(xi.size, np.int32))
        assert np.max(np.abs(mesh.reshape(-1, 2) - want)) < 1e-13


def test_fd_one_dimensional_density_gives_the_discrete_1d_solution(ref):
    """w = w(xi): with boundary data U_i from the discrete 1D equation
    (w_{i+1/2}(U_{i+1}-U_i) = const, i.e. U_i = sum_{m<i} 1/w_{m+1/2} / sum 1/w),
    the 2D solution is U_i on every row and y = eta exactly."""
    d = W.cfg_sin2_sweep()["density"]
    nx, ny = 41, 21
    wm = ref.density_eval(d, np.stack([(np.arange(nx - 1) + 0.5) / (nx - 1), np.zeros(nx - 1)], 1))[0]
    U = np.concatenate([[0.0], np.cumsum(1.0 / wm)]) / np.sum(1.0 / wm)
    frame = np.zeros((ny, nx, 2))
    frame[:, :, 0] = U[None, :]
    frame[:, :, 1] = (np.arange(ny) / (ny - 1))[:, None]
    blk = ref.dirichlet_solve(d, nx, ny, 0, nx - 1, 0, ny - 1, frame)
    assert np.max(np.abs(blk[:, :, 0] - U[None, :])) < 1e-13
    assert np.max(np.abs(blk[:, :, 1] - frame[:, :, 1])) < 1e-13


def test_fd_converges_to_closed_form_at_second_order(ref):
    c = W.cfg_sin2_sweep()
    errs = []
    for n in (33, 65):
        mesh = ref.global_solve(c["density"], ref.Bmap(c["bmap"], c["density"]), n, n)
        xi = np.arange(n) / (n - 1)
        errs.append(np.max(np.abs(mesh[(n - 1) // 2, :, 0] - closed_form_sin2(xi))))
    assert errs[1] < errs[0] / 3.2 and errs[1] < 2e-3


def test_decomposition_with_exact_interfaces_reproduces_global_solve(ref):
    """Non-iterative DD (Sec. 2.1): exact interface values make the
    independent subdomain solves reproduce the single-domain solution."""
    d = W.random_density(4)
    B = ref.Bmap({"kind": "annulus", "p": [1.0, 2.0, 0.0, 0.5 * math.pi]})
    L = {"nx": 33, "ny": 25, "sx": 4, "sy": 3}
    g = ref.global_solve(d, B, 33, 25)
    vert = np.stack([g[:, 8 * a] for a in range(1, 4)])
    horiz = np.stack([g[8 * b, :] for b in range(1, 3)])
    mesh = ref.subdomain_solve(d, B, L, vert, horiz)
    assert np.max(np.abs(mesh - g)) < 1e-12


def _min_cell_jacobian(mesh):
    x, y = mesh[..., 0], mesh[..., 1]
    dxx = x[:-1, 1:] - x[:-1, :-1]
    dyx = y[:-1, 1:] - y[:-1, :-1]
    dxy = x[1:, :-1] - x[:-1, :-1]
    dyy = y[1:, :-1] - y[:-1, :-1]
    return (dxx * dyy - dxy * dyx).min()


def test_pipeline_small_workload_gives_a_valid_mesh(ref):
    c = W.cfg_plain_fp64()
    out = ref.pipeline(c)
    mesh = out["mesh"]
    assert mesh.shape == (33, 65, 2)
    assert np.all(np.isfinite(mesh))
    # at 2000 paths the standard error (~0.005) matches the smallest mesh
    # spacing near the bump centre, so a cell may fold there (the paper's
    # point that small N gives poor meshes); with 8x the paths none does
    many = dict(c, paths=16000)
    assert _min_cell_jacobian(ref.pipeline(many)["mesh"]) > 0
    # the interface column carries the filled estimates
    assert np.array_equal(mesh[2::2, 32][:15], out["est"]["mean"])
    # and lies within MC error of the brute-force solution on the same grid
    g = ref.global_solve(c["density"], ref.Bmap(c["bmap"]), 65, 33)
    assert np.max(np.abs(mesh - g)) < 0.05


def test_grid_nodes_and_assembly(ref):
    nodes = ref.grid_nodes(6, 5)
    assert nodes.shape == (4 * 3, 2)
    # row by row: eta outer, xi inner, interior only
    assert np.array_equal(nodes[:4, 0], np.arange(1, 5) / 5) and np.all(nodes[:4, 1] == 1 / 4)
    assert np.array_equal(nodes[4:8, 1], np.full(4, 2 / 4))
    B = ref.Bmap({"kind": "annulus", "p": [1.0, 2.0, 0.0, 0.5 * math.pi]})
    vals = np.arange(24, dtype=float).reshape(12, 2)
    mesh = ref.assemble_mesh(B, 6, 5, vals)
    frame = ref.boundary_frame(B, 6, 5)
    ring = np.ones((5, 6), dtype=bool)
    ring[1:-1, 1:-1] = False
    assert np.array_equal(mesh[ring], frame[ring])
    assert np.array_equal(mesh[1:-1, 1:-1].reshape(-1, 2), vals)


def test_whole_grid_mesh_of_constant_density_is_the_identity(ref):
    # w = 1 and the identity map: x = xi, y = eta exactly; the bridge walk's
    # bias is O(dt), so the Monte Carlo mesh is within 4 SE + 4 dt of the grid
    cfg = {"density": {"base": 1.0, "terms": []}, "bmap": {"kind": "identity"},
           "layout": {"nx": 9, "ny": 7, "sx": 1, "sy": 1}, "paths": 4000, "dt": 1e-4, "seed": 3,
           "exit_test": "bridge"}
    r = ref.probabilistic_mesh(cfg)
    exact = ref.grid_nodes(9, 7)
    err = np.abs(r["est"]["mean"] - exact)
    assert np.all(err <= 4 * r["est"]["se"] + 4e-4)
    m = r["mesh"]
    assert np.allclose(m[0, :, 0], np.arange(9) / 8) and np.allclose(m[:, 0, 1], np.arange(7) / 6)


def test_extrema_of_a_gaussian_crossing_the_line(ref):
    # w = 1 + A exp(-c((xi - 0.3)^2 + (eta - 0.55)^2)) along the vertical line
    # xi = 0.3: f = exp(-c u^2), u = eta - 0.55; f' has extrema at
    # u^2 = 1/(2c), f'' at u = 0 and u^2 = 3/(2c)
    c = 60.0
    d = {"base": 1.0, "terms": [{"kind": "gauss", "amp": 5.0, "coef": c, "cx": 0.3, "cy": 0.55}]}
    t = ref.extrema_params(d, 0.3, True, 0.0, 1.0)
    u1, u2 = 1 / math.sqrt(2 * c), math.sqrt(3 / (2 * c))
    want = np.sort(0.55 + np.array([-u2, -u1, 0.0, u1, u2]))
    assert t.shape == (5,)
    assert np.abs(t - want).max() < 1e-6
    # the same bump along a horizontal line through its centre
    t = ref.extrema_params(d, 0.55, False, 0.0, 1.0)
    assert np.abs(t - np.sort(0.3 + np.array([-u2, -u1, 0.0, u1, u2]))).max() < 1e-6
    # restricted to a segment, only the extrema inside it
    t = ref.extrema_params(d, 0.3, True, 0.5, 1.0)
    assert np.abs(t - want[want > 0.5]).max() < 1e-6


def test_extrema_of_sin2_and_of_a_constant(ref):
    # w = 1 + 3 sin^2(2 pi xi): w_xi = 6 pi sin(4 pi xi) has extrema at 1/8, 3/8;
    # w_xixi = 24 pi^2 cos(4 pi xi) at 1/4 (0 and 1/2 are the segment ends)
    d = {"base": 1.0, "terms": [{"kind": "sin2", "amp": 3.0, "coef": 2 * math.pi, "nx": 1.0, "ny": 0.0}]}
    t = ref.extrema_params(d, 0.5, False, 0.0, 0.5)
    assert np.abs(t - np.array([0.125, 0.25, 0.375])).max() < 1e-7
    flat = {"base": 2.0, "terms": []}
    assert ref.extrema_params(flat, 0.5, True, 0.0, 1.0).size == 0


def test_extrema_layout_and_fill_with_counts(ref):
    d = {"base": 1.0, "terms": [{"kind": "gauss", "amp": 5.0, "coef": 60.0, "cx": 0.3, "cy": 0.55}]}
    L = {"nx": 33, "ny": 33, "sx": 2, "sy": 2}
    nodes, counts = ref.layout_nodes_extrema(L, d, 4)
    assert nodes.shape == (1 + 4 * 4, 2) and counts.shape == (4,)
    # the vertical line xi = 1/2 is 0.2 from the bump centre: its extrema
    # split between the two segments; unused slots are off the square
    for s in range(4):
        k = min(counts[s], 4)
        slot = nodes[1 + 4 * s: 1 + 4 * s + 4]
        assert np.all(slot[k:] == -1.0) and np.all((slot[:k] > 0) & (slot[:k] < 1))
    # linear data along the lines are reproduced by the fill whatever the counts
    vals = np.where(nodes >= 0, 0.3 + 0.2 * nodes, np.nan)
    vert, horiz = ref.fill_interfaces(L, 4, {"kind": "affine", "p": [0.3, 0.2, 0.0, 0.0, 0.0, 0.2]}, nodes,
                                      vals * np.array([1.0, 1.0]) + np.array([0.0, -0.3]), "pchip",
                                      counts=counts)
    eta = np.arange(33) / 32
    assert np.allclose(vert[0, :, 0], 0.3 + 0.2 * 0.5) and np.allclose(vert[0, :, 1], 0.2 * eta)
    assert np.all(np.isfinite(horiz))
