"""GPU parity of mesh quality and smoothing against the oracle.

* quality (eq. (11)): every cell's Q within 1e-12 relative, Q_max and
  Q_mean within 1e-12, folded counts equal; ragged and large grids;
* l_inf and displacement (Sec. 3.3) within 1e-13 relative;
* Perona-Malik FTCS (eq. (12)), per subdomain and global, odd and even step
  counts: within 1e-13 (the kernels and the oracle differ only in exp);
* interface local regression (Sec. 4): within 1e-12 (normal equations by
  Cramer's rule against the oracle's least-squares solver);
* the smoothed pipeline end to end against the oracle's.
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


def noisy_mesh(nx, ny, seed, amp=0.01):
    rng = np.random.default_rng(seed)
    xi, eta = np.meshgrid(np.linspace(0, 1, nx), np.linspace(0, 1, ny))
    m = np.stack([xi + 0.05 * np.sin(np.pi * xi) * np.sin(2 * np.pi * eta),
                  eta + 0.04 * np.sin(2 * np.pi * xi) * np.sin(np.pi * eta)], -1)
    m[1:-1, 1:-1] += rng.normal(0, amp / max(nx, ny), size=m[1:-1, 1:-1].shape)
    return m


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("nx,ny", [(2, 2), (33, 17), (130, 67), (1025, 1025)])
def test_quality_matches_oracle(ctx, ref, nx, ny):
    import torch

    import paper_1310_3435_amd as sdd
    m = noisy_mesh(nx, ny, nx + ny)
    say(f"quality {nx}x{ny}")
    g = sdd.sdd_mesh_quality(ctx, dev(m), want_cells=True)
    torch.cuda.synchronize()
    out, q = g["out"].cpu().numpy(), g["q"].cpu().numpy()
    r = ref.mesh_quality(m)
    assert np.allclose(q, r["q"], rtol=1e-12, atol=0)
    assert out[0] == pytest.approx(r["q_max"], rel=1e-12)
    assert out[1] == pytest.approx(r["q_mean"], rel=1e-12)
    assert int(out[2]) == r["folded"]


def test_quality_folds_and_degenerate_cells(ctx, ref):
    import torch

    import paper_1310_3435_amd as sdd
    m = noisy_mesh(17, 17, 1)
    m[8, 8, 0] = m[8, 10, 0] + 0.02        # folds the cells around node (8, 8)
    g = sdd.sdd_mesh_quality(ctx, dev(m))["out"].cpu().numpy()
    r = ref.mesh_quality(m)
    assert int(g[2]) == r["folded"] >= 1 and g[0] == pytest.approx(r["q_max"], rel=1e-12)
    c = np.array([[[0.0, 0.0], [1.0, 0.0]], [[1.0, 0.0], [2.0, 0.0]]])
    g = sdd.sdd_mesh_quality(ctx, dev(c))["out"].cpu().numpy()
    torch.cuda.synchronize()
    assert g[0] == np.inf and int(g[2]) == 1
    # one cell of a grid collapsed to a point: Q = inf there, as in the oracle
    m = noisy_mesh(9, 9, 2)
    m[3:5, 3:5] = m[3, 3]
    out = sdd.sdd_mesh_quality(ctx, dev(m), want_cells=True)
    g, q = out["out"].cpu().numpy(), out["q"].cpu().numpy()
    r = ref.mesh_quality(m)
    assert q[3, 3] == np.inf and r["q"][3, 3] == np.inf and g[0] == np.inf
    assert int(g[2]) == r["folded"]


def test_compare_matches_oracle(ctx, ref):
    import torch

    import paper_1310_3435_amd as sdd
    d = W.random_density(4, 4)
    a, b = noisy_mesh(65, 33, 2, 0.5), noisy_mesh(65, 33, 3, 0.5)
    g = sdd.sdd_mesh_compare(ctx, d, dev(a), dev(b)).cpu().numpy()
    torch.cuda.synchronize()
    r = ref.mesh_compare(a, b, d)
    say(f"compare: linf {g[0]:.6e} (oracle {r['linf']:.6e}), disp {g[1]:.6e}")
    assert g[0] == pytest.approx(r["linf"], rel=1e-13) and g[1] == pytest.approx(r["max_disp"], rel=1e-13)


@pytest.mark.parametrize("per_subdomain", [True, False, "shifted"])
@pytest.mark.parametrize("steps", [0, 1, 4, 7])
def test_perona_malik_matches_oracle(ctx, ref, per_subdomain, steps):
    import torch

    import paper_1310_3435_amd as sdd
    L = {"nx": 65, "ny": 49, "sx": 4, "sy": 3}
    m = noisy_mesh(65, 49, 5, 2.0)
    dt = 0.9 / (2 * 64**2 + 2 * 48**2)
    t = dev(m)
    sdd.sdd_mesh_smooth(ctx, L, t, dt, 2.0, steps, per_subdomain)
    g = t.cpu().numpy()
    torch.cuda.synchronize()
    r = ref.perona_malik(m, dt, 2.0, steps, L if per_subdomain else None, shifted=per_subdomain == "shifted")
    say(f"perona-malik steps={steps} per_subdomain={per_subdomain}: max diff {np.abs(g - r).max():.3e}")
    assert np.abs(g - r).max() <= 1e-13
    if steps:
        assert np.abs(g - m).max() > 1e-6


def test_perona_malik_rejects_unstable_steps(ctx):
    import paper_1310_3435_amd as sdd
    L = {"nx": 33, "ny": 33, "sx": 2, "sy": 2}
    t = dev(noisy_mesh(33, 33, 0))
    with pytest.raises(sdd.SddError, match="invalid"):
        sdd.sdd_mesh_smooth(ctx, L, t, 1e-3, 1.0, 2)
    with pytest.raises(sdd.SddError, match="invalid"):
        sdd.sdd_mesh_smooth(ctx, L, t, 1e-5, -1.0, 2)


@pytest.mark.parametrize("span", [5, 9, 15])
def test_interface_smoothing_matches_oracle(ctx, ref, span):
    import torch

    import paper_1310_3435_amd as sdd
    rng = np.random.default_rng(span)
    L = {"nx": 65, "ny": 49, "sx": 4, "sy": 3}
    vert = rng.normal(size=(3, 49, 2))
    horiz = rng.normal(size=(2, 65, 2))
    tv, th = dev(vert), dev(horiz)
    sdd.sdd_smooth_interfaces(ctx, L, tv, th, span)
    gv, gh = tv.cpu().numpy(), th.cpu().numpy()
    torch.cuda.synchronize()
    rv, rh = ref.smooth_interfaces(L, vert, horiz, span)
    d = max(np.abs(gv - rv).max(), np.abs(gh - rh).max())
    say(f"local regression span {span}: max diff {d:.3e}")
    assert d <= 1e-12
    assert np.array_equal(gv[:, ::16], vert[:, ::16]) and np.array_equal(gh[:, ::16], horiz[:, ::16])


def test_interface_smoothing_rejects_bad_spans(ctx):
    import paper_1310_3435_amd as sdd
    L = {"nx": 17, "ny": 9, "sx": 2, "sy": 2}
    tv, th = dev(np.zeros((1, 9, 2))), dev(np.zeros((1, 17, 2)))
    for span in (3, 6, 11):      # too small, even, longer than a vertical line
        with pytest.raises(sdd.SddError, match="invalid"):
            sdd.sdd_smooth_interfaces(ctx, L, tv, th, span)


def test_smoothed_pipeline_matches_oracle(ctx, ref):
    import torch

    import paper_1310_3435_amd as sdd
    c = dict(W.cfg_plain_fp64(), smooth_span=7, pm={"dt": 0.2 / (2 * 64**2 + 2 * 32**2), "k": 3.0, "steps": 5})
    say("smoothed pipeline")
    g = sdd.run_pipeline(ctx, c)
    mesh = g["mesh"].cpu().numpy()
    torch.cuda.synchronize()
    r = ref.pipeline(c)
    d = np.abs(mesh - r["mesh"]).max()
    say(f"smoothed pipeline vs oracle: max diff {d:.3e}")
    assert d <= 1e-9
    q = sdd.sdd_mesh_quality(ctx, g["mesh"])["out"].cpu().numpy()
    assert q[0] == pytest.approx(ref.mesh_quality(r["mesh"])["q_max"], rel=1e-9)


def test_whole_grid_mesh_matches_oracle(ctx, ref):
    import torch

    import paper_1310_3435_amd as sdd
    g = sdd.sdd_grid_nodes(ctx, 29, 23).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(g, ref.grid_nodes(29, 23))
    c = dict(W.cfg_paper_example(), paths=500, prec="fp64",
             pm={"dt": 1e-4, "k": 1000.0, "steps": 5})
    say("whole-grid Monte Carlo mesh, 29 x 29, fp64, smoothed")
    out = sdd.run_probabilistic(ctx, c)
    mesh = out["mesh"].cpu().numpy()
    torch.cuda.synchronize()
    r = ref.probabilistic_mesh(c)
    d = np.abs(mesh - r["mesh"]).max()
    say(f"whole-grid mesh vs oracle: max diff {d:.3e}")
    assert d <= 1e-10
