"""Plain CPU oracle of the stochastic-deterministic mesh pipeline.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library ``paper_1310_3435_amd`` and never imports it; the
two meet only in the seeded inputs of ``workloads``.

Parts (Bihlo & Haynes, arXiv 1310.3435):

* ``interface_estimate`` -- the Monte Carlo estimate of the mesh map at
  interface nodes, eq. (7a)/(7b) with Euler-Maruyama stepping and the
  end-of-step exit test of Sec. 2.2 (plain C in ``walk_ref.c``).
* ``edge1d_table`` -- boundary data whose tangential coordinate solves the
  one-dimensional generator along each edge (Sec. 3.2, single-domain
  reference).
* ``layout_nodes`` -- interface points of a non-overlapping decomposition
  (Sec. 2.1, Fig. 1), uniformly spaced or equidistributing w along each
  segment (Sec. 3.6 places the points from the monitor function).
* ``fill_interfaces`` -- Monte Carlo values at a few points plus
  interpolation along each interface (Sec. 3.6), linear or monotone cubic.
* ``subdomain_solve`` -- the independent Dirichlet solves of every
  subdomain by centred finite differences (Sec. 2.1, Sec. 3.2), here solved
  directly by a sparse LU rather than iterated, so that it is the exact
  discrete solution.
* ``grid_nodes``, ``assemble_mesh``, ``probabilistic_mesh`` -- the mesh by
  Monte Carlo at every grid point (Sec. 3.3).
* ``mesh_quality``, ``mesh_compare``, ``perona_malik``,
  ``smooth_interfaces`` -- quality measure and smoothing (``postprocess.py``).

Every array is float64 and C-contiguous.
"""

from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "walk_ref.c")]

FP64, FP32 = 0, 1
_PREC = {"fp64": FP64, "fp32": FP32}
_KIND = {"gauss": 0, "ring": 1, "sech2": 2, "sin2": 3}
_BMAP = {"identity": 0, "affine": 1, "annulus": 2, "table": 3, "edge1d": 3}
MAX_TERMS = 8


class RefTerm(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("amp", C.c_double), ("coef", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("r0", C.c_double), ("nx", C.c_double),
                ("ny", C.c_double)]


class RefDensity(C.Structure):
    _fields_ = [("base", C.c_double), ("n_terms", C.c_int32), ("pad", C.c_int32),
                ("term", RefTerm * MAX_TERMS)]


class RefBmap(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_per_edge", C.c_int32), ("p", C.c_double * 8),
                ("table", C.c_void_p)]


PATH_RECORD = np.dtype([("exit_xi", "<f8"), ("exit_eta", "<f8"), ("steps", "<i8"),
                        ("side", "<i4"), ("capped", "<i4")])


def build(force: bool = True) -> str:
    """Compile walk_ref.c into liboracle.so (plain C, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", _LIB_PATH + ".tmp"] + _SRC + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        L.sddref_philox4x32_10.argtypes = [P, P, P]
        L.sddref_philox_many.argtypes = [C.c_int64, P, P, P]
        L.sddref_normals64.argtypes = [C.c_int64, P, P]
        L.sddref_block_uniforms.argtypes = [C.c_int64, P, P]
        L.sddref_density_eval.argtypes = [C.POINTER(RefDensity), C.c_int64, P, P, P]
        L.sddref_bmap_eval.argtypes = [C.POINTER(RefBmap), C.c_int64, P, P, P]
        L.sddref_exit_point.argtypes = [C.c_double] * 4 + [P, P]
        L.sddref_exit_point.restype = C.c_int
        L.sddref_bridge_uniforms.argtypes = [C.c_int64, P, P]
        L.sddref_bridge_exit_prob.argtypes = [C.c_double] * 5 + [P]
        L.sddref_bridge_exit_prob.restype = C.c_double
        L.sddref_expo_steps.argtypes = [C.c_int64, P, C.c_double, P]
        L.sddref_interface_estimate.argtypes = [
            C.POINTER(RefDensity), C.POINTER(RefBmap), P, P, C.c_int64, C.c_int64, C.c_int64,
            C.c_double, C.c_uint64, C.c_int, C.c_double, C.c_int, C.c_int, P, P, P, P, P, C.c_int]
        L.sddref_interface_estimate.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------------ inputs

def make_density(d: dict) -> RefDensity:
    D = RefDensity()
    D.base = d["base"]
    terms = d["terms"]
    if len(terms) > MAX_TERMS:
        raise ValueError("too many density terms")
    D.n_terms = len(terms)
    for i, t in enumerate(terms):
        T = D.term[i]
        T.kind = _KIND[t["kind"]]
        for f in ("amp", "coef", "cx", "cy", "r0", "nx", "ny"):
            setattr(T, f, float(t.get(f, 0.0)))
    return D


class Bmap:
    """Boundary map plus the table it may reference (kept alive here)."""

    def __init__(self, b: dict, density: Optional[dict] = None):
        self.desc = b
        self.s = RefBmap()
        self.s.kind = _BMAP[b["kind"]]
        self.table = None
        for i, v in enumerate(b.get("p", [])):
            self.s.p[i] = float(v)
        if b["kind"] == "edge1d":
            if density is None:
                raise ValueError("edge1d map needs the density")
            self.table = edge1d_table(density, int(b.get("n_per_edge", 4097)))
        elif b["kind"] == "table":
            self.table = np.ascontiguousarray(b["table"], dtype=np.float64)
        if self.table is not None:
            self.s.n_per_edge = self.table.shape[1]
            self.s.table = self.table.ctypes.data_as(C.c_void_p).value

    def eval(self, pts: np.ndarray, side: np.ndarray) -> np.ndarray:
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
        side = np.ascontiguousarray(side, dtype=np.int32).reshape(-1)
        out = np.empty_like(pts)
        lib().sddref_bmap_eval(C.byref(self.s), pts.shape[0], _ptr(side), _ptr(pts), _ptr(out))
        return out

    def eval_boundary(self, pts: np.ndarray) -> np.ndarray:
        """Map at boundary points, side chosen in the order xi=0, xi=1, eta=0, eta=1."""
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, 2)
        side = np.full(pts.shape[0], -1, dtype=np.int32)
        for s, (c, v) in reversed(list(enumerate([(0, 0.0), (0, 1.0), (1, 0.0), (1, 1.0)]))):
            side[pts[:, c] == v] = s
        if np.any(side < 0):
            raise ValueError("point not on the boundary")
        return self.eval(pts, side)


# ------------------------------------------------------------------ RNG

def philox(ctr: np.ndarray, key) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.asarray(key, dtype=np.uint32).reshape(2).copy()
    out = np.empty_like(ctr)
    lib().sddref_philox_many(ctr.shape[0], _ptr(ctr), _ptr(k), _ptr(out))
    return out


def normals64(fields: np.ndarray) -> np.ndarray:
    """Box-Muller of 21-bit field pairs [n][2] (u = (b + 1/2) 2^-21)."""
    fields = np.ascontiguousarray(fields, dtype=np.uint32).reshape(-1, 2)
    z = np.empty(fields.shape, dtype=np.float64)
    lib().sddref_normals64(fields.shape[0], _ptr(fields), _ptr(z))
    return z


def block_uniforms(blocks: np.ndarray) -> np.ndarray:
    """The six uniforms [n][6] of Philox blocks [n][4]: (u_a, u_b) of steps
    3m, 3m+1, 3m+2."""
    blocks = np.ascontiguousarray(blocks, dtype=np.uint32).reshape(-1, 4)
    u = np.empty((blocks.shape[0], 6), dtype=np.float64)
    lib().sddref_block_uniforms(blocks.shape[0], _ptr(blocks), _ptr(u))
    return u


# ------------------------------------------------------------------ density

def density_eval(d: dict, pts: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """w and grad w at pts[n][2]."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    D = make_density(d)
    w = np.empty(pts.shape[0])
    g = np.empty_like(pts)
    lib().sddref_density_eval(C.byref(D), pts.shape[0], _ptr(pts), _ptr(w), _ptr(g))
    return w, g


def exit_point(p, q):
    ex, ey = C.c_double(), C.c_double()
    side = lib().sddref_exit_point(float(p[0]), float(p[1]), float(q[0]), float(q[1]),
                                   C.byref(ex), C.byref(ey))
    return side, (ex.value, ey.value)


def bridge_uniforms(words: np.ndarray) -> np.ndarray:
    """Uniforms of the bridge test from words of the counter-word-3 = 1
    blocks (the low 23 bits)."""
    words = np.ascontiguousarray(words, dtype=np.uint32).reshape(-1)
    u = np.empty(words.shape[0], dtype=np.float64)
    lib().sddref_bridge_uniforms(words.shape[0], _ptr(words), _ptr(u))
    return u


def bridge_exit_prob(p, q, dt: float):
    """Brownian-bridge exit probability of the step p -> q (both inside the
    square) and the side it exits through (Sec. 2.2)."""
    side = C.c_int()
    prob = lib().sddref_bridge_exit_prob(float(p[0]), float(p[1]), float(q[0]), float(q[1]), float(dt),
                                         C.byref(side))
    return prob, side.value


def expo_steps(words: np.ndarray, dt: float) -> np.ndarray:
    """Exponential step lengths tau = -ln(u) dt from words of the
    counter-word-3 = 2 blocks (u formed as for the bridge test)."""
    words = np.ascontiguousarray(words, dtype=np.uint32).reshape(-1)
    tau = np.empty(words.shape[0], dtype=np.float64)
    lib().sddref_expo_steps(words.shape[0], _ptr(words), float(dt), _ptr(tau))
    return tau


# ------------------------------------------------------------------ estimate

_EXIT = {"step": 0, "bridge": 1, "expo": 2}


def interface_estimate(density: dict, bmap, nodes: np.ndarray, paths: int, dt: float, seed: int,
                       prec: str = "fp64", t_max: float = 8.0, node_ids=None, path_begin: int = 0,
                       per_path: bool = False, proj_mode: int = 0, nthreads: int = 0,
                       bridge: bool = False, allow_off: bool = False, exit_test: str = None) -> dict:
    """Monte Carlo estimate of (x, y) at every node (eq. (7a), Sec. 2.2).

    exit_test: "step" (end of step), "bridge" (plus the Brownian-bridge
    test: the conditional exit probability of Sec. 2.2) or "expo"
    (exponential time stepping with mean step dt, Sec. 2.2).  bridge=True is
    exit_test="bridge".

    Returns dict(mean[n,2], se[n,2], sums[n,4], steps, paths, capped[, per_path]).
    """
    if exit_test is None:
        exit_test = "bridge" if bridge else "step"
    B = bmap if isinstance(bmap, Bmap) else Bmap(bmap, density)
    D = make_density(density)
    nodes = np.ascontiguousarray(nodes, dtype=np.float64).reshape(-1, 2)
    if allow_off:
        # nodes off the open square walk nothing and get NaN; the others keep
        # their list index as counter word g
        inside = (nodes[:, 0] > 0) & (nodes[:, 0] < 1) & (nodes[:, 1] > 0) & (nodes[:, 1] < 1)
        idx = np.flatnonzero(inside) if node_ids is None else np.asarray(node_ids)[inside]
        sub = interface_estimate(density, B, nodes[inside], paths, dt, seed, prec, t_max, idx, path_begin,
                                 per_path, proj_mode, nthreads, exit_test=exit_test)
        out = dict(sub)
        for key, width in (("mean", 2), ("se", 2), ("sums", 4)):
            full = np.full((nodes.shape[0], width), np.nan)
            full[inside] = sub[key]
            out[key] = full
        out["paths"] = int(nodes.shape[0]) * int(paths)
        return out
    n = nodes.shape[0]
    ids = None if node_ids is None else np.ascontiguousarray(node_ids, dtype=np.int64)
    mean = np.empty((n, 2))
    se = np.empty((n, 2))
    sums = np.empty((n, 4))
    stats = np.zeros(3, dtype=np.int64)
    rec = np.zeros((n, paths), dtype=PATH_RECORD) if per_path else None
    rc = lib().sddref_interface_estimate(
        C.byref(D), C.byref(B.s), _ptr(nodes), _ptr(ids), n, int(paths), int(path_begin), float(dt),
        C.c_uint64(int(seed)), _PREC[prec], float(t_max), int(proj_mode), _EXIT[exit_test], _ptr(mean), _ptr(se),
        _ptr(sums), _ptr(stats), _ptr(rec), int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    out = {"mean": mean, "se": se, "sums": sums, "steps": int(stats[0]), "paths": int(stats[1]),
           "capped": int(stats[2])}
    if per_path:
        out["per_path"] = rec
    return out


# ------------------------------------------------------------------ edge data

def _cumulative_simpson(f, a: float, b: float, n: int) -> np.ndarray:
    """F(s_q) = integral of f from a to s_q, s_q = a + q (b-a)/(n-1), by Simpson's
    rule on every sample interval."""
    s = a + (b - a) * np.arange(n) / (n - 1)
    h = (b - a) / (n - 1)
    mid = s[:-1] + 0.5 * h
    panel = (h / 6.0) * (f(s[:-1]) + 4.0 * f(mid) + f(s[1:]))
    return np.concatenate([[0.0], np.cumsum(panel)])


def edge1d_table(density: dict, n: int) -> np.ndarray:
    """values[4][n][2]: on each side the tangential coordinate solves the
    one-dimensional generator (w u')' = 0 along that side with end values 0
    and 1, i.e. u(s) = int_0^s 1/w / int_0^1 1/w (Sec. 3.2 takes the
    tangential boundary values from the 1D form of the generator); the
    normal coordinate is the side's own value."""
    out = np.empty((4, n, 2))
    for side in range(4):
        if side < 2:
            fixed = float(side)

            def inv_w(t, fixed=fixed):
                return 1.0 / density_eval(density, np.stack([np.full_like(t, fixed), t], 1))[0]
        else:
            fixed = float(side - 2)

            def inv_w(t, fixed=fixed):
                return 1.0 / density_eval(density, np.stack([t, np.full_like(t, fixed)], 1))[0]
        F = _cumulative_simpson(inv_w, 0.0, 1.0, n)
        u = F / F[-1]
        if side < 2:
            out[side, :, 0] = fixed
            out[side, :, 1] = u
        else:
            out[side, :, 0] = u
            out[side, :, 1] = fixed
    return out


# ------------------------------------------------------------------ layout

def check_layout(L: dict) -> Tuple[int, int, int, int, int, int]:
    nx, ny, sx, sy = L["nx"], L["ny"], L["sx"], L["sy"]
    if sx < 1 or sy < 1 or (nx - 1) % sx or (ny - 1) % sy:
        raise ValueError("layout does not divide evenly")
    mx, my = (nx - 1) // sx, (ny - 1) // sy
    if mx < 2 or my < 2:
        raise ValueError("subdomains need an interior")
    return nx, ny, sx, sy, mx, my


def node_count(L: dict, k: int) -> int:
    _, _, sx, sy, _, _ = check_layout(L)
    return (sx - 1) * (sy - 1) + k * ((sx - 1) * sy + (sy - 1) * sx)


def _segment_params(a: float, b: float, k: int, placement: str, w_along) -> np.ndarray:
    """k interior points of the segment [a, b] of an interface line."""
    if k == 0:
        return np.empty(0)
    if placement == "uniform":
        return a + (b - a) * np.arange(1, k + 1) / (k + 1)
    if placement == "equidistributed":
        # int_a^{s_i} w = i/(k+1) int_a^b w, by cumulative Simpson on 4096
        # panels and linear inversion inside the panel that holds the target.
        M = 4096
        F = _cumulative_simpson(w_along, a, b, M + 1)
        s = a + (b - a) * np.arange(M + 1) / M
        out = np.empty(k)
        for i in range(1, k + 1):
            T = F[-1] * i / (k + 1)
            q = int(np.searchsorted(F, T, side="right") - 1)
            q = min(max(q, 0), M - 1)
            out[i - 1] = s[q] + (s[q + 1] - s[q]) * (T - F[q]) / (F[q + 1] - F[q])
        return out
    raise ValueError(placement)


def layout_nodes(L: dict, k: int, placement: str = "uniform", density: Optional[dict] = None) -> np.ndarray:
    """MC node list of a layout: crosspoints (row by row), then k points on
    every vertical-line segment (line by line, bottom to top), then k points
    on every horizontal-line segment (line by line, left to right)."""
    nx, ny, sx, sy, mx, my = check_layout(L)
    pts = []
    for b in range(1, sy):
        for a in range(1, sx):
            pts.append((a / sx, b / sy))
    for a in range(1, sx):
        xi = a / sx
        for b in range(sy):
            def w_along(t, xi=xi):
                return density_eval(density, np.stack([np.full_like(t, xi), t], 1))[0]
            for t in _segment_params(b / sy, (b + 1) / sy, k, placement, w_along):
                pts.append((xi, t))
    for b in range(1, sy):
        eta = b / sy
        for a in range(sx):
            def w_along(t, eta=eta):
                return density_eval(density, np.stack([t, np.full_like(t, eta)], 1))[0]
            for t in _segment_params(a / sx, (a + 1) / sx, k, placement, w_along):
                pts.append((t, eta))
    return np.array(pts, dtype=np.float64).reshape(-1, 2)


EXTREMA_PANELS = 4096


def _sampled_extrema(f: np.ndarray, q0: int, q1: int, s: np.ndarray, h: float) -> list:
    """Strict local extrema of samples f at q in [q0, q1] (the differences on
    either side have opposite signs), each moved to the vertex of the
    parabola through its three samples."""
    out = []
    for q in range(q0, q1 + 1):
        d0, d1 = f[q] - f[q - 1], f[q + 1] - f[q]
        if d0 * d1 < 0.0:
            delta = 0.5 * (f[q - 1] - f[q + 1]) / (f[q - 1] - 2.0 * f[q] + f[q + 1])
            out.append(s[q] + delta * h)
    return out


def extrema_params(density: dict, fixed: float, vertical: bool, a: float, b: float) -> np.ndarray:
    """Parameters on the segment [a, b] of an interface line where the
    density's first or second derivative along the line has a local extremum
    (Sec. 3.6 places the Monte Carlo points at the maxima and minima of the
    first and second derivatives of the monitor function along the dividing
    lines).  The derivative comes from the analytic gradient at M + 1 = 4097
    samples, the second derivative from its central differences; extrema
    are located on the samples and refined by a parabola; points closer than
    one sample to the previous one are dropped."""
    M = EXTREMA_PANELS
    h = (b - a) / M
    s = a + (b - a) * np.arange(M + 1) / M
    pts = np.stack([np.full(M + 1, fixed), s], 1) if vertical else np.stack([s, np.full(M + 1, fixed)], 1)
    _, g = density_eval(density, pts)
    f1 = g[:, 1] if vertical else g[:, 0]
    f2 = np.zeros(M + 1)
    f2[1:M] = (f1[2:] - f1[:-2]) / (2.0 * h)
    cand = sorted(_sampled_extrema(f1, 1, M - 1, s, h) + _sampled_extrema(f2, 2, M - 2, s, h))
    kept = []
    for t in cand:
        if not kept or t - kept[-1] >= h:
            kept.append(t)
    return np.array(kept, dtype=np.float64)


def layout_nodes_extrema(L: dict, density: dict, cap: int) -> Tuple[np.ndarray, np.ndarray]:
    """Node list with the crosspoints first and then `cap` slots per segment
    (segments in the order of layout_nodes): segment s holds its extrema
    points (extrema_params, increasing) in its first min(count, cap) slots
    and (-1, -1) in the rest.  Returns (nodes, counts) with the number of
    points each segment found."""
    nx, ny, sx, sy, mx, my = check_layout(L)
    ncross = (sx - 1) * (sy - 1)
    nseg = (sx - 1) * sy + (sy - 1) * sx
    nodes = np.full((ncross + nseg * cap, 2), -1.0)
    counts = np.zeros(nseg, dtype=np.int32)
    c = 0
    for b in range(1, sy):
        for a in range(1, sx):
            nodes[c] = (a / sx, b / sy)
            c += 1
    seg = 0
    for a in range(1, sx):
        for b in range(sy):
            t = extrema_params(density, a / sx, True, b / sy, (b + 1) / sy)
            counts[seg] = t.size
            k = min(t.size, cap)
            nodes[ncross + seg * cap: ncross + seg * cap + k] = np.stack([np.full(k, a / sx), t[:k]], 1)
            seg += 1
    for b in range(1, sy):
        for a in range(sx):
            t = extrema_params(density, b / sy, False, a / sx, (a + 1) / sx)
            counts[seg] = t.size
            k = min(t.size, cap)
            nodes[ncross + seg * cap: ncross + seg * cap + k] = np.stack([t[:k], np.full(k, b / sy)], 1)
            seg += 1
    return nodes, counts


# ------------------------------------------------------------------ fill

def pchip_slopes(t: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Shape-preserving knot slopes of Fritsch & Carlson (SIAM J. Numer. Anal.
    17, 1980) with the weighted harmonic mean of Fritsch & Butland and the
    three-point shape-preserving end slopes (Moler, Numerical Computing with
    MATLAB, Sec. 3.4)."""
    n = t.shape[0]
    h = np.diff(t)
    delta = np.diff(v) / h
    d = np.zeros(n)
    if n == 2:
        d[:] = delta[0]
        return d
    for m in range(1, n - 1):
        a, b = delta[m - 1], delta[m]
        if a == 0.0 or b == 0.0 or (a > 0) != (b > 0):
            d[m] = 0.0
        else:
            w1 = 2.0 * h[m] + h[m - 1]
            w2 = h[m] + 2.0 * h[m - 1]
            d[m] = (w1 + w2) / (w1 / a + w2 / b)

    def end(h0, h1, d0, d1):
        e = ((2.0 * h0 + h1) * d0 - h0 * d1) / (h0 + h1)
        if np.sign(e) != np.sign(d0):
            return 0.0
        if np.sign(d0) != np.sign(d1) and abs(e) > 3.0 * abs(d0):
            return 3.0 * d0
        return e

    d[0] = end(h[0], h[1], delta[0], delta[1])
    d[-1] = end(h[-1], h[-2], delta[-1], delta[-2])
    return d


def interp_segment(t: np.ndarray, v: np.ndarray, te: np.ndarray, kind: str) -> np.ndarray:
    """Interpolate knot values v(t) (t increasing) at te, inside [t0, t_end]."""
    m = np.clip(np.searchsorted(t, te, side="right") - 1, 0, t.shape[0] - 2)
    h = t[m + 1] - t[m]
    tau = (te - t[m]) / h
    if kind == "linear":
        return v[m] + tau * (v[m + 1] - v[m])
    if kind == "pchip":
        d = pchip_slopes(t, v)
        h00 = 2 * tau**3 - 3 * tau**2 + 1
        h10 = tau**3 - 2 * tau**2 + tau
        h01 = -2 * tau**3 + 3 * tau**2
        h11 = tau**3 - tau**2
        return h00 * v[m] + h10 * h * d[m] + h01 * v[m + 1] + h11 * h * d[m + 1]
    raise ValueError(kind)


def fill_interfaces(L: dict, k: int, bmap, nodes: np.ndarray, values: np.ndarray, interp: str,
                    density: Optional[dict] = None, counts: Optional[np.ndarray] = None) -> Tuple[np.ndarray, np.ndarray]:
    """All interface mesh values from the node estimates (Sec. 3.6).

    Returns (vert[sx-1][ny][2], horiz[sy-1][nx][2]).  Line ends take the
    boundary map, crosspoints their own estimate, segment interiors the
    interpolant through (start, k nodes, end) in the segment parameter.
    With `counts`, every segment has k slots of which it uses the first
    min(counts[s], k).
    """
    nx, ny, sx, sy, mx, my = check_layout(L)
    B = bmap if isinstance(bmap, Bmap) else Bmap(bmap, density)
    nodes = np.asarray(nodes, dtype=np.float64).reshape(-1, 2)
    values = np.asarray(values, dtype=np.float64).reshape(-1, 2)
    ncross = (sx - 1) * (sy - 1)

    def cross(a, b):  # a in 1..sx-1, b in 1..sy-1
        return values[(b - 1) * (sx - 1) + (a - 1)]

    vert = np.empty((max(sx - 1, 0), ny, 2))
    horiz = np.empty((max(sy - 1, 0), nx, 2))
    base = ncross
    segno = 0
    eta_mesh = np.arange(ny) / (ny - 1)
    xi_mesh = np.arange(nx) / (nx - 1)
    for a in range(1, sx):
        xi = a / sx
        vert[a - 1, 0] = B.eval_boundary([(xi, 0.0)])[0]
        vert[a - 1, ny - 1] = B.eval_boundary([(xi, 1.0)])[0]
        for b in range(1, sy):
            vert[a - 1, b * my] = cross(a, b)
        for b in range(sy):
            t0, t1 = b / sy, (b + 1) / sy
            v0 = vert[a - 1, 0] if b == 0 else cross(a, b)
            v1 = vert[a - 1, ny - 1] if b == sy - 1 else cross(a, b + 1)
            used = k if counts is None else min(int(counts[segno]), k)
            seg = slice(base, base + used)
            base += k
            segno += 1
            t = np.concatenate([[t0], nodes[seg, 1], [t1]])
            vv = np.concatenate([[v0], values[seg], [v1]])
            j = np.arange(b * my + 1, (b + 1) * my)
            for c in range(2):
                vert[a - 1, j, c] = interp_segment(t, vv[:, c], eta_mesh[j], interp)
    for b in range(1, sy):
        eta = b / sy
        horiz[b - 1, 0] = B.eval_boundary([(0.0, eta)])[0]
        horiz[b - 1, nx - 1] = B.eval_boundary([(1.0, eta)])[0]
        for a in range(1, sx):
            horiz[b - 1, a * mx] = cross(a, b)
        for a in range(sx):
            t0, t1 = a / sx, (a + 1) / sx
            v0 = horiz[b - 1, 0] if a == 0 else cross(a, b)
            v1 = horiz[b - 1, nx - 1] if a == sx - 1 else cross(a + 1, b)
            used = k if counts is None else min(int(counts[segno]), k)
            seg = slice(base, base + used)
            base += k
            segno += 1
            t = np.concatenate([[t0], nodes[seg, 0], [t1]])
            vv = np.concatenate([[v0], values[seg], [v1]])
            i = np.arange(a * mx + 1, (a + 1) * mx)
            for c in range(2):
                horiz[b - 1, i, c] = interp_segment(t, vv[:, c], xi_mesh[i], interp)
    return vert, horiz


# ------------------------------------------------------------------ FD

def fd_coefficients(density: dict, nx: int, ny: int, i: np.ndarray, j: np.ndarray):
    """Conservative centred 5-point coefficients of div(w grad u) at nodes
    (i, j) of the global nx x ny grid: w at the four edge midpoints over h^2."""
    hx, hy = 1.0 / (nx - 1), 1.0 / (ny - 1)
    xi = i / (nx - 1)
    eta = j / (ny - 1)

    def w(a, b):
        return density_eval(density, np.stack([a, b], 1))[0]

    aE = w((i + 0.5) / (nx - 1), eta) / (hx * hx)
    aW = w((i - 0.5) / (nx - 1), eta) / (hx * hx)
    aN = w(xi, (j + 0.5) / (ny - 1)) / (hy * hy)
    aS = w(xi, (j - 0.5) / (ny - 1)) / (hy * hy)
    return aE, aW, aN, aS


def dirichlet_solve(density: dict, nx: int, ny: int, i0: int, i1: int, j0: int, j1: int,
                    frame: np.ndarray) -> np.ndarray:
    """Exact solution of the discrete Dirichlet problem on nodes
    [i0..i1] x [j0..j1] of the global grid.  frame[j1-j0+1][i1-i0+1][2] holds
    the boundary values on its outer ring (interior entries are ignored).
    Returns the full block with the interior filled."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    Mx, My = i1 - i0 - 1, j1 - j0 - 1
    jj, ii = np.meshgrid(np.arange(j0 + 1, j1), np.arange(i0 + 1, i1), indexing="ij")
    ii, jj = ii.ravel().astype(np.float64), jj.ravel().astype(np.float64)
    aE, aW, aN, aS = fd_coefficients(density, nx, ny, ii, jj)
    n = Mx * My
    idx = np.arange(n)
    li, lj = idx % Mx, idx // Mx
    rows, cols, vals = [idx], [idx], [aE + aW + aN + aS]
    rhs = np.zeros((n, 2))
    for a, di, dj in ((aE, 1, 0), (aW, -1, 0), (aN, 0, 1), (aS, 0, -1)):
        ni, nj = li + di, lj + dj
        inside = (ni >= 0) & (ni < Mx) & (nj >= 0) & (nj < My)
        rows.append(idx[inside])
        cols.append((nj * Mx + ni)[inside])
        vals.append(-a[inside])
        out = ~inside
        rhs[out] += a[out, None] * frame[nj[out] + 1, ni[out] + 1]
    A = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    lu = spla.splu(A)
    sol = np.stack([lu.solve(rhs[:, 0]), lu.solve(rhs[:, 1])], 1)
    block = frame.copy()
    block[1:-1, 1:-1] = sol.reshape(My, Mx, 2)
    return block


def boundary_frame(bmap: Bmap, nx: int, ny: int) -> np.ndarray:
    """mesh[ny][nx][2] with the boundary ring set from the map, NaN inside."""
    mesh = np.full((ny, nx, 2), np.nan)
    xi = np.arange(nx) / (nx - 1)
    eta = np.arange(ny) / (ny - 1)
    mesh[0, :] = bmap.eval_boundary(np.stack([xi, np.zeros(nx)], 1))
    mesh[ny - 1, :] = bmap.eval_boundary(np.stack([xi, np.ones(nx)], 1))
    mesh[:, 0] = bmap.eval_boundary(np.stack([np.zeros(ny), eta], 1))
    mesh[:, nx - 1] = bmap.eval_boundary(np.stack([np.ones(ny), eta], 1))
    return mesh


def subdomain_solve(density: dict, bmap, L: dict, vert: np.ndarray, horiz: np.ndarray) -> np.ndarray:
    """Global mesh[ny][nx][2]: boundary from the map, interfaces from the
    filled values, every subdomain interior by its own Dirichlet solve
    (Sec. 2.1: the subdomain solves are independent and done once)."""
    nx, ny, sx, sy, mx, my = check_layout(L)
    B = bmap if isinstance(bmap, Bmap) else Bmap(bmap, density)
    mesh = boundary_frame(B, nx, ny)
    for a in range(1, sx):
        mesh[:, a * mx] = vert[a - 1]
    for b in range(1, sy):
        mesh[b * my, :] = horiz[b - 1]
    for b in range(sy):
        for a in range(sx):
            i0, i1, j0, j1 = a * mx, (a + 1) * mx, b * my, (b + 1) * my
            blk = dirichlet_solve(density, nx, ny, i0, i1, j0, j1, mesh[j0:j1 + 1, i0:i1 + 1])
            mesh[j0 + 1:j1, i0 + 1:i1] = blk[1:-1, 1:-1]
    return mesh


def global_solve(density: dict, bmap, nx: int, ny: int) -> np.ndarray:
    """Single-domain discrete solution (the brute-force reference)."""
    B = bmap if isinstance(bmap, Bmap) else Bmap(bmap, density)
    frame = boundary_frame(B, nx, ny)
    return dirichlet_solve(density, nx, ny, 0, nx - 1, 0, ny - 1, frame)


# ------------------------------------------------------------------ pipeline

def grid_nodes(nx: int, ny: int) -> np.ndarray:
    """Every interior node of the nx x ny grid, row by row (eta outer, xi
    inner): the node set of a mesh computed by Monte Carlo at every grid point
    (Sec. 3.3)."""
    i = np.arange(1, nx - 1)
    j = np.arange(1, ny - 1)
    xi = i / (nx - 1)
    eta = j / (ny - 1)
    return np.stack([np.tile(xi, ny - 2), np.repeat(eta, nx - 2)], 1)


def assemble_mesh(bmap, nx: int, ny: int, values: np.ndarray) -> np.ndarray:
    """mesh[ny][nx][2]: the boundary map on the ring, `values` (in the order
    of grid_nodes) inside."""
    mesh = boundary_frame(bmap, nx, ny)
    mesh[1:-1, 1:-1] = np.asarray(values, dtype=np.float64).reshape(ny - 2, nx - 2, 2)
    return mesh


def probabilistic_mesh(cfg: dict, nthreads: int = 0) -> dict:
    """The whole mesh by Monte Carlo at every interior node (Sec. 3.3), with
    optional Perona-Malik smoothing over the whole grid (Sec. 3.4)."""
    dens = cfg["density"]
    B = Bmap(cfg["bmap"], dens)
    nx, ny = cfg["layout"]["nx"], cfg["layout"]["ny"]
    nodes = grid_nodes(nx, ny)
    est = interface_estimate(dens, B, nodes, cfg["paths"], cfg["dt"], cfg["seed"], cfg.get("prec", "fp64"),
                             nthreads=nthreads, exit_test=cfg.get("exit_test", "step"))
    mesh = assemble_mesh(B, nx, ny, est["mean"])
    pm = cfg.get("pm")
    if pm:
        mesh = perona_malik(mesh, pm["dt"], pm["k"], pm["steps"])
    return {"nodes": nodes, "est": est, "mesh": mesh}


def pipeline(cfg: dict, nthreads: int = 0) -> dict:
    """Nodes -> interface estimate -> fill [-> interface smoothing] ->
    subdomain solves [-> Perona-Malik smoothing]."""
    dens = cfg["density"]
    B = Bmap(cfg["bmap"], dens)
    L = cfg["layout"]
    counts = None
    if cfg.get("placement") == "extrema":
        nodes, counts = layout_nodes_extrema(L, dens, cfg["k"])
    else:
        nodes = layout_nodes(L, cfg["k"], cfg.get("placement", "uniform"), dens)
    est = interface_estimate(dens, B, nodes, cfg["paths"], cfg["dt"], cfg["seed"], cfg.get("prec", "fp64"),
                             t_max=cfg.get("t_max", 8.0), nthreads=nthreads,
                             exit_test=cfg.get("exit_test", "step"), allow_off=True)
    vert, horiz = fill_interfaces(L, cfg["k"], B, nodes, est["mean"], cfg.get("interp", "linear"), counts=counts)
    if cfg.get("smooth_span", 0) > 0:
        vert, horiz = smooth_interfaces(L, vert, horiz, int(cfg["smooth_span"]))
    mesh = subdomain_solve(dens, B, L, vert, horiz)
    pm = cfg.get("pm")
    if pm:
        mesh = perona_malik(mesh, pm["dt"], pm["k"], pm["steps"], L if pm.get("per_subdomain", True) else None)
    return {"nodes": nodes, "est": est, "vert": vert, "horiz": horiz, "mesh": mesh}


from oracle.postprocess import (cell_jacobians, fixed_nodes, ftcs_stable, loess_line, loess_value,  # noqa: E402
                                mesh_compare, mesh_quality, perona_malik, quality_of, smooth_interfaces)
