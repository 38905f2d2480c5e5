"""Mesh quality and smoothing: plain numpy reference (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import the oracle.  This module shares no code with the HIP
library.

Parts (Bihlo & Haynes, arXiv 1310.3435):

* ``mesh_quality`` -- the geometric quality measure Q(K) of eq. (11)
  (Sec. 3.1) for every cell of the computational grid, with its maximum and
  mean (Sec. 3.3).
* ``mesh_compare`` -- the l_inf measure of Sec. 3.3 (the density evaluated
  at the nodes of two meshes of the same logical grid) and the largest node
  displacement.
* ``perona_malik`` -- anisotropic diffusion of the mesh map, eq. (12), by a
  forward-in-time centred-in-space scheme (Sec. 3.4), on the whole grid or
  on every subdomain separately with its interfaces held fixed (Sec. 3.5).
* ``smooth_interfaces`` -- pre-smoothing of the interface values by locally
  weighted quadratic least squares before the subdomain solves (Sec. 4).

Readings (the paper leaves these open):

* Q(K) uses the Jacobian of the cell's bilinear map at the cell centre,
  x_xi = ((x10 + x11) - (x00 + x01)) / (2 h_xi) and so on, h_xi = 1/(nx-1),
  h_eta = 1/(ny-1).  Cells with det J <= 0 are counted as folded.
* l_inf evaluates the density at the nodes' physical positions (meaningful
  when the physical domain lies in the unit square, as for the identity and
  unit-square affine maps).
* Perona-Malik's face coefficient uses the one-sided difference across the
  face, c_E = exp(-((u_E - u_P)/h_xi)^2 / k^2), as in Perona and Malik's
  own discretisation; each mesh component u in {x, y} has its own c.
* Local regression: tricube weights (1 - (|t|/d)^3)^3 over the `span`
  points nearest in index (the window shifted to stay on the line), d the
  largest |t| in the window (Cleveland's definition); the value at the
  point is the fitted quadratic there.  Boundary ends and crosspoints stay.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


# ------------------------------------------------------------------ quality

def cell_jacobians(mesh: np.ndarray) -> np.ndarray:
    """J[j, i] (2x2) of cell (i, j) at its centre from the four corners.
    mesh: [ny][nx][2]."""
    ny, nx = mesh.shape[0], mesh.shape[1]
    hx, hy = 1.0 / (nx - 1), 1.0 / (ny - 1)
    p00, p10 = mesh[:-1, :-1], mesh[:-1, 1:]
    p01, p11 = mesh[1:, :-1], mesh[1:, 1:]
    d_xi = ((p10 + p11) - (p00 + p01)) / (2.0 * hx)     # (x_xi, y_xi)
    d_eta = ((p01 + p11) - (p00 + p10)) / (2.0 * hy)    # (x_eta, y_eta)
    J = np.empty(d_xi.shape[:2] + (2, 2))
    J[..., 0, 0], J[..., 1, 0] = d_xi[..., 0], d_xi[..., 1]
    J[..., 0, 1], J[..., 1, 1] = d_eta[..., 0], d_eta[..., 1]
    return J


def quality_of(J: np.ndarray) -> np.ndarray:
    """Q = tr(J^T J) / (2 sqrt(det(J^T J))), eq. (11).  A cell whose Jacobian
    is singular (det = 0) has Q = inf, also a cell collapsed to a point
    (J = 0), where the quotient is 0/0."""
    JtJ = np.einsum("...ki,...kj->...ij", J, J)
    tr = JtJ[..., 0, 0] + JtJ[..., 1, 1]
    det = JtJ[..., 0, 0] * JtJ[..., 1, 1] - JtJ[..., 0, 1] * JtJ[..., 1, 0]
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(det == 0.0, np.inf, 0.5 * tr / np.sqrt(det))


def mesh_quality(mesh: np.ndarray) -> dict:
    """Q(K) of every cell, Q_max, Q_mean and the number of cells with
    det J <= 0 (Sec. 3.3 lists the maximum and mean of Q over the domain)."""
    J = cell_jacobians(np.asarray(mesh, dtype=np.float64))
    q = quality_of(J)
    detj = J[..., 0, 0] * J[..., 1, 1] - J[..., 0, 1] * J[..., 1, 0]
    return {"q": q, "q_max": float(np.max(q)), "q_mean": float(np.mean(q)), "folded": int(np.sum(detj <= 0))}


def mesh_compare(mesh: np.ndarray, ref: np.ndarray, density: dict) -> dict:
    """l_inf = max over nodes |w(x_mesh) - w(x_ref)| (Sec. 3.3), and the
    largest node displacement max |x_mesh - x_ref|."""
    from oracle import density_eval
    a = np.asarray(mesh, dtype=np.float64).reshape(-1, 2)
    b = np.asarray(ref, dtype=np.float64).reshape(-1, 2)
    wa, _ = density_eval(density, a)
    wb, _ = density_eval(density, b)
    return {"linf": float(np.max(np.abs(wa - wb))),
            "max_disp": float(np.max(np.hypot(a[:, 0] - b[:, 0], a[:, 1] - b[:, 1])))}


# ------------------------------------------------------------ Perona-Malik

def fixed_nodes(nx: int, ny: int, L: dict = None, shifted: bool = False) -> np.ndarray:
    """Nodes held fixed: the boundary ring and, when a layout is given, its
    interface lines; shifted: the lines half a subdomain further on (the
    subdomains of a second cycle, whose interiors hold the original
    interfaces, Sec. 4)."""
    f = np.zeros((ny, nx), dtype=bool)
    f[0, :] = f[-1, :] = f[:, 0] = f[:, -1] = True
    if L is not None:
        mx, my = (nx - 1) // L["sx"], (ny - 1) // L["sy"]
        ox, oy = (mx // 2, my // 2) if shifted else (0, 0)
        f[:, ox::mx] = True
        f[oy::my, :] = True
    return f


def perona_malik(mesh: np.ndarray, dt: float, k: float, steps: int, L: dict = None,
                 shifted: bool = False) -> np.ndarray:
    """`steps` FTCS steps of u_t = div(exp(-|grad u|^2/k^2) grad u) for u = x
    and u = y over the computational grid (eq. (12)); L given: its interface
    lines are fixed too, i.e. every subdomain is smoothed on its own (with
    shifted, the subdomains moved by half their size)."""
    u = np.array(mesh, dtype=np.float64)
    ny, nx = u.shape[0], u.shape[1]
    hx, hy = 1.0 / (nx - 1), 1.0 / (ny - 1)
    free = ~fixed_nodes(nx, ny, L, shifted)
    for _ in range(steps):
        P = u[1:-1, 1:-1]
        dE = u[1:-1, 2:] - P
        dW = u[1:-1, :-2] - P
        dN = u[2:, 1:-1] - P
        dS = u[:-2, 1:-1] - P
        cE = np.exp(-(dE / hx) ** 2 / k**2)
        cW = np.exp(-(dW / hx) ** 2 / k**2)
        cN = np.exp(-(dN / hy) ** 2 / k**2)
        cS = np.exp(-(dS / hy) ** 2 / k**2)
        new = u.copy()
        upd = P + dt * ((cE * dE + cW * dW) / hx**2 + (cN * dN + cS * dS) / hy**2)
        inner = new[1:-1, 1:-1]
        m = free[1:-1, 1:-1]
        inner[m] = upd[m]
        u = new
    return u


def ftcs_stable(nx: int, ny: int, dt: float) -> bool:
    """The update is a convex combination of the old values when
    dt (2/h_xi^2 + 2/h_eta^2) <= 1 (c <= 1)."""
    return dt * (2.0 * (nx - 1) ** 2 + 2.0 * (ny - 1) ** 2) <= 1.0


# ------------------------------------------------- interface pre-smoothing

def loess_value(t: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Weighted quadratic least squares at t = 0 of points (t_j, y_j[:, c]),
    tricube weights with d = max |t_j|."""
    d = np.max(np.abs(t))
    w = (1.0 - (np.abs(t) / d) ** 3) ** 3
    V = np.stack([np.ones_like(t), t / d, (t / d) ** 2], 1)
    sw = np.sqrt(w)[:, None]
    coef, *_ = np.linalg.lstsq(V * sw, y * sw, rcond=None)
    return coef[0]


def loess_line(values: np.ndarray, s: np.ndarray, fixed: np.ndarray, span: int) -> np.ndarray:
    """Smoothed copy of one line of values [n][2] at parameters s[n]; fixed
    points are kept."""
    n = values.shape[0]
    out = values.copy()
    for i in range(n):
        if fixed[i]:
            continue
        a = min(max(i - span // 2, 0), n - span)
        idx = np.arange(a, a + span)
        out[i] = loess_value(s[idx] - s[i], values[idx])
    return out


def smooth_interfaces(L: dict, vert: np.ndarray, horiz: np.ndarray, span: int) -> Tuple[np.ndarray, np.ndarray]:
    """Each full interface line smoothed on its own (vert [sx-1][ny][2],
    horiz [sy-1][nx][2]); outer-boundary ends and crosspoints stay."""
    nx, ny, sx, sy = L["nx"], L["ny"], L["sx"], L["sy"]
    mx, my = (nx - 1) // sx, (ny - 1) // sy
    v = np.array(vert, dtype=np.float64)
    h = np.array(horiz, dtype=np.float64)
    fv = np.zeros(ny, dtype=bool)
    fv[::my] = True
    fh = np.zeros(nx, dtype=bool)
    fh[::mx] = True
    sv = np.arange(ny) / (ny - 1)
    sh = np.arange(nx) / (nx - 1)
    for a in range(sx - 1):
        v[a] = loess_line(v[a], sv, fv, span)
    for b in range(sy - 1):
        h[b] = loess_line(h[b], sh, fh, span)
    return v, h
