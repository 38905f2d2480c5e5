"""Seeded synthetic workloads shared by the oracle and the HIP path.

This module is pure data plus seeded random draws.  It holds none of the
method's arithmetic: no walk, no density evaluation, no interpolation, no
finite differences.  Both sides (``oracle/`` and ``paper_1310_3435_amd``)
turn these plain dictionaries into their own native structures.

Vocabulary (Bihlo & Haynes, Sec. 2, eq. (5)-(7)):

* density ``w(xi, eta) = base + sum of terms`` is the diffusion coefficient
  of the linear Winslow generator ``div(w grad x) = 0``; every term is
  non-negative, so ``w >= base > 0``.
* the boundary map ``(x_b, y_b)`` is the Dirichlet data on the boundary of
  the computational unit square.
* a layout is a global ``nx x ny`` node grid on ``[0,1]^2`` split into
  ``sx x sy`` subdomains (Sec. 2.1, Fig. 1: interface points between
  non-overlapping subdomains).

Term kinds and their parameters (all terms are ``amp * f`` with ``amp >= 0``):

* ``gauss``: f = exp(-coef * ((xi-cx)^2 + (eta-cy)^2))
* ``ring``:  f = exp(-coef * (r - r0)^2), r = |(xi,eta) - (cx,cy)|
* ``sech2``: f = sech^2(coef * (nx*(xi-cx) + ny*(eta-cy)))
* ``sin2``:  f = sin^2(coef * (nx*(xi-cx) + ny*(eta-cy)))

Boundary-map kinds: ``identity``; ``affine`` (p = [x0, x_xi, x_eta, y0,
y_xi, y_eta]); ``annulus`` (p = [r0, r1, theta0, theta1]); ``edge1d`` (the
tangential coordinate on every edge solves the one-dimensional generator
along that edge, the convention of the paper's single-domain reference in
Sec. 3.2; it is tabulated with ``n_per_edge`` samples).
"""

from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

TWO_PI = 2.0 * math.pi


def _term(kind, amp, coef, cx=0.0, cy=0.0, r0=0.0, nx=0.0, ny=0.0):
    return {"kind": kind, "amp": float(amp), "coef": float(coef), "cx": float(cx),
            "cy": float(cy), "r0": float(r0), "nx": float(nx), "ny": float(ny)}


def density(base: float, terms: List[dict]) -> dict:
    return {"base": float(base), "terms": list(terms)}


# ---------------------------------------------------------------------------
# The five workloads.  Index 0 is the small FP64 case, index 1 the FP32 ring
# case that the throughput figure is quoted on.
# ---------------------------------------------------------------------------

def cfg_plain_fp64() -> dict:
    """Gaussian bump, identity map, two 33x33 subdomains split at xi=1/2."""
    return {
        "name": "plain_fp64_gauss",
        "density": density(1.0, [_term("gauss", 5.0, 50.0, 0.5, 0.5)]),
        "bmap": {"kind": "identity"},
        "layout": {"nx": 65, "ny": 33, "sx": 2, "sy": 1},
        "k": 15, "placement": "uniform", "interp": "linear",
        "paths": 2000, "dt": 1e-4, "seed": 1, "prec": "fp64",
    }


def cfg_ring_fp32() -> dict:
    """Ring density, 4x4 subdomains of 65x65, every interior interface node."""
    return {
        "name": "ring_fp32_4x4x65",
        "density": density(1.0, [_term("ring", 10.0, 200.0, 0.5, 0.5, r0=0.3)]),
        "bmap": {"kind": "identity"},
        "layout": {"nx": 257, "ny": 257, "sx": 4, "sy": 4},
        "k": 63, "placement": "uniform", "interp": "linear",
        "paths": 10000, "dt": 1e-5, "seed": 2, "prec": "fp32",
        "oracle_subset": 64,
    }


def cfg_annulus_fp32() -> dict:
    """Shear layer on a quarter annulus, 8x8 subdomains of 129x129."""
    return {
        "name": "annulus_fp32_8x8x129",
        "density": density(1.0, [_term("sech2", 20.0, 40.0, 0.0, 0.0, nx=1.0, ny=-1.0)]),
        "bmap": {"kind": "annulus", "p": [1.0, 2.0, 0.0, 0.5 * math.pi]},
        "layout": {"nx": 1025, "ny": 1025, "sx": 8, "sy": 8},
        "k": 32, "placement": "equidistributed", "interp": "pchip",
        "paths": 100000, "dt": 1e-5, "seed": 3, "prec": "fp32",
    }


def cfg_sin2_sweep() -> dict:
    """w depends on xi only: the interface values have a closed form."""
    return {
        "name": "sin2_bias_sweep",
        "density": density(1.0, [_term("sin2", 3.0, TWO_PI, 0.0, 0.0, nx=1.0, ny=0.0)]),
        "bmap": {"kind": "edge1d", "n_per_edge": 4097},
        "nodes": [(j / 65.0, 0.5) for j in range(1, 65)],
        "paths": 1000000, "dts": [1e-3, 1e-4, 1e-5, 1e-6], "seed": 5,
        "precs": ["fp32", "fp64"],
    }


def serving_requests(n_requests: int = 2000, master_seed: int = 4,
                     grids=(33, 65, 129, 257), splits=(2, 4, 8)) -> List[dict]:
    """Random mesh requests: 1-4 Gaussian bumps, grid and split drawn uniformly.

    Amplitudes U[1,20], widths (the exponent coefficient) U[20,200], centres
    U[0.15,0.85]^2; identity map; dt = 1e-4; every interior interface node is
    estimated; paths per node come from the requested standard error.
    """
    rng = np.random.default_rng(master_seed)
    out = []
    for r in range(n_requests):
        nb = int(rng.integers(1, 5))
        terms = [_term("gauss", rng.uniform(1.0, 20.0), rng.uniform(20.0, 200.0),
                       rng.uniform(0.15, 0.85), rng.uniform(0.15, 0.85)) for _ in range(nb)]
        n = int(rng.choice(grids))
        s = int(rng.choice([v for v in splits if (n - 1) % v == 0 and (n - 1) // v >= 4]))
        out.append({
            "id": r,
            "density": density(1.0, terms),
            "bmap": {"kind": "identity"},
            "layout": {"nx": n, "ny": n, "sx": s, "sy": s},
            "k": (n - 1) // s - 1, "placement": "uniform", "interp": "linear",
            "se_target": 1e-3, "pilot": 1024, "dt": 1e-4,
            "seed": int(rng.integers(1, 2**63 - 1)), "prec": "fp32",
        })
    return out


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 4) -> np.ndarray:
    """Arrival times (s) of a Poisson stream with the given rate."""
    rng = np.random.default_rng(seed + 1)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def random_nodes(n: int, seed: int, lo: float = 0.02, hi: float = 0.98) -> np.ndarray:
    """n start points drawn uniformly from [lo,hi]^2, shape (n, 2), float64."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, 2))


def random_density(seed: int, n_terms: int = 3) -> dict:
    """A density mixing every term kind, for parity tests."""
    rng = np.random.default_rng(seed)
    kinds = ["gauss", "ring", "sech2", "sin2"]
    terms = []
    for t in range(n_terms):
        kind = kinds[(seed + t) % 4]
        ang = rng.uniform(0, TWO_PI)
        terms.append(_term(kind, rng.uniform(0.5, 8.0), rng.uniform(5.0, 60.0) if kind != "sin2" else rng.uniform(1.0, 8.0),
                           rng.uniform(0.2, 0.8), rng.uniform(0.2, 0.8), r0=rng.uniform(0.05, 0.3),
                           nx=math.cos(ang), ny=math.sin(ang)))
    return density(rng.uniform(0.5, 2.0), terms)


def cfg_paper_example() -> dict:
    """The shape of the paper's running example (Sec. 3, its Gaussian monitor
    function with R = 15): w = 1 + 15 exp(-1/2) exp(-50 |(xi, eta) - (3/4, 1/2)|^2)
    on a 29 x 29 grid in four square subdomains, every interface node by
    Monte Carlo (Sec. 3.5) with N = 1e4; Brownian-bridge exits at dt = 1e-4."""
    return {
        "name": "paper_example_29",
        "density": density(1.0, [_term("gauss", 15.0 * math.exp(-0.5), 50.0, 0.75, 0.5)]),
        "bmap": {"kind": "identity"},
        "layout": {"nx": 29, "ny": 29, "sx": 2, "sy": 2},
        "k": 13, "placement": "uniform", "interp": "linear",
        "paths": 10000, "dt": 1e-4, "exit_test": "bridge", "seed": 6, "prec": "fp32",
    }


CONFIGS: Dict[str, callable] = {
    "plain_fp64_gauss": cfg_plain_fp64,
    "ring_fp32_4x4x65": cfg_ring_fp32,
    "annulus_fp32_8x8x129": cfg_annulus_fp32,
    "sin2_bias_sweep": cfg_sin2_sweep,
    "paper_example_29": cfg_paper_example,
}
