"""Pins of the oracle's exponential time stepping (Sec. 2.2: every step
length an independent exponential variate with density lambda e^{-lambda t},
and the boundary test made both at the end of the step and through the
conditional probability of a crossing within it).

Our reading: step k has length tau_k = -ln(u_k) dt (mean dt = 1/lambda), the
step is X + b(X) tau + sqrt(2 tau) Z (for constant b the exact law of the
diffusion after time tau), and the crossing test is the Brownian bridge's
with tau in place of dt.  For w = 1 the scheme is then exact step by step,
which fixes two closed forms independent of the oracle's code:

* First passage through an exponential clock.  Brownian motion with
  diffusion coefficient 2 started a from a wall hits it before an
  independent Exp(lambda) time with probability E[e^{-lambda T_a}] =
  exp(-a sqrt(lambda)) (Laplace transform of the first-passage time).  The
  end of step k is a Gamma(k, lambda) time, so with c = a sqrt(lambda) the
  path has left by the end of step k with probability
      F_1 = e^{-c},  F_2 = e^{-c} (1 + c/2),  F_3 = e^{-c} (1 + 5c/8 + c^2/8)
  (the series sum_{i<k} (-lambda)^i / i! d^i/ds^i E[e^{-s T_a}] at s = lambda).
* Mean step count.  Step ends form a Poisson process of rate lambda
  independent of the path, so the step holding the exit time T is step
  N(T) + 1 and E[steps] = v(x0)/dt + 1 exactly, v the torsion function
  (Laplace v = -1, v = 0 on the boundary).

Beyond those: the sin^2 closed form to O(dt), the step-length law, the
counter block of the step lengths (word 3 = 2), float against double.
"""
import math

import numpy as np
import pytest
from scipy import stats

from tests.test_oracle_walk import closed_form_sin2, torsion

FLAT = {"base": 1.0, "terms": []}
IDENT = {"kind": "identity"}


def test_step_length_values_and_law(ref):
    dt = 1e-3
    # hand words: the low 23 bits give u = (q + 1/2) 2^-23
    w = np.array([0xFF800000, 0x007FFFFF, 0x00400000], dtype=np.uint32)
    tau = ref.expo_steps(w, dt)
    assert tau[0] == pytest.approx(24 * math.log(2.0) * dt, rel=1e-15)           # u = 2^-24
    assert tau[1] == pytest.approx(-math.log1p(-2.0**-24) * dt, rel=1e-9)        # u = 1 - 2^-24
    assert tau[2] == pytest.approx(-math.log((2**22 + 0.5) * 2.0**-23) * dt, rel=1e-15)
    # exponential with mean dt: Kolmogorov-Smirnov, mean and variance
    rng = np.random.default_rng(17)
    t = ref.expo_steps(rng.integers(0, 2**32, size=200000, dtype=np.uint64).astype(np.uint32), dt)
    assert np.all(t > 0)
    assert stats.kstest(t / dt, "expon").pvalue > 1e-3
    assert abs(t.mean() / dt - 1.0) < 4 / math.sqrt(t.size)
    assert abs(t.var() / dt**2 - 1.0) < 4 * math.sqrt(8 / t.size)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_first_passage_through_an_exponential_clock(ref, prec):
    dt = 1e-3
    lam = 1.0 / dt
    a = np.array([0.01, 0.03, 0.06])
    nodes = np.stack([a, np.full_like(a, 0.5)], 1)
    N = 400000
    # t_max = 3 dt: every path stops after at most three steps
    r = ref.interface_estimate(FLAT, IDENT, nodes, N, dt, 29, prec=prec, t_max=3 * dt, per_path=True,
                               exit_test="expo")
    pp = r["per_path"]
    exited = pp["capped"] == 0
    for i, ai in enumerate(a):
        c = ai * math.sqrt(lam)
        F = [math.exp(-c), math.exp(-c) * (1 + c / 2), math.exp(-c) * (1 + 5 * c / 8 + c * c / 8)]
        for k in (1, 2, 3):
            f = float((exited[i] & (pp["steps"][i] <= k)).mean())
            se = math.sqrt(F[k - 1] * (1 - F[k - 1]) / N)
            assert abs(f - F[k - 1]) <= 4.5 * se, (ai, k, f, F[k - 1])
        # the exits are through the near wall xi = 0; the walls eta = 0, 1 half
        # a unit away are reached within one step with probability
        # exp(-0.5 sqrt(lambda)) = 1.4e-7 each, ~0.2 exits per node here
        assert int((pp["side"][i][exited[i]] != 0).sum()) <= 3


def test_mean_step_count_is_torsion_over_dt_plus_one(ref):
    nodes = np.array([[0.5, 0.5], [0.1, 0.3], [0.05, 0.05], [0.8, 0.6]])
    dt = 1e-3
    r = ref.interface_estimate(FLAT, IDENT, nodes, 20000, dt, 31, per_path=True, exit_test="expo")
    k = r["per_path"]["steps"].astype(np.float64)
    want = np.array([torsion(*p) for p in nodes]) / dt + 1.0
    m, s = k.mean(1), k.std(1) / math.sqrt(k.shape[1])
    z = (m - want) / s
    assert np.all(np.abs(z) <= 4.3), z
    assert r["capped"] == 0


def test_closed_form_to_first_order(ref):
    import workloads as W
    c = W.cfg_sin2_sweep()
    d = c["density"]
    B = ref.Bmap(c["bmap"], d)
    xi = np.array([1, 8, 16, 32, 40, 64]) / 65.0
    nodes = np.stack([xi, np.full_like(xi, 0.5)], 1)
    exact = closed_form_sin2(xi)
    dt = 1e-3
    r = ref.interface_estimate(d, B, nodes, 40000, dt, 7, exit_test="expo")
    assert np.all(np.abs(r["mean"][:, 0] - exact) <= 4 * r["se"][:, 0] + 8 * dt)
    assert np.all(np.abs(r["mean"][:, 1] - 0.5) <= 4.3 * r["se"][:, 1])


def test_step_lengths_come_from_their_own_block(ref):
    # w = 1, three steps from (0.5, 0.5), then capped: the capped path takes
    # the nearest boundary point of X_3, which reveals X_3's other
    # coordinate; rebuild X_3 from the counter blocks (m, p, g, 0) (normals)
    # and (m, p, g, 2) (step lengths)
    dt, seed, g0 = 1e-3, 41, 0
    r = ref.interface_estimate(FLAT, IDENT, np.array([[0.5, 0.5]]), 64, dt, seed, t_max=3 * dt, per_path=True,
                               exit_test="expo")
    pp = r["per_path"][0]
    key = [seed & 0xFFFFFFFF, seed >> 32]
    checked = 0
    for p in range(64):
        if not pp["capped"][p]:
            continue
        nrm = ref.philox(np.array([[0, p, g0, 0]], dtype=np.uint32), key)[0]
        stp = ref.philox(np.array([[0, p, g0, 2]], dtype=np.uint32), key)[0]
        u = ref.block_uniforms(nrm[None, :])[0]
        tau = ref.expo_steps(stp[:3], dt)
        X = np.array([0.5, 0.5])
        for j in range(3):
            rad = math.sqrt(-2 * math.log(u[2 * j]))
            z = np.array([rad * math.cos(2 * math.pi * u[2 * j + 1]), rad * math.sin(2 * math.pi * u[2 * j + 1])])
            X = X + math.sqrt(2 * tau[j]) * z
        side = pp["side"][p]
        other = X[1] if side < 2 else X[0]
        got = pp["exit_eta"][p] if side < 2 else pp["exit_xi"][p]
        assert got == pytest.approx(other, abs=1e-12)
        checked += 1
    assert checked > 40


def test_float_agrees_with_double_and_differs_from_fixed_steps(ref):
    import workloads as W
    c = W.cfg_plain_fp64()
    nodes = np.array([[0.25, 0.5], [0.6, 0.4]])
    a = ref.interface_estimate(c["density"], c["bmap"], nodes, 4000, 1e-4, 9, per_path=True, exit_test="expo")
    b = ref.interface_estimate(c["density"], c["bmap"], nodes, 4000, 1e-4, 9, prec="fp32", per_path=True,
                               exit_test="expo")
    flips = (a["per_path"]["steps"] != b["per_path"]["steps"]).mean()
    assert flips < 5e-3
    assert np.abs(a["mean"] - b["mean"]).max() < 0.25 * a["se"].max()
    f = ref.interface_estimate(c["density"], c["bmap"], nodes, 4000, 1e-4, 9, per_path=True, exit_test="bridge")
    assert (f["per_path"]["steps"] != a["per_path"]["steps"]).mean() > 0.9
