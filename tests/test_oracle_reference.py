"""Pins of the iterative implicit reference solver (6.6) in the oracle.

* sigma independent of T (m = 0): the opacity is not updated, one Picard
  iteration is the whole solve, and the result is the prediction of the AP
  step (E*, O*, U*) exactly;
* a Planckian uniform state with matching inflow is a fixed point;
* both schemes are consistent with the same equations, so from a smooth state
  the reference and the AP step differ by O(dt^2) per step: halving dt divides
  the one-step difference by about four.
"""
import numpy as np

from oracle.ap1d import Physics, ap_step, implicit_reference_step
from oracle.quadrature import gauss_legendre_pairs


def _smooth_state(N, nv, eps, m, a=1.0, c=1.0):
    mu, om = gauss_legendre_pairs(nv)
    x = (np.arange(N) + 0.5) / N
    T = 0.6 + 0.2 * np.sin(2 * np.pi * x)
    E = np.repeat((a * c * T ** 4)[:, None], mu.size, axis=1)
    O = np.zeros((N + 1, mu.size))
    b = a * c * T[0] ** 4 * np.ones(mu.size), a * c * T[-1] ** 4 * np.ones(mu.size)
    return mu, om, T, E, O, b


def test_temperature_independent_opacity_is_one_prediction():
    N, nv = 40, 8
    mu, om, T, E, O, (bL, bR) = _smooth_state(N, nv, 1e-2, 0)
    ph = Physics(eps=1e-2, dt=0.5 / N, m=0)
    s0 = np.linspace(0.5, 2.0, N)
    r = implicit_reference_step(E, O, T, s0, mu, om, bL, bR, ph)
    a = ap_step(E, O, T, s0, mu, om, bL, bR, ph)
    assert r["converged"] and r["iterations"] <= 2
    assert np.max(np.abs(r["E"] - a["E_star"])) <= 1e-15 * np.max(np.abs(a["E_star"]))
    assert np.max(np.abs(r["U"] - a["U_star"])) <= 1e-15 * np.max(np.abs(a["U_star"]))


def test_planckian_equilibrium_is_a_fixed_point():
    N, nv, T0 = 30, 8, 0.75
    mu, om = gauss_legendre_pairs(nv)
    T = np.full(N, T0)
    E = np.full((N, nv // 2), T0 ** 4)
    O = np.zeros((N + 1, nv // 2))
    b = np.full(nv // 2, T0 ** 4)
    ph = Physics(eps=1.0, dt=0.5 / N, m=3)
    r = implicit_reference_step(E, O, T, np.ones(N), mu, om, b, b, ph)
    assert r["converged"]
    assert np.max(np.abs(r["T"] - T0)) <= 1e-12
    assert np.max(np.abs(r["E"] - T0 ** 4)) <= 1e-12


def test_reference_and_ap_step_agree_to_second_order_per_step():
    N, nv, eps = 50, 8, 1.0
    mu, om, T, E, O, (bL, bR) = _smooth_state(N, nv, eps, 3)
    s0 = np.ones(N)
    diffs = []
    for dt in (0.04, 0.02, 0.01):
        ph = Physics(eps=eps, dt=dt, m=3)
        r = implicit_reference_step(E, O, T, s0, mu, om, bL, bR, ph)
        a = ap_step(E, O, T, s0, mu, om, bL, bR, ph)
        assert r["converged"]
        diffs.append(np.max(np.abs(r["T"] - a["T"])))
    assert diffs[0] / diffs[1] > 3.0 and diffs[1] / diffs[2] > 3.0, diffs
