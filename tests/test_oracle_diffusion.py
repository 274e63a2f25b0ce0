"""Pins of the diffusion-limit solvers and of the AP oracle's stability.

* Barenblatt: with the a d_t T^4 term dropped the limits (1.3)/(1.5) are the
  porous-medium equations T_t = D (T^q)_xx (q = 4, D = ac/(3 sigma Cv);
  q = 7, D = 4ac/(21 sigma Cv)); both the implicit solvers (6.1)/(6.7) and
  the three-stage scheme (2.7)/(2.9) must converge to the closed form.
* the three-stage scheme moves a compactly supported front, the two-stage
  scheme (2.8) does not (the remark after (2.8)).
* the three-stage and fully implicit solvers converge to each other on the
  striped-opacity problem of Fig. 1 ((6.2), sigma0 = 0.2).
* Tables 1 and 2 (golden fixture): at dx = 1/100 the AP oracle stays below the
  initial maximum at the printed C and overshoots it at three times that C.
"""
import os

import numpy as np
import pytest

from oracle.ap1d import Physics, ap_step
from oracle.diffusion1d import (barenblatt, face_sigma, implicit_step,
                                three_stage_step, two_stage_step)
from oracle.quadrature import gauss_legendre_pairs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "stability_tables.txt")


def _barenblatt_errors(q, solver, Ns=(50, 100, 200)):
    D = (1.0 / 3.0) if q == 4 else (4.0 / 21.0)
    # support stays inside [0, 1]: half-width sqrt(C/k) (D t)^(1/(q+1))
    Cb, t0, t1 = (0.05 if q == 4 else 0.01), 0.01, 0.05
    errs = []
    for N in Ns:
        x = (np.arange(N) + 0.5) / N
        T = barenblatt(x, t0, q, D, Cb)
        dt = 0.1 / N
        steps = int(round((t1 - t0) / dt))
        for _ in range(steps):
            T = solver(T, N, dt)
        errs.append(np.sum(np.abs(T - barenblatt(x, t0 + steps * dt, q, D, Cb))) / N)
    return errs


@pytest.mark.parametrize("q", [4, 7])
def test_implicit_solver_converges_to_barenblatt(q):
    def solver(T, N, dt):
        return implicit_step(T, np.ones(N - 1), dt, q=q, a_time=0.0)
    errs = _barenblatt_errors(q, solver)
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] / errs[2] > 2.0, errs   # the steep q = 7 front converges slowly
    assert errs[2] < 5e-3


@pytest.mark.parametrize("q", [4, 7])
def test_three_stage_converges_to_barenblatt(q):
    m = 0 if q == 4 else 3

    def solver(T, N, dt):
        return three_stage_step(T, np.ones(N), dt, m=m, a_time=0.0)[0]
    errs = _barenblatt_errors(q, solver)
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] / errs[2] > 2.0, errs   # the steep q = 7 front converges slowly
    assert errs[2] < 5e-3


def test_front_moves_three_stage_not_two_stage():
    N = 100
    x = (np.arange(N) + 0.5) / N
    T0 = np.maximum(1 - 40 * (x - 0.5) ** 2, 0.0)
    cold = T0 == 0
    for m in (0, 3):
        T3, _ = three_stage_step(T0, np.ones(N), 1e-3, m=m)
        T2 = two_stage_step(T0, np.ones(N), 1e-3, m=m)
        assert np.any(T3[cold] > 0)
        assert np.all(T2[cold] == 0)


def _striped(x, s0=0.2):
    return np.where(((x >= 0.2) & (x <= 0.35)) | ((x >= 0.65) & (x <= 0.8)), s0, 1.0)


def test_three_stage_and_implicit_agree_on_striped_opacity():
    # Fig. 1 setup: T0 = max(sin 2 pi (x - 1/4), 0)^(1/4), sigma (6.2) with
    # sigma0 = 0.2, dt = 0.05 dx; the two solvers converge to each other.
    diffs = []
    for N in (50, 100, 200):
        x = (np.arange(N) + 0.5) / N
        T0 = np.maximum(np.sin(2 * np.pi * (x - 0.25)), 0.0) ** 0.25
        sig_cell = _striped(x)
        sig_face = _striped(np.arange(1, N) / N)
        dt = 0.05 / N
        Ta = T0.copy()
        Tb = T0.copy()
        for _ in range(int(round(0.05 / dt))):
            Ta, _ = three_stage_step(Ta, sig_cell, dt)
            Tb = implicit_step(Tb, sig_face, dt, q=4)
        diffs.append(np.sum(np.abs(Ta - Tb)) / N)
    assert diffs[0] > diffs[1] > diffs[2], diffs
    assert diffs[2] < 2e-3


def _golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                t = line.split()
                rows.append((int(t[0]), float(t[1]), [float(v) for v in t[2:]]))
    return rows


def _max_T(N, C, eps, m, tend=0.1):
    mu, om = gauss_legendre_pairs(16)
    P = mu.size
    x = (np.arange(N) + 0.5) / N
    T = np.maximum(1 - 40 * (x - 0.5) ** 2, 0.0)
    E = np.repeat((T ** 4)[:, None], P, 1)
    O = np.zeros((N + 1, P))
    ph = Physics(eps=eps, dt=C / N, m=m)
    mx = 0.0
    for _ in range(int(np.ceil(tend / ph.dt))):
        r = ap_step(E, O, T, np.ones(N), mu, om, np.zeros(P), np.zeros(P), ph)
        E, O, T = r["E"], r["O"], r["T"]
        assert np.all(np.isfinite(T)) and T.min() >= 0
        mx = max(mx, float(T.max()))
    return mx


@pytest.mark.slow
@pytest.mark.parametrize("table,eps", [(1, 1e-3), (2, 1e-3), (1, 1.0)])
def test_stability_tables_at_dx_1_100(table, eps):
    rows = {(t, e): cs for t, e, cs in _golden_rows()}
    C = rows[(table, eps)][2]          # dx = 1/100 column
    m = 0 if table == 1 else 3
    assert _max_T(100, C, eps, m) <= 1.0
    if eps < 1:
        assert _max_T(100, 3 * C, eps, m) > 1.0


@pytest.mark.parametrize("m", [0, 3])
def test_semi_cor_limit_conserves_its_own_sum(m):
    """The (3.14) limit update a (U* - U^n) + Cv (T^{n+1} - T^n) = dt div(F grad U*)
    telescopes with closed ends: sum(a U* + Cv T^{n+1}) = sum(a U^n + Cv T^n) to
    rounding -- while the energy with U^{n+1} = (T^{n+1})^4 does not balance."""
    from oracle.diffusion1d import semi_cor_step
    N = 80
    x = (np.arange(N) + 0.5) / N
    T = 0.5 + 0.3 * np.cos(2 * np.pi * x) + 0.1 * np.sin(6 * np.pi * x)
    sig = 0.5 + np.random.default_rng(3).uniform(0, 1.5, N)
    T1, Us = semi_cor_step(T, sig, 0.5 / N, m=m)
    before = np.sum(T ** 4 + T)
    assert abs(np.sum(Us + T1) - before) < 1e-13 * before
    assert abs(np.sum(T1 ** 4 + T1) - before) > 1e-8 * before


def test_semi_cor_limit_first_order_on_smooth_data():
    """sigma independent of T, smooth data, closed ends: the (3.14) limit
    converges at first order to the implicit reference (6.1) under refinement
    (the case the paper reports as behaving well)."""
    from oracle.diffusion1d import semi_cor_step
    errs = []
    for N in (50, 100, 200):
        x = (np.arange(N) + 0.5) / N
        T = 0.5 + 0.4 * np.cos(2 * np.pi * x)
        Tr = T.copy()
        dt = 0.5 / N
        for _ in range(int(round(0.05 / dt))):
            T, _ = semi_cor_step(T, np.ones(N), dt, m=0)
            Tr = implicit_step(Tr, np.ones(N - 1), dt, q=4)
        errs.append(np.mean(np.abs(T - Tr)))
    assert errs[0] / errs[1] > 1.7 and errs[1] / errs[2] > 1.7, errs
