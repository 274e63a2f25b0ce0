"""Pins of the oracle's quadrature and scalar temperature solve.

Quadrature: the pair weights reproduce the angular average <f> = (1/2) int f
of Section 4 exactly for the polynomials a Gauss-Legendre rule integrates.
Newton: the normalised form of (4.13) is checked on cases solved by hand from
the printed equation, and against an independent bisection.
"""
import numpy as np
import pytest

from oracle.ap1d import Physics, bisect_temperature, newton_temperature
from oracle.linsolve import XP
from oracle.quadrature import gauss_legendre_pairs


@pytest.mark.parametrize("nv", [2, 4, 8, 16, 32, 64])
def test_pair_weights_integrate_even_moments(nv):
    mu, om = gauss_legendre_pairs(nv)
    assert mu.shape == (nv // 2,) and np.all(np.diff(mu) > 0) and np.all(mu > 0)
    # <v^(2k)> = (1/2) int_{-1}^{1} v^(2k) dv = 1/(2k+1), exact for 2k <= 2 nv - 1
    for k in range(nv):
        assert abs(np.sum(om * mu ** (2 * k)) - 1.0 / (2 * k + 1)) < 2e-15


def test_rho_equals_angular_average_of_isotropic_and_linear_intensity():
    # I(v) = A + B v: E = A, O = B v / eps, rho = <I> = A (odd part averages out)
    mu, om = gauss_legendre_pairs(16)
    assert abs(np.sum(om * 3.0) - 3.0) < 1e-14


def _ph(**kw):
    base = dict(a=1.0, c=1.0, Cv=1.0, eps=0.0, dt=1.0, m=0)
    base.update(kw)
    return Physics(**base)


@pytest.mark.parametrize("case", [
    # (4.13) with a=c=Cv=sigma=dt=1, eps=0:  T^4 + (T - Tn) = rho_n - D
    dict(ph=_ph(), Tn=0.5, rho=1.5, D=0.0, K=1.0, root=1.0),
    # same with a flux term: T^4 + T = 0.25 + 3 - 1.25 = 2
    dict(ph=_ph(), Tn=0.25, rho=3.0, D=1.25, K=1.0, root=1.0),
    # eps=1, K*=1: [T^4 + (T - Tn)] + (T - Tn) = rho_n - D  ->  T^4 + 2T = 3
    dict(ph=_ph(eps=1.0), Tn=0.5, rho=2.0, D=0.0, K=1.0, root=1.0),
    # c=2, eps=1: (1/2)[2T^4 + (T-Tn)] + (T-Tn) = rho_n/2 - D -> T^4 + 1.5T = 2.5
    dict(ph=_ph(c=2.0, eps=1.0), Tn=0.0, rho=5.0, D=0.0, K=1.0, root=1.0),
    # a=2, Cv=3, dt=0.5, eps=0: a(T^4-Tn... ) form: (1/(c dt))*a c T^4 + Cv(T-Tn)/dt = rho/(c dt) - D
    #   -> 4 T^4 + 6 (T - Tn) = 2 rho - D ;  Tn=1, rho=2, D=0 -> 4T^4 + 6T = 10 -> T=1
    dict(ph=_ph(a=2.0, Cv=3.0, dt=0.5), Tn=1.0, rho=2.0, D=0.0, K=1.0, root=1.0),
    # sigma/T^3 form, K* = 8: eps=1 -> [T^4 + 8 (T - Tn)] + (T - Tn) = rho - D
    #   Tn = 0.5, rho = 5.5 -> T^4 + 9T = 10 -> T = 1
    dict(ph=_ph(eps=1.0, m=3), Tn=0.5, rho=5.5, D=0.0, K=8.0, root=1.0),
])
def test_newton_hand_solved(case):
    one = lambda v: np.array([v], dtype=XP)
    T, its, conv = newton_temperature(one(case["Tn"]), one(case["rho"]), one(case["D"]),
                                      one(case["K"]), one(1.0), case["ph"])
    assert conv[0]
    assert abs(float(T[0]) - case["root"]) < 1e-15


def test_newton_matches_bisection_random():
    rng = np.random.default_rng(7)
    n = 4000
    for m in (0, 3):
        ph = Physics(a=1.0, c=1.0, Cv=1.0, eps=float(10 ** rng.uniform(-5, 0)), dt=1e-3, m=m)
        Tn = 10 ** rng.uniform(-3, 0.5, n)
        rho = 10 ** rng.uniform(-12, 1, n)
        D = rng.normal(size=n) * 10 ** rng.uniform(-3, 3, n)
        sig = 10 ** rng.uniform(-2, 3, n)
        K = 10 ** rng.uniform(-6, 1, n) if m else np.ones(n)
        args = [np.asarray(v, dtype=XP) for v in (Tn, rho, D, K, sig)]
        Tb, s = bisect_temperature(*args, ph)
        ok = s >= 0
        Tn_, its, conv = newton_temperature(*args, ph)
        assert np.all(conv[ok])
        rel = np.abs(Tn_[ok] - Tb[ok]) / np.maximum(np.maximum(Tb[ok], args[0][ok]), 1e-300)
        assert float(rel.max()) < 1e-15


def test_newton_zero_opacity_keeps_temperature():
    one = lambda v: np.array([v], dtype=XP)
    ph = Physics(eps=0.1, dt=1e-2)
    T, its, conv = newton_temperature(one(0.3), one(2.0), one(5.0), one(1.0), one(0.0), ph)
    assert float(T[0]) == 0.3
