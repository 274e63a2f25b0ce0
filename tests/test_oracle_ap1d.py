"""Pins of the 1-D AP oracle against what the paper and the mathematics fix.

* equilibrium: a uniform Planckian state with matching inflow is a fixed point;
* free streaming (sigma = 0): T is untouched, prediction and correction
  coincide, the uniform two-stream state is an exact fixed point, and the
  solution converges (first order) to the exact transport solution;
* mirror symmetry x -> L - x (b_L <-> b_R, O -> -O);
* the fully discrete conservation identity (3.13) per cell;
* the eps -> 0 limit: the AP step approaches the three-stage diffusion scheme
  (2.7) / (2.9), which Section 4's limit analysis says it reduces to;
* the assembled systems satisfy (4.5a-c), (4.6), (4.11a,b), (4.13)
  evaluated equation by equation (an assembly check).
"""
import numpy as np
import pytest

from oracle.ap1d import Physics, ap_step, node_sigma
from oracle.diffusion1d import three_stage_step
from oracle.energy import conservation_terms
from oracle.quadrature import gauss_legendre_pairs


def _rand_state(N, P, rng, T_lo=0.2, T_hi=1.0):
    T = rng.uniform(T_lo, T_hi, N)
    E = (T ** 4)[:, None] * rng.uniform(0.8, 1.2, (N, P))
    O = rng.normal(size=(N + 1, P)) * 0.1
    return E, O, T


@pytest.mark.parametrize("quad", ["dyadic", "gl"])
@pytest.mark.parametrize("m", [0, 3])
@pytest.mark.parametrize("eps", [1.0, 1e-2, 1e-4])
def test_equilibrium_is_fixed_point(m, eps, quad):
    # With weights summing exactly to one the Planckian is an exact fixed
    # point; with rounded Gauss-Legendre weights (sum 1 +- 1e-16) the stiff
    # coupling amplifies that rounding by ~eps^-2, hence the looser bound.
    N = 16
    if quad == "gl":
        mu, om = gauss_legendre_pairs(8)
        tol = 1e-13 + 1e-17 / eps ** 2
    else:
        mu = (np.arange(4) + 0.5) / 4
        om = np.full(4, 0.25)
        tol = 1e-12     # ac beta reaches ~1e7 at eps = 1e-4 here
    P = mu.size
    rng = np.random.default_rng(1)
    sig = rng.uniform(0.5, 2.0, N)
    # a c T0^4 exactly representable, so the initial state is exactly Planckian
    T0 = 0.75
    ph = Physics(a=2.0, c=0.5, Cv=2.1, eps=eps, dt=0.5 / N, m=m)
    acU = ph.a * ph.c * T0 ** 4
    E = np.full((N, P), acU)
    O = np.zeros((N + 1, P))
    T = np.full(N, T0)
    b = np.full(P, acU)
    r = ap_step(E, O, T, sig, mu, om, b, b, ph)
    assert np.max(np.abs(r["T"] - T0)) < tol
    assert np.max(np.abs(r["E"] - acU)) < tol * acU
    assert np.max(np.abs(r["O"])) < 10 * tol * acU / min(eps, 1.0)


@pytest.mark.parametrize("eps", [1.0, 1e-3])
def test_free_streaming_fixed_point_and_stage_coincidence(eps):
    # sigma = 0: E_p = (bL+bR)/2, O_p = (bL-bR)/(2 eps) satisfies every equation
    # of (4.5) and (4.6) with a non-zero flux.
    N, nv = 12, 8
    mu, om = gauss_legendre_pairs(nv)
    P = mu.size
    rng = np.random.default_rng(2)
    bL = rng.uniform(0.5, 2.0, P)
    bR = rng.uniform(0.0, 1.0, P)
    E = np.tile((bL + bR) / 2, (N, 1))
    O = np.tile((bL - bR) / (2 * eps), (N + 1, 1))
    T = rng.uniform(0.1, 1.0, N)
    for m in (0, 3):
        ph = Physics(eps=eps, dt=0.3 / N, m=m)
        r = ap_step(E, O, T, np.zeros(N), mu, om, bL, bR, ph)
        assert np.array_equal(r["T"], T)
        assert np.max(np.abs(r["E"] - E)) < 1e-14
        assert np.max(np.abs(r["O"] - O)) < 1e-13 * np.max(np.abs(O))
        # prediction and correction solve the same system at sigma = 0
        E2, O2, T2 = _rand_state(N, P, rng)
        r2 = ap_step(E2, O2, T2, np.zeros(N), mu, om, bL, bR, ph)
        assert np.array_equal(r2["T"], T2)
        assert np.max(np.abs(r2["E"] - r2["E_star"])) < 1e-14 * np.max(np.abs(r2["E"]))
        assert np.max(np.abs(r2["O"] - r2["O_star"])) < 1e-13 * np.max(np.abs(r2["O"]))


def _bump(x):
    return np.maximum(1.0 - 40.0 * (x - 0.5) ** 2, 0.0) ** 2


def test_free_streaming_converges_to_exact_transport():
    # (1/c) I_t + (v/eps) I_x = 0 with zero inflow: I(t,x,v) = I0(x - c v t/eps).
    nv = 8
    mu, om = gauss_legendre_pairs(nv)
    P = mu.size
    eps, c, tend = 1.0, 1.0, 0.1
    errs = []
    for N in (50, 100, 200, 400):
        x = (np.arange(N) + 0.5) / N
        ph = Physics(eps=eps, c=c, dt=0.5 / N, m=0)
        E = np.tile(_bump(x)[:, None], (1, P))
        O = np.zeros((N + 1, P))
        T = np.full(N, 0.5)
        steps = int(round(tend / ph.dt))
        for _ in range(steps):
            r = ap_step(E, O, T, np.zeros(N), mu, om, np.zeros(P), np.zeros(P), ph)
            E, O, T = r["E"], r["O"], r["T"]
        shift = c * mu[None, :] * tend / eps
        Eex = 0.5 * (_bump(x[:, None] - shift) + _bump(x[:, None] + shift))
        errs.append(np.sum(np.abs(E - Eex) @ om) / N)
    ratios = [errs[k] / errs[k + 1] for k in range(len(errs) - 1)]
    # implicit Euler in time at fixed CFL: first order
    assert all(1.6 < q < 2.6 for q in ratios), (errs, ratios)


@pytest.mark.parametrize("m", [0, 3])
@pytest.mark.parametrize("eps", [1.0, 1e-2, 1e-4])
def test_mirror_symmetry(m, eps):
    N, nv = 14, 8
    mu, om = gauss_legendre_pairs(nv)
    P = mu.size
    rng = np.random.default_rng(3)
    E, O, T = _rand_state(N, P, rng)
    sig = rng.uniform(0.3, 3.0, N)
    bL = rng.uniform(0.5, 1.5, P)
    bR = rng.uniform(0.0, 0.5, P)
    ph = Physics(a=1.1, c=1.7, Cv=0.6, eps=eps, dt=0.4 / N, m=m)
    r = ap_step(E, O, T, sig, mu, om, bL, bR, ph)
    q = ap_step(E[::-1], -O[::-1], T[::-1], sig[::-1], mu, om, bR, bL, ph)
    # the mirrored run rounds differently; this state is far from equilibrium
    # and at small eps the stiff coupling (ac beta ~ 1e7 here) amplifies
    # rounding, so the bound grows as eps shrinks.  A sign or index mistake
    # shows up as an O(1) asymmetry.
    tol = 1e-13 * max(1.0, (1e-2 / eps) ** 2)
    sc = np.max(np.abs(r["E"]))
    assert np.max(np.abs(q["E"][::-1] - r["E"])) < tol * sc
    assert np.max(np.abs(-q["O"][::-1] - r["O"])) < 10 * tol * np.max(np.abs(r["O"]))
    assert np.max(np.abs(q["T"][::-1] - r["T"])) < tol * np.max(r["T"])


@pytest.mark.parametrize("m", [0, 3])
@pytest.mark.parametrize("eps", [1.0, 1e-2, 1e-4])
def test_conservation_identity_per_cell(m, eps):
    # sum of (4.13) and of (4.11b) over directions: the fully discrete (3.13)
    N, nv = 20, 16
    mu, om = gauss_legendre_pairs(nv)
    P = mu.size
    rng = np.random.default_rng(4)
    E, O, T = _rand_state(N, P, rng)
    sig = rng.uniform(0.5, 2.0, N)
    bL = np.ones(P)
    bR = np.zeros(P)
    ph = Physics(a=1.0, c=1.0, Cv=1.0, eps=eps, dt=0.5 / N, m=m)
    r = ap_step(E, O, T, sig, mu, om, bL, bR, ph)
    lhs, rhs, sc = conservation_terms(r, E, T, sig, mu, om, ph)
    assert np.max(np.abs(lhs - rhs) / sc) < 1e-12
    # summed over cells, D* telescopes to the boundary fluxes of O*
    dx = 1.0 / N
    flux = (r["O_star"][-1] - r["O_star"][0]) @ (mu * om)
    assert abs(np.sum(dx * r["D"]) - flux) < 1e-12 * (abs(flux) + np.sum(dx * np.abs(r["D"])))


@pytest.mark.parametrize("m", [0, 3])
def test_eps_to_zero_reaches_three_stage_diffusion(m):
    # IC (6.3), sigma = 1, zero inflow, dt = 0.1 dx: the AP step tends to the
    # three-stage scheme (2.7)/(2.9) as eps -> 0, at the rate eps^2.
    N, nv = 50, 16
    mu, om = gauss_legendre_pairs(nv)
    P = mu.size
    x = (np.arange(N) + 0.5) / N
    T0 = np.maximum(1 - 40 * (x - 0.5) ** 2, 0.0)
    diffs = []
    for eps in (1e-2, 1e-3, 1e-4):
        ph = Physics(eps=eps, dt=0.1 / N, m=m)
        T = T0.copy()
        E = np.repeat((T ** 4)[:, None], P, 1)
        O = np.zeros((N + 1, P))
        Td = T0.copy()
        for _ in range(10):
            r = ap_step(E, O, T, np.ones(N), mu, om, np.zeros(P), np.zeros(P), ph)
            E, O, T = r["E"], r["O"], r["T"]
            Td, _ = three_stage_step(Td, np.ones(N), ph.dt, m=m, corr_K="old")
        diffs.append(np.max(np.abs(T - Td)))
    assert diffs[2] < 1e-5
    assert diffs[0] / diffs[1] > 50 and diffs[1] / diffs[2] > 50, diffs


def _residuals_by_equation(E, O, T, sig, mu, om, bL, bR, ph, r):
    """Evaluate every equation of the step, element by element, in binary64."""
    N, P = E.shape
    a, c, Cv, eps, dt, m = ph.a, ph.c, ph.Cv, ph.eps, ph.dt, ph.m
    dx = ph.L / N
    sn = node_sigma(sig)
    Kc = np.ones(N) if m == 0 else T ** m
    Es, Os, Us = r["E_star"], r["O_star"], r["U_star"]
    rho_s = Es @ om
    out = []
    for p in range(P):
        v = mu[p]
        for i in range(1, N):           # (4.5a) / (5.2a)
            K = 0.5 * (Kc[i - 1] + Kc[i])
            lhs = K * ((Os[i, p] - O[i, p]) / (c * dt) + v * (Es[i, p] - Es[i - 1, p]) / (eps ** 2 * dx))
            rhs = -sn[i - 1] * Os[i, p] / eps ** 2
            out.append(abs(lhs - rhs) / (abs(lhs) + abs(rhs) + abs(K * v * Es[i, p] / (eps ** 2 * dx)) + 1e-300))
        for j in range(N):              # (4.5b) / (5.2b)
            lhs = Kc[j] * ((Es[j, p] - E[j, p]) / (c * dt) + v * (Os[j + 1, p] - Os[j, p]) / dx)
            rhs = sig[j] * (a * c * Us[j] - Es[j, p]) / eps ** 2
            sc = abs(Kc[j] * Es[j, p] / (c * dt)) + abs(Kc[j] * v * Os[j, p] / dx) + abs(sig[j] * Es[j, p] / eps ** 2)
            out.append(abs(lhs - rhs) / (sc + 1e-300))
        # (4.6)
        out.append(abs(Es[0, p] + eps / 2 * (Os[0, p] + Os[1, p]) - bL[p]) / (abs(bL[p]) + abs(Es[0, p]) + 1e-300))
        out.append(abs(Es[-1, p] - eps / 2 * (Os[-1, p] + Os[-2, p]) - bR[p]) / (abs(bR[p]) + abs(Es[-1, p]) + 1e-300))
    for j in range(N):                  # (4.5c) / (5.2c)
        lhs = Cv * (Us[j] - T[j] ** 4) / dt
        rhs = 4 * sig[j] * T[j] ** (3 - m) * (rho_s[j] - a * c * Us[j]) / eps ** 2
        sc = abs(Cv * Us[j] / dt) + abs(Cv * T[j] ** 4 / dt) + abs(4 * sig[j] * T[j] ** (3 - m) * rho_s[j] / eps ** 2)
        out.append(abs(lhs - rhs) / sc)
    # (4.13): T^{n+1}
    Tn1 = r["T"]
    rho_n = E @ om
    D = ((Os[1:] - Os[:-1]) * mu) @ om / dx
    Ks = r["K_star"]
    for j in range(N):
        lhs = (a * c * Tn1[j] ** 4 + eps ** 2 * Ks[j] * Cv * (Tn1[j] - T[j]) / (sig[j] * dt)) / (c * dt) \
            + Cv * (Tn1[j] - T[j]) / dt
        rhs = rho_n[j] / (c * dt) - D[j]
        out.append(abs(lhs - rhs) / (abs(a * Tn1[j] ** 4 / dt) + abs(Cv * T[j] / dt) + abs(rho_n[j] / (c * dt)) + abs(D[j])))
    # (4.11a,b) with (4.12): E = ac U + eps E_J, O = O_J
    U1 = Tn1 ** 4
    K1 = np.ones(N) if m == 0 else Tn1 ** m
    EJ, OJ = r["E_J"], r["O_J"]
    for p in range(P):
        v = mu[p]
        for i in range(1, N):
            K = 0.5 * (K1[i - 1] + K1[i])
            lhs = K * ((OJ[i, p] - O[i, p]) / (c * dt) + a * c * v * (U1[i] - U1[i - 1]) / (eps ** 2 * dx)
                       + v * (EJ[i, p] - EJ[i - 1, p]) / (eps * dx))
            rhs = -sn[i - 1] * OJ[i, p] / eps ** 2
            sc = abs(K * OJ[i, p] / (c * dt)) + abs(K * O[i, p] / (c * dt)) + abs(K * a * c * v * U1[i] / (eps ** 2 * dx)) \
                + abs(K * v * EJ[i, p] / (eps * dx)) + abs(rhs)
            out.append(abs(lhs - rhs) / (sc + 1e-300))
        for j in range(N):
            lhs = K1[j] * ((a * c * U1[j] + eps * EJ[j, p] - E[j, p]) / (c * dt) + v * (OJ[j + 1, p] - OJ[j, p]) / dx)
            rhs = -sig[j] * EJ[j, p] / eps
            sc = abs(K1[j] * a * c * U1[j] / (c * dt)) + abs(K1[j] * E[j, p] / (c * dt)) + abs(K1[j] * v * OJ[j, p] / dx) + abs(rhs)
            out.append(abs(lhs - rhs) / (sc + 1e-300))
        E1 = a * c * U1 + eps * EJ[:, p]
        out.append(abs(E1[0] + eps / 2 * (OJ[0, p] + OJ[1, p]) - bL[p]) / (abs(bL[p]) + abs(E1[0])))
        out.append(abs(E1[-1] - eps / 2 * (OJ[-1, p] + OJ[-2, p]) - bR[p]) / (abs(bR[p]) + abs(E1[-1])))
    return np.array(out)


@pytest.mark.parametrize("m", [0, 3])
@pytest.mark.parametrize("eps", [1.0, 1e-3])
def test_every_equation_holds(m, eps):
    N, nv = 9, 6
    mu, om = gauss_legendre_pairs(nv)
    P = mu.size
    rng = np.random.default_rng(5)
    E, O, T = _rand_state(N, P, rng)
    sig = rng.uniform(0.5, 2.0, N)
    bL = rng.uniform(0.5, 1.5, P)
    bR = rng.uniform(0.0, 0.3, P)
    ph = Physics(a=0.8, c=1.3, Cv=1.7, eps=eps, dt=0.5 / N, m=m)
    r = ap_step(E, O, T, sig, mu, om, bL, bR, ph)
    res = _residuals_by_equation(E, O, T, sig, mu, om, bL, bR, ph, r)
    assert res.max() < 1e-12
