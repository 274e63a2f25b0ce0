"""Pins of the 2-D AP oracle against what the paper and the mathematics fix.

* the direction set: weights, second moments, no direction parallel to an edge;
* reduction to 1-D: with y-periodic boundaries and y-independent data the 2-D
  step equals the (pinned) 1-D oracle's step with ordinates |mu_p| (the odd
  parity changes sign for the pairs whose mu_p < 0);
* transposition: exchanging x and y (the pairs relabelled by
  theta -> pi/2 - theta, edges swapped) transposes the solution; with the
  reduction above this fixes the y-direction rows by the x-direction ones;
* free streaming (sigma = 0): T is untouched, a spatially uniform state with
  matching inflow on all four edges is a fixed point, and smooth data converge
  first order to the exact solution I(t, x, Omega) = I0(x - c Omega t / eps)
  (which fixes the cross-derivative terms the two pins above cannot see);
* the per-cell conservation identity of the full step (the 2-D form of (3.13))
  and the telescoping of the flux divergence into the boundary outflow;
* every cell's temperature is the root of (4.13) (bisection on [0, s]);
* the thick limit: as eps -> 0 the step tends, at the rate eps^2, to the 2-D
  three-stage scheme (2.7)/(2.9) whose diffusion coefficient carries the
  dimension factor <mu^2> = 1/2 (not 1/3).
"""
import numpy as np
import pytest

from oracle import ap1d, ap2d
from oracle.ap1d import Physics, bisect_temperature
from oracle.quadrature import circle_pairs


def _state(g, P, rng, T_lo=0.3, T_hi=1.0):
    T = rng.uniform(T_lo, T_hi, (g.ny, g.nx))
    E = (T ** 4)[:, :, None] * rng.uniform(0.8, 1.2, (g.ny, g.nx, P))
    Ox = rng.normal(size=(g.ny, g.nx + 1, P)) * 0.1
    Oy = rng.normal(size=(g.ny + 1, g.nx, P)) * 0.1
    return E, Ox, Oy, T


def test_circle_directions():
    for nv in (4, 8, 32, 64):
        mu, eta, om = circle_pairs(nv)
        assert mu.size == nv // 2
        assert abs(om.sum() - 1) < 1e-15
        assert abs(om @ mu ** 2 - 0.5) < 1e-15
        assert abs(om @ eta ** 2 - 0.5) < 1e-15
        assert abs(om @ (mu * eta)) < 1e-15
        assert np.all(eta > 0) and np.all(np.abs(mu) > 1e-3)
        np.testing.assert_allclose(mu ** 2 + eta ** 2, 1, rtol=0, atol=1e-15)
    for bad in (2, 6, 10):
        with pytest.raises(ValueError):
            circle_pairs(bad)


@pytest.mark.parametrize("m", [0, 3])
@pytest.mark.parametrize("eps", [1.0, 1e-2])
def test_reduces_to_1d(m, eps):
    nx, ny, nv = 10, 3, 8
    g = ap2d.Grid2D(nx, ny, periodic_y=True)
    mu, eta, om = circle_pairs(nv)
    P = mu.size
    rng = np.random.default_rng(5)
    T1 = rng.uniform(0.3, 1.0, nx)
    E1 = (T1 ** 4)[:, None] * rng.uniform(0.8, 1.2, (nx, P))
    O1 = rng.normal(size=(nx + 1, P)) * 0.1          # odd parity of the 1-D pairs (|mu|)
    s1 = rng.uniform(0.5, 2.0, nx)
    bL, bR = rng.uniform(0, 1, P), rng.uniform(0, 0.5, P)
    sgn = np.sign(mu)
    E = np.broadcast_to(E1, (ny, nx, P)).copy()
    Ox = np.broadcast_to(O1 * sgn, (ny, nx + 1, P)).copy()
    Oy = np.broadcast_to(rng.normal(size=(nx, P)) * 0.1, (ny + 1, nx, P)).copy()
    T = np.broadcast_to(T1, (ny, nx)).copy()
    sig = np.broadcast_to(s1, (ny, nx)).copy()
    b = np.stack([bL, bR, np.zeros(P), np.zeros(P)])
    ph = Physics(a=1.3, c=0.7, Cv=1.1, eps=eps, dt=0.5 / nx, m=m)
    r2 = ap2d.ap_step(g, E, Ox, Oy, T, sig, mu, eta, om, b, ph)
    r1 = ap1d.ap_step(E1, O1, T1, s1, np.abs(mu), om, bL, bR, ph)
    for iy in range(ny):
        np.testing.assert_allclose(r2["T"][iy], r1["T"], rtol=1e-13, atol=0)
        np.testing.assert_allclose(r2["E"][iy], r1["E"], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(r2["Ox"][iy] * sgn, r1["O"], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(r2["E_star"][iy], r1["E_star"], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(r2["D"][iy], r1["D"], rtol=1e-11, atol=1e-12)


def _transpose_pairs(nv):
    """Pair q and sign s of the direction (eta_p, mu_p) (theta -> pi/2 - theta)."""
    P = nv // 2
    q = np.empty(P, dtype=int)
    s = np.empty(P)
    for p in range(P):
        if p < nv // 4:
            q[p], s[p] = nv // 4 - 1 - p, 1.0
        else:
            q[p], s[p] = 3 * nv // 4 - 1 - p, -1.0
    return q, s


@pytest.mark.parametrize("m", [0, 3])
def test_transposition(m):
    nx, ny, nv = 5, 4, 8
    g = ap2d.Grid2D(nx, ny, Lx=1.0, Ly=0.8)
    gt = ap2d.Grid2D(ny, nx, Lx=0.8, Ly=1.0)
    mu, eta, om = circle_pairs(nv)
    P = mu.size
    q, s = _transpose_pairs(nv)
    np.testing.assert_allclose(mu[q], eta * s, atol=1e-15)
    np.testing.assert_allclose(eta[q], mu * s, atol=1e-15)
    rng = np.random.default_rng(11)
    E, Ox, Oy, T = _state(g, P, rng)
    sig = rng.uniform(0.5, 3.0, (ny, nx))
    b = rng.uniform(0, 1, (4, P))
    ph = Physics(a=1.0, c=1.0, Cv=0.9, eps=0.05, dt=0.05, m=m)
    r = ap2d.ap_step(g, E, Ox, Oy, T, sig, mu, eta, om, b, ph)
    # transposed problem: cell (ix, iy), pair q(p); x-faces <- y-faces
    Et = np.empty((nx, ny, P)); Oxt = np.empty((nx, ny + 1, P)); Oyt = np.empty((nx + 1, ny, P))
    bt = np.empty((4, P))
    for p in range(P):
        Et[:, :, q[p]] = E[:, :, p].T
        Oxt[:, :, q[p]] = s[p] * Oy[:, :, p].T
        Oyt[:, :, q[p]] = s[p] * Ox[:, :, p].T
        bt[[2, 3, 0, 1], q[p]] = b[[0, 1, 2, 3], p]
    rt = ap2d.ap_step(gt, Et, Oxt, Oyt, T.T.copy(), sig.T.copy(), mu, eta, om, bt, ph)
    for p in range(P):
        np.testing.assert_allclose(rt["E"][:, :, q[p]], r["E"][:, :, p].T, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(rt["Ox"][:, :, q[p]], s[p] * r["Oy"][:, :, p].T, rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(rt["Oy"][:, :, q[p]], s[p] * r["Ox"][:, :, p].T, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(rt["T"], r["T"].T, rtol=1e-13, atol=0)


@pytest.mark.parametrize("eps", [1.0, 1e-3])
def test_free_streaming_uniform_state(eps):
    nx, ny, nv = 6, 5, 8
    g = ap2d.Grid2D(nx, ny)
    mu, eta, om = circle_pairs(nv)
    P = mu.size
    rng = np.random.default_rng(3)
    fp, fm = rng.uniform(0.1, 1.0, P), rng.uniform(0.1, 1.0, P)   # I(+Omega_p), I(-Omega_p)
    E = np.broadcast_to((fp + fm) / 2, (ny, nx, P)).copy()
    Oc = (fp - fm) / (2 * eps)
    Ox = np.broadcast_to(Oc, (ny, nx + 1, P)).copy()
    Oy = np.broadcast_to(Oc, (ny + 1, nx, P)).copy()
    # entering direction per edge: x = 0: sign(mu); x = L: -sign(mu); y = 0: +; y = L: -
    ent = lambda s: np.where(s > 0, fp, fm)
    b = np.stack([ent(mu), ent(-mu), ent(eta), ent(-eta)])
    T = rng.uniform(0.2, 1.0, (ny, nx))
    sig = np.zeros((ny, nx))
    ph = Physics(eps=eps, dt=0.1, m=0)
    r = ap2d.ap_step(g, E, Ox, Oy, T, sig, mu, eta, om, b, ph)
    assert np.array_equal(r["T"], T)
    np.testing.assert_allclose(r["E"], E, rtol=1e-14, atol=0)
    np.testing.assert_allclose(r["Ox"], Ox, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(r["Oy"], Oy, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(r["E_star"], E, rtol=1e-14, atol=0)


def _exact(x, y, t, mu, eta, w):
    """I0(x, y) = exp(-(x - 1/2)^2 / w^2) (1 + cos(2 pi y) / 2), transported."""
    I0 = lambda X, Y: np.exp(-((X - 0.5) / w) ** 2) * (1 + 0.5 * np.cos(2 * np.pi * Y))
    X, Y = x[None, :, None], y[:, None, None]
    fwd = I0(X - mu * t, Y - eta * t)
    bwd = I0(X + mu * t, Y + eta * t)
    return fwd, bwd


def _free_stream_error(n, nv=8, w=0.1, t_end=0.125):
    g = ap2d.Grid2D(n, n, periodic_y=True)
    mu, eta, om = circle_pairs(nv)
    P = mu.size
    h = 1.0 / n
    xc = (np.arange(n) + 0.5) * h
    xf = np.arange(n + 1) * h
    dt = h / 4
    steps = int(round(t_end / dt))
    fwd, bwd = _exact(xc, xc, 0.0, mu, eta, w)
    E = (fwd + bwd) / 2
    # O at the faces from the exact initial data (it is zero: isotropic I0)
    Ox = np.zeros((n, n + 1, P)); Oy = np.zeros((n + 1, n, P))
    T = np.full((n, n), 0.5)
    sig = np.zeros((n, n))
    ph = Physics(eps=1.0, dt=dt, m=0)
    b = np.zeros((4, P))
    for _ in range(steps):
        r = ap2d.ap_step(g, E, Ox, Oy, T, sig, mu, eta, om, b, ph)
        E, Ox, Oy = r["E"], r["Ox"], r["Oy"]
    fwd, bwd = _exact(xc, xc, steps * dt, mu, eta, w)
    return np.sum(np.abs(E - (fwd + bwd) / 2) @ om) * h * h


def test_free_streaming_converges_first_order():
    e = [_free_stream_error(n) for n in (8, 16, 32)]
    assert e[0] / e[1] > 1.5 and e[1] / e[2] > 1.6, e
    assert e[2] < 0.02, e


@pytest.mark.parametrize("m", [0, 3])
@pytest.mark.parametrize("eps", [1.0, 1e-2])
def test_conservation_identity(m, eps):
    nx, ny, nv = 6, 5, 8
    g = ap2d.Grid2D(nx, ny, Lx=1.0, Ly=0.7)
    mu, eta, om = circle_pairs(nv)
    P = mu.size
    rng = np.random.default_rng(21)
    E, Ox, Oy, T = _state(g, P, rng)
    sig = rng.uniform(0.5, 2.0, (ny, nx))
    b = rng.uniform(0, 1, (4, P))
    ph = Physics(a=1.0, c=1.0, Cv=1.2, eps=eps, dt=0.04, m=m)
    r = ap2d.ap_step(g, E, Ox, Oy, T, sig, mu, eta, om, b, ph)
    c, Cv, dt = ph.c, ph.Cv, ph.dt
    dx, dy = g.Lx / nx, g.Ly / ny
    Dv = lambda X, Y: (((X[:, 1:] - X[:, :-1]) * mu) @ om / dx + ((Y[1:] - Y[:-1]) * eta) @ om / dy)
    Ds, D1 = Dv(r["Ox_star"], r["Oy_star"]), Dv(r["Ox"], r["Oy"])
    np.testing.assert_allclose(r["D"], Ds, rtol=1e-12, atol=1e-12)
    rho_n, rho1 = E @ om, r["E"] @ om
    dT = r["T"] - T
    lhs = (rho1 - rho_n) / (c * dt) + Cv * dT / dt + Ds
    Ks = r["K_star"]
    K1 = np.ones_like(dT) if m == 0 else r["T"] ** m
    rhs = (eps ** 2 * K1 * (Ds - D1) + Cv * dT / dt * eps ** 2 * (K1 - Ks)) / (eps ** 2 * K1 + c * sig * dt)
    scale = np.abs(rho1 / (c * dt)) + np.abs(rho_n / (c * dt)) + np.abs(Cv * dT / dt) + np.abs(Ds) + np.abs(D1)
    assert np.max(np.abs(lhs - rhs) / scale) < 1e-12
    # the divergence telescopes into the outflow through the four edges
    out = ap2d.boundary_outflow(g, r["Ox_star"], r["Oy_star"], mu, eta, om)
    assert abs(np.sum(Ds) * dx * dy - out) < 1e-12 * (np.sum(np.abs(Ds)) * dx * dy)


def test_temperature_is_the_root_of_4_13():
    nx, ny, nv = 5, 5, 8
    g = ap2d.Grid2D(nx, ny)
    mu, eta, om = circle_pairs(nv)
    P = mu.size
    rng = np.random.default_rng(8)
    E, Ox, Oy, T = _state(g, P, rng)
    sig = rng.uniform(0.5, 2.0, (ny, nx))
    b = rng.uniform(0, 1, (4, P))
    ph = Physics(eps=1e-2, dt=0.05, m=3)
    r = ap2d.ap_step(g, E, Ox, Oy, T, sig, mu, eta, om, b, ph)
    Tb, _ = bisect_temperature(T.ravel(), r["rho_n"].ravel(), r["D"].ravel(), r["K_star"].ravel(),
                               sig.ravel(), ph)
    np.testing.assert_allclose(r["T"].ravel(), np.asarray(Tb, dtype=np.float64), rtol=4e-16 * 4, atol=0)


@pytest.mark.parametrize("m", [0, 3])
def test_eps_to_zero_reaches_2d_diffusion_limit(m):
    """A compact bump (IC (6.3)'s shape in 2-D), sigma = 1, zero inflow, dt = 0.1 dx:
    as eps -> 0 the 2-D AP step tends to the three-stage scheme (2.7)/(2.9) with
    the 2-D diffusion coefficient ac K <mu^2>/sigma, <mu^2> = 1/2 -- the dimension
    factor D_d = 2 of the limit -- at the rate eps^2, as the 1-D step does."""
    from oracle.diffusion2d import three_stage_step
    n, nv = 14, 8
    g = ap2d.Grid2D(n, n)
    mu, eta, om = circle_pairs(nv)
    P = mu.size
    xc = (np.arange(n) + 0.5) / n
    T0 = np.maximum(1 - 40 * ((xc[None, :] - 0.5) ** 2 + (xc[:, None] - 0.5) ** 2), 0.0)
    b = np.zeros((4, P))
    diffs, wrong = [], []
    for eps in (1e-2, 1e-3, 1e-4):
        ph = Physics(eps=eps, dt=0.1 / n, m=m)
        T = T0.copy()
        E = np.repeat((T ** 4)[:, :, None], P, 2)
        Ox, Oy = np.zeros((n, n + 1, P)), np.zeros((n + 1, n, P))
        Td, Tw = T0.copy(), T0.copy()
        for _ in range(6):
            r = ap2d.ap_step(g, E, Ox, Oy, T, np.ones((n, n)), mu, eta, om, b, ph)
            E, Ox, Oy, T = r["E"], r["Ox"], r["Oy"], r["T"]
            Td, _ = three_stage_step(Td, np.ones((n, n)), ph.dt, m=m, mu2=0.5)
            Tw, _ = three_stage_step(Tw, np.ones((n, n)), ph.dt, m=m, mu2=1.0 / 3.0)
        diffs.append(np.max(np.abs(T - Td)))
        wrong.append(np.max(np.abs(T - Tw)))
    assert diffs[2] < 1e-5, diffs
    assert diffs[0] / diffs[1] > 50 and diffs[1] / diffs[2] > 50, diffs
    # the 1-D coefficient (<mu^2> = 1/3) is a different limit
    assert min(wrong) > 100 * diffs[2], (wrong, diffs)
