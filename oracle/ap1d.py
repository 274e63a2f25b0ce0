"""One fully discrete AP step for the 1-D gray radiative transfer equation.

Test infrastructure only (see the package docstring).  Each stage is written
as the equations of the paper, in its order and notation, so that a reader
can check it against the paper by eye.  Arithmetic is carried out in 80-bit
extended precision and the linear systems are solved to full accuracy (see
linsolve); results are returned in binary64.

Algorithm 2 (Section 4; Section 5 for sigma_T = sigma / T^3):
  Prediction      (4.5a-c) with the inflow relations (4.6)/(4.7); for
                  sigma/T^3 the K-multiplied form (5.2), K = T^3.
  Correction 1    the scalar equation (4.13) per cell (for sigma/T^3 the sum
                  of (5.4)-(5.5)), solved by Newton from T^n.
  Correction 2    per-direction linear system (4.11a,b) with (4.12), U* and K*
                  replaced by (T^{n+1})^4 and (T^{n+1})^m, inflow relations as
                  stated after (4.13).
  Projection      (4.14): U = T^4, O = O_J, E = acU + eps E_J.

Index conventions (0-based).  Cells j = 0..N-1 are the paper's i+1/2
(x_{j+1/2} = (j+1/2) dx on [0, L]); nodes i = 0..N are the paper's x_{i+1};
node i separates cell i-1 (left) from cell i (right).  Parity arrays are
cell-major: E[j, p], O[i, p], p the parity pair (mu_p > 0).

Readings of points the paper leaves open:
  * sigma at an interior node: harmonic mean of the two adjacent cell values
    (the arithmetic mean of 1/sigma, the face rule of (6.7));
  * K at an interior node: arithmetic mean of the adjacent cell values, as
    stated after (5.2); K = 1 when sigma does not depend on T (m = 0);
  * K* = max(U*, 0)^(3/4) (clamped so a negative U* cannot give NaN);
  * the right-boundary relation of the projection uses the sign of (4.7)
    (the printed projection relation swaps b_R and E, contradicting (4.6));
  * (4.11b) holds in every cell 1 <= j <= N, the boundary cells closing
    through the inflow relations, as the text after (4.13) says;
  * sigma0 = 0 together with K* = 0 leaves (4.13) empty: T^{n+1} = T^n.
"""
from dataclasses import dataclass

import numpy as np

from .linsolve import XP, coo, solve_refined


@dataclass
class Physics:
    """Constants of (1.1)/(1.4) and the discretisation parameters."""
    a: float = 1.0       # radiation constant
    c: float = 1.0       # speed of light
    Cv: float = 1.0      # heat capacity
    eps: float = 1e-2    # scaled mean free path
    dt: float = 5e-3     # time step
    L: float = 1.0       # slab length, x in [0, L]
    m: int = 0           # opacity law sigma_T = sigma0 * T^(-m), m in {0, 3}

    def ext(self):
        """The floating-point constants in extended precision."""
        return (XP(self.a), XP(self.c), XP(self.Cv), XP(self.eps),
                XP(self.dt), XP(self.L))


# --------------------------------------------------------------------------
# coefficients
# --------------------------------------------------------------------------
def node_sigma(sigma0):
    """sigma_i at the N-1 interior nodes: harmonic mean of the two cells."""
    sl, sr = sigma0[:-1], sigma0[1:]
    den = sl + sr
    out = np.zeros_like(den)
    nz = den > 0
    out[nz] = 2 * sl[nz] * sr[nz] / den[nz]
    return out


def cell_K(T, m):
    """K_{i+1/2} = (T_{i+1/2})^m (Section 5: K = T^3; K = 1 when m = 0)."""
    return np.ones_like(T) if m == 0 else T ** m


def node_K(Kc):
    """K_i = (K_{i+1/2} + K_{i-1/2}) / 2 at the interior nodes (after (5.2))."""
    return (Kc[:-1] + Kc[1:]) / 2


def moment(E, omega):
    """rho_j = int_0^1 E_j dv = sum_p omega_p E_{j,p}."""
    return E @ omega


def _index(N, P):
    """Unknown numbering: E[j, p] first (cell-major), then O[i, p]."""
    j = np.arange(N)[:, None]
    i = np.arange(N + 1)[:, None]
    p = np.arange(P)[None, :]
    iE = j * P + p                       # (N, P)
    iO = N * P + i * P + p               # (N+1, P)
    return iE, iO


# --------------------------------------------------------------------------
# Prediction: (4.5a)-(4.5c), inflow relations (4.6); sigma/T^3 form (5.2)
# --------------------------------------------------------------------------
def predict(E, O, T, sigma0, mu, omega, bL, bR, ph, T_K=None):
    """Solve the prediction system for E*, O*, U* (extended precision).

    Following the recipe after (4.5): U* is written in terms of E* with
    (4.5c), substituted into (4.5b), and (4.5a)+(4.5b)+(4.6) is solved as one
    linear system in (E*, O*).  Rows of (4.5a) and (4.5b) are multiplied by
    eps^2 c dt (a row scaling; the solution is unchanged).  `T_K` (default T)
    is the temperature that defines K = T^m of the sigma/T^3 form (5.2); U^n
    and beta always come from T.
    """
    N, P = E.shape
    a, c, Cv, eps, dt, L = ph.ext()
    m = ph.m
    dx = L / N
    U = T ** 4
    Kc = cell_K(T if T_K is None else T_K, m)
    Kn = node_K(Kc)
    sn = node_sigma(sigma0)
    # (4.5c): Cv (U* - U^n)/dt = 4 sigma0 (T^n)^(3-m) (rho* - ac U*) / eps^2
    #   =>  U* = (U^n + beta rho*) / (1 + ac beta)
    beta = 4 * sigma0 * dt * T ** (3 - m) / (eps ** 2 * Cv)

    iE, iO = _index(N, P)
    n = N * P + (N + 1) * P
    rows, cols, vals = [], [], []
    rhs = np.zeros(n, dtype=XP)
    v = mu[None, :]

    # (4.5a), interior nodes i = 1..N-1:
    #   K_i [ (O_i - O^n_i)/(c dt) + v (E_i - E_{i-1})/(eps^2 dx) ] = -sigma_i O_i / eps^2
    r = iO[1:N]
    Ki, si = Kn[:, None], sn[:, None]
    rows += [r, r, r]
    cols += [iO[1:N], iE[1:N], iE[0:N - 1]]
    vals += [np.broadcast_to(Ki * eps ** 2 + si * c * dt, r.shape),
             Ki * v * c * dt / dx, -Ki * v * c * dt / dx]
    rhs[r.ravel()] = (Ki * eps ** 2 * O[1:N]).ravel()

    # (4.6) at x = 0:  E_{3/2} + (eps/2)(O_2 + O_1) = b_L(v)
    r = iO[0]
    rows += [r, r, r]
    cols += [iE[0], iO[0], iO[1]]
    one = np.ones(P, dtype=XP)
    vals += [one, one * eps / 2, one * eps / 2]
    rhs[r] = bL
    # (4.6) at x = L:  E_{N+1/2} - (eps/2)(O_N + O_{N+1}) = b_R(-v)
    r = iO[N]
    rows += [r, r, r]
    cols += [iE[N - 1], iO[N - 1], iO[N]]
    vals += [one, -one * eps / 2, -one * eps / 2]
    rhs[r] = bR

    # (4.5b) with (4.5c) substituted, cells j = 0..N-1:
    #   K_j [ (E_j - E^n_j)/(c dt) + v (O_{j+1} - O_j)/dx ]
    #     = sigma0_j/eps^2 [ ac (U^n_j + beta_j sum_q omega_q E_{j,q})/(1 + ac beta_j) - E_j ]
    r = iE
    Kj, s0 = Kc[:, None], sigma0[:, None]
    bj = beta[:, None]
    g = s0 * c * dt * a * c * bj / (1 + a * c * bj)                  # (N, 1)
    rows += [r, r, r]
    cols += [iE, iO[1:N + 1], iO[0:N]]
    vals += [np.broadcast_to(Kj * eps ** 2 + s0 * c * dt, r.shape),
             Kj * eps ** 2 * v * c * dt / dx, -Kj * eps ** 2 * v * c * dt / dx]
    # the angular coupling -g_j omega_q E_{j,q} in row (j, p), for every q
    rr = np.broadcast_to(iE[:, :, None], (N, P, P))
    cc = np.broadcast_to(iE[:, None, :], (N, P, P))
    rows.append(rr)
    cols.append(cc)
    vals.append(np.broadcast_to(-g[:, :, None] * omega[None, None, :], (N, P, P)))
    rhs[r.ravel()] = (Kj * eps ** 2 * E
                      + s0 * c * dt * a * c * U[:, None] / (1 + a * c * bj)).ravel()

    A = coo(rows, cols, vals, n)

    x, _, _ = solve_refined(A, rhs)
    Es = x[:N * P].reshape(N, P)
    Os = x[N * P:].reshape(N + 1, P)
    rho_s = moment(Es, omega)
    Us = (U + beta * rho_s) / (1 + a * c * beta)
    return Es, Os, Us


# --------------------------------------------------------------------------
# Correction substep 1: the scalar equation (4.13) / its sigma/T^3 form
# --------------------------------------------------------------------------
def flux_divergence(O, mu, omega, dx):
    """D_{i+1/2} = int_0^1 v (O_{i+1} - O_i)/dx dv (right side of (4.13))."""
    return ((O[1:, :] - O[:-1, :]) * mu) @ omega / dx


def temperature_equation(T, Tn, rho_n, D, Kstar, sigma0, ph):
    """(4.13) times c sigma0 dt^2, written as G(T) = 0, and G'(T).

    (4.13): [ac T^4 + eps^2 K* Cv (T - T^n)/(sigma0 dt)]/(c dt)
            + Cv (T - T^n)/dt = rho^n/(c dt) - D,
    with K* = 1 for m = 0 and K* = (U*)^(3/4) for sigma/T^3 ((5.4)+(5.5)).
    """
    a, c, Cv, eps, dt, _ = ph.ext()
    lin = Cv * (eps ** 2 * Kstar + c * sigma0 * dt)
    G = (a * c * sigma0 * dt * T ** 4 + lin * (T - Tn)
         - sigma0 * dt * (rho_n - c * dt * D))
    dG = 4 * a * c * sigma0 * dt * T ** 3 + lin
    return G, dG


def newton_temperature(Tn, rho_n, D, Kstar, sigma0, ph, maxit=200):
    """Scalar Newton per cell from T^n (the remark after (2.7)).

    Returns (T, iterations, converged mask).  G is convex with G' > 0 for
    T >= 0, so Newton from T^n >= 0 converges to the unique root.
    """
    N = Tn.size
    T = np.array(Tn, dtype=XP)
    its = np.zeros(N, dtype=np.int64)
    done = (sigma0 == 0) & (Kstar == 0)
    for _ in range(maxit):
        act = ~done
        if not act.any():
            break
        G, dG = temperature_equation(T, Tn, rho_n, D, Kstar, sigma0, ph)
        step = np.zeros(N, dtype=XP)
        step[act] = G[act] / dG[act]
        T[act] -= step[act]
        its[act] += 1
        done = done | (act & (np.abs(step) <= XP(2.0) ** -56 * np.maximum(np.abs(T), np.abs(Tn))))
    return T, its, done


def bisect_temperature(Tn, rho_n, D, Kstar, sigma0, ph, iters=300):
    """Independent root of G on [0, s] by bisection (used by the pins).

    s = T^n + sigma0 dt (rho^n - c dt D) / (Cv (eps^2 K* + c sigma0 dt)) is
    where the linear part alone would put T; G(0) <= 0 <= G(s) when s >= 0.
    """
    a, c, Cv, eps, dt, _ = ph.ext()
    lin = Cv * (eps ** 2 * Kstar + c * sigma0 * dt)
    s = Tn + sigma0 * dt * (rho_n - c * dt * D) / lin
    lo = np.zeros_like(s)
    hi = np.maximum(s, 0)
    for _ in range(iters):
        mid = (lo + hi) / 2
        G, _ = temperature_equation(mid, Tn, rho_n, D, Kstar, sigma0, ph)
        pos = G > 0
        hi = np.where(pos, mid, hi)
        lo = np.where(pos, lo, mid)
    return (lo + hi) / 2, s


# --------------------------------------------------------------------------
# Correction substep 2: (4.11a,b) + (4.12) with U* -> (T^{n+1})^4
# --------------------------------------------------------------------------
def correct_J(E, O, Tnew, sigma0, mu, bL, bR, ph):
    """Solve the per-direction systems for E_J (cells) and O_J (nodes).

    Rows of (4.11a) are multiplied by eps^2 c dt, rows of (4.11b) by
    eps c dt.  For sigma/T^3 every row carries K^{n+1} = (T^{n+1})^3 (5.3).
    """
    N, P = E.shape
    a, c, Cv, eps, dt, L = ph.ext()
    dx = L / N
    U = Tnew ** 4
    Kc = cell_K(Tnew, ph.m)
    Kn = node_K(Kc)
    sn = node_sigma(sigma0)
    iE, iO = _index(N, P)
    n = N * P + (N + 1) * P
    rows, cols, vals = [], [], []
    rhs = np.zeros(n, dtype=XP)
    v = mu[None, :]

    # (4.11a), interior nodes:
    #   K_i [ (O_J,i - O^n_i)/(c dt) + ac v (U_i - U_{i-1})/(eps^2 dx)
    #         + v (E_J,i - E_J,i-1)/(eps dx) ] = -sigma_i O_J,i / eps^2
    r = iO[1:N]
    Ki, si = Kn[:, None], sn[:, None]
    dU = (U[1:N] - U[0:N - 1])[:, None]
    rows += [r, r, r]
    cols += [iO[1:N], iE[1:N], iE[0:N - 1]]
    vals += [np.broadcast_to(Ki * eps ** 2 + si * c * dt, r.shape),
             Ki * eps * v * c * dt / dx, -Ki * eps * v * c * dt / dx]
    rhs[r.ravel()] = (Ki * eps ** 2 * O[1:N] - Ki * a * c * v * c * dt / dx * dU).ravel()

    # inflow relations with E = ac U + eps E_J (text after (4.13))
    one = np.ones(P, dtype=XP)
    r = iO[0]
    rows += [r, r, r]
    cols += [iE[0], iO[0], iO[1]]
    vals += [one * eps, one * eps / 2, one * eps / 2]
    rhs[r] = bL - a * c * U[0]
    r = iO[N]
    rows += [r, r, r]
    cols += [iE[N - 1], iO[N - 1], iO[N]]
    vals += [one * eps, -one * eps / 2, -one * eps / 2]
    rhs[r] = bR - a * c * U[N - 1]

    # (4.11b) with (4.12), cells j = 0..N-1:
    #   K_j [ (ac U_j + eps E_J,j - E^n_j)/(c dt) + v (O_J,j+1 - O_J,j)/dx ]
    #     = -sigma0_j E_J,j / eps
    r = iE
    Kj, s0 = Kc[:, None], sigma0[:, None]
    rows += [r, r, r]
    cols += [iE, iO[1:N + 1], iO[0:N]]
    vals += [np.broadcast_to(Kj * eps ** 2 + s0 * c * dt, r.shape),
             Kj * eps * v * c * dt / dx, -Kj * eps * v * c * dt / dx]
    rhs[r.ravel()] = (Kj * eps * (E - a * c * U[:, None])).ravel()

    A = coo(rows, cols, vals, n)
    x, _, _ = solve_refined(A, rhs)
    EJ = x[:N * P].reshape(N, P)
    OJ = x[N * P:].reshape(N + 1, P)
    return EJ, OJ


# --------------------------------------------------------------------------
# Algorithm 2
# --------------------------------------------------------------------------
def ap_step(E, O, T, sigma0, mu, omega, bL, bR, ph, newton_maxit=200):
    """Advance (E, O, T) by one time step.  Returns a dict of every stage
    (binary64 arrays)."""
    E = np.asarray(E, dtype=np.float64)
    O = np.asarray(O, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    sigma0 = np.asarray(sigma0, dtype=np.float64)
    N, P = E.shape
    if N < 2:
        raise ValueError("the staggered grid needs at least two cells")
    if O.shape != (N + 1, P) or T.shape != (N,) or sigma0.shape != (N,):
        raise ValueError("shape mismatch")
    if ph.m not in (0, 3):
        raise ValueError("opacity law exponent must be 0 or 3")
    # extended-precision copies of every input
    Ex, Ox, Tx, sx = (np.asarray(x, dtype=XP) for x in (E, O, T, sigma0))
    mux, omx = np.asarray(mu, dtype=XP), np.asarray(omega, dtype=XP)
    bLx, bRx = np.asarray(bL, dtype=XP), np.asarray(bR, dtype=XP)
    dx = XP(ph.L) / N

    # Prediction
    Es, Os, Us = predict(Ex, Ox, Tx, sx, mux, omx, bLx, bRx, ph)

    # Correction, substep 1 (uses O*_J = O* from the prediction)
    rho_n = moment(Ex, omx)
    D = flux_divergence(Os, mux, omx, dx)
    Kstar = np.ones(N, dtype=XP) if ph.m == 0 else np.maximum(Us, 0) ** XP(0.75)
    Tnew, its, conv = newton_temperature(Tx, rho_n, D, Kstar, sx, ph,
                                         maxit=newton_maxit)
    Tnew = np.where((sx == 0) & (Kstar == 0), Tx, Tnew)

    # Correction, substep 2
    EJ, OJ = correct_J(Ex, Ox, Tnew, sx, mux, bLx, bRx, ph)

    # Projection (4.14)
    a, c, _, eps, _, _ = ph.ext()
    Unew = Tnew ** 4
    Enew = a * c * Unew[:, None] + eps * EJ
    Onew = OJ

    f64 = lambda x: np.asarray(x, dtype=np.float64)
    return dict(E=f64(Enew), O=f64(Onew), T=f64(Tnew), U=f64(Unew),
                E_star=f64(Es), O_star=f64(Os), U_star=f64(Us),
                rho_n=f64(rho_n), rho_star=f64(moment(Es, omx)), D=f64(D),
                K_star=f64(Kstar), E_J=f64(EJ), O_J=f64(OJ),
                rho=f64(moment(Enew, omx)),
                newton_its=its, newton_converged=conv)


def implicit_reference_step(E, O, T, sigma0, mu, omega, bL, bR, ph, tol=1e-14, maxit=500):
    """The iterative implicit reference solver of the paper's nonlinear-opacity
    examples, (6.6): backward Euler in I and U with the opacity sigma0/T^3
    evaluated at the previous iterate T^(k) = (U^(k))^(1/4), iterated from
    T^(0) = T^n until T stops changing (max |T^(k+1) - T^(k)| <= tol max T).
    On the parity grid one iteration is the prediction system (5.2) with K
    from T^(k) (U^n and the material coupling from T^n); at the fixed point
    E^{n+1} = E*, O^{n+1} = O*, U^{n+1} = U*.  Returns a dict with E, O, T, U,
    the iteration count and whether it converged."""
    E = np.asarray(E, dtype=np.float64)
    O = np.asarray(O, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    Ex, Ox, Tx, sx = (np.asarray(x, dtype=XP) for x in (E, O, T, np.asarray(sigma0, dtype=np.float64)))
    mux, omx = np.asarray(mu, dtype=XP), np.asarray(omega, dtype=XP)
    bLx, bRx = np.asarray(bL, dtype=XP), np.asarray(bR, dtype=XP)
    Tk = Tx.copy()
    conv = False
    for k in range(1, maxit + 1):
        Es, Os, Us = predict(Ex, Ox, Tx, sx, mux, omx, bLx, bRx, ph, T_K=Tk)
        Tn1 = np.maximum(Us, 0) ** XP(0.25)
        done = np.max(np.abs(Tn1 - Tk)) <= tol * np.max(np.abs(Tn1))
        Tk = Tn1
        if done:
            conv = True
            break
    f64 = lambda x: np.asarray(x, dtype=np.float64)
    return dict(E=f64(Es), O=f64(Os), T=f64(Tk), U=f64(Us), iterations=k, converged=conv)


def intensity(E, O, eps):
    """Cell-centre I(+mu_p), I(-mu_p) from the parities via (4.2):
    I(+-mu) = E +- eps * O, with O averaged from the two adjacent nodes
    (the same interpolation the inflow relations (4.6) use)."""
    Oc = 0.5 * (O[1:, :] + O[:-1, :])
    return E + eps * Oc, E - eps * Oc
