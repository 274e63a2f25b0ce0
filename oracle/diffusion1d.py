"""Solvers of the nonlinear diffusion limit (test infrastructure).

The AP step must reduce, as eps -> 0, to a discretisation of
    a d_t T^4 + Cv d_t T = d_x( ac K / (3 sigma) d_x T^4 ),   K = T^m,
(1.3) for m = 0 and (1.5) for sigma_T = sigma/T^3 (m = 3).  This module holds

  three_stage_step  the prediction-correction-projection scheme (2.7) and its
                    sigma/T^3 form (2.9) (fully discrete version after (2.9));
  two_stage_step    the counter-example (2.8) (prediction + projection only);
  implicit_step     the fully implicit reference solvers (6.1) (q = 4) and
                    (6.7) (q = 7), solved by a global Newton iteration;
  semi_cor_step     the diffusion limit of the alternative correction (3.14)
                    that the remark closing Section 3 gives: the prediction of
                    (2.7)/(2.9), then the linear update
                      a (U* - U^n)/dt + Cv (T - T^n)/dt = div(F^n grad U*)
                    (no nonlinear solve; the paper reports that it fails for a
                    T-dependent sigma and is not energy-conservative).

All live on the AP step's cell-centred grid (cells j = 0..N-1 on [0, L],
interior faces i = 1..N-1 between cells i-1 and i).  A face coefficient at an
interior face uses sigma_i = harmonic mean of the two cell values (the
arithmetic mean of 1/sigma used in (6.7)) and, for m = 3, K_i = mean of the two
cell values of T^3 (as after (5.2)).  Boundaries are either closed (zero flux,
"neumann") or held by ghost cells one cell outside the slab ("dirichlet").

`a_time` replaces a in the time-derivative terms only (the flux keeps ac);
with a_time = 0 both limits become porous-medium equations
T_t = D (T^q)_xx whose Barenblatt solutions pin these solvers.

Reading: the discrete correction of the AP scheme takes its flux from the
prediction (O* is computed with K^n), so its eps -> 0 limit has K^n in both
fluxes.  The printed (2.9) writes (T^{n+1*})^3 in the correction flux; both
variants are available through `corr_K` ("old" = K^n, "predicted" =
(U*)^(3/4)).
"""
import numpy as np
from scipy.linalg import solve_banded


def face_sigma(sigma0):
    """Harmonic mean of sigma at the N-1 interior faces."""
    sl, sr = sigma0[:-1], sigma0[1:]
    return 2.0 * sl * sr / (sl + sr)


def _face_coeff(T_or_K, sigma0, m, a, c, from_K=False):
    """ac K_i / (3 sigma_i) at interior faces (the D_d = 3 flux of (2.7))."""
    K = T_or_K if from_K else (np.ones_like(T_or_K) if m == 0 else T_or_K ** m)
    Kf = 0.5 * (K[:-1] + K[1:])
    return a * c * Kf / (3.0 * face_sigma(sigma0))


def _div_flux(Fint, U, dx, bc, ghost, Fb):
    """(1/dx)[F_{j+1}(U_{j+1}-U_j)/dx - F_j(U_j-U_{j-1})/dx] for every cell."""
    N = U.size
    flux = np.zeros(N + 1)                      # flux through node i, +x direction
    flux[1:N] = Fint * (U[1:] - U[:-1]) / dx
    if bc == "dirichlet":
        flux[0] = Fb[0] * (U[0] - ghost[0]) / dx
        flux[N] = Fb[1] * (ghost[1] - U[N - 1]) / dx
    return (flux[1:] - flux[:-1]) / dx


def _diffusion_matrix(Fint, N, dx, bc, Fb):
    """Banded form of -(1/dx^2) div F grad (without ghost right-hand side)."""
    lo = np.zeros(N)
    up = np.zeros(N)
    di = np.zeros(N)
    w = Fint / dx ** 2
    di[:-1] += w
    di[1:] += w
    up[:-1] = -w
    lo[1:] = -w
    if bc == "dirichlet":
        di[0] += Fb[0] / dx ** 2
        di[-1] += Fb[1] / dx ** 2
    return lo, di, up


def _solve_tri(lo, di, up, rhs):
    N = di.size
    ab = np.zeros((3, N))
    ab[0, 1:] = up[:-1]
    ab[1] = di
    ab[2, :-1] = lo[1:]
    return solve_banded((1, 1), ab, rhs)


def _bc_data(bc, ghost_T, sigma0, K_cells, a, c):
    if bc == "dirichlet":
        ghost_U = np.asarray(ghost_T, dtype=np.float64) ** 4
        Fb = (a * c * K_cells[0] / (3.0 * sigma0[0]),
              a * c * K_cells[-1] / (3.0 * sigma0[-1]))
        return ghost_U, Fb
    return np.zeros(2), (0.0, 0.0)


def three_stage_step(T, sigma0, dt, L=1.0, a=1.0, c=1.0, Cv=1.0, m=0,
                     a_time=None, bc="neumann", ghost_T=(0.0, 0.0),
                     corr_K="old", maxit=200):
    """One step of (2.7) (m = 0) or of the fully discrete form of (2.9) (m = 3).

    Stage 1 (prediction, linear):
      (U* - U^n)/dt = 4 T^3/(4 a T^3 + Cv) * div(F^n grad U*)
    Stage 2 (correction, one scalar equation per cell):
      a (T^4 - U^n)/dt + Cv (T - T^n)/dt = div(F^c grad U*)
    Stage 3 (projection): U^{n+1} = (T^{n+1})^4.
    Returns (T^{n+1}, U*).
    """
    T = np.asarray(T, dtype=np.float64)
    sigma0 = np.asarray(sigma0, dtype=np.float64)
    at = a if a_time is None else a_time
    N = T.size
    dx = L / N
    U = T ** 4
    Kn = np.ones(N) if m == 0 else T ** m
    Fint = _face_coeff(Kn, sigma0, m, a, c, from_K=True)
    ghost_U, Fb = _bc_data(bc, ghost_T, sigma0, Kn, a, c)
    # stage 1
    pref = 4.0 * T ** 3 / (4.0 * at * T ** 3 + Cv)
    lo, di, up = _diffusion_matrix(Fint, N, dx, bc, Fb)
    rhs = U.copy()
    if bc == "dirichlet":
        rhs[0] += dt * pref[0] * Fb[0] * ghost_U[0] / dx ** 2
        rhs[-1] += dt * pref[-1] * Fb[1] * ghost_U[1] / dx ** 2
    Us = _solve_tri(dt * pref * lo, 1.0 + dt * pref * di, dt * pref * up, rhs)
    # stage 2
    if m == 0 or corr_K == "old":
        Fc, Fbc = Fint, Fb
    else:
        Ks = np.maximum(Us, 0.0) ** 0.75
        Fc = _face_coeff(Ks, sigma0, m, a, c, from_K=True)
        _, Fbc = _bc_data(bc, ghost_T, sigma0, Ks, a, c)
    rhs_T = dt * _div_flux(Fc, Us, dx, bc, ghost_U, Fbc) + at * U + Cv * T
    Tn1 = _scalar_quartic(at, Cv, rhs_T, T, maxit)
    return Tn1, Us


def semi_cor_step(T, sigma0, dt, L=1.0, a=1.0, c=1.0, Cv=1.0, m=0, a_time=None, bc="neumann",
                  ghost_T=(0.0, 0.0)):
    """One step of the diffusion limit of (3.14): stage 1 of (2.7)/(2.9), then
        T^{n+1} = T^n + [dt div(F^n grad U*) - a (U* - U^n)] / Cv,
    the limit equation printed in the remark after (3.13).  Returns (T^{n+1}, U*)."""
    T = np.asarray(T, dtype=np.float64)
    sigma0 = np.asarray(sigma0, dtype=np.float64)
    at = a if a_time is None else a_time
    N = T.size
    dx = L / N
    U = T ** 4
    Kn = np.ones(N) if m == 0 else T ** m
    Fint = _face_coeff(Kn, sigma0, m, a, c, from_K=True)
    ghost_U, Fb = _bc_data(bc, ghost_T, sigma0, Kn, a, c)
    pref = 4.0 * T ** 3 / (4.0 * at * T ** 3 + Cv)
    lo, di, up = _diffusion_matrix(Fint, N, dx, bc, Fb)
    rhs = U.copy()
    if bc == "dirichlet":
        rhs[0] += dt * pref[0] * Fb[0] * ghost_U[0] / dx ** 2
        rhs[-1] += dt * pref[-1] * Fb[1] * ghost_U[1] / dx ** 2
    Us = _solve_tri(dt * pref * lo, 1.0 + dt * pref * di, dt * pref * up, rhs)
    Tn1 = T + (dt * _div_flux(Fint, Us, dx, bc, ghost_U, Fb) - at * (Us - U)) / Cv
    return Tn1, Us


def _scalar_quartic(at, Cv, rhs, T0, maxit):
    """Solve at*T^4 + Cv*T = rhs per cell (Newton from T0, monotone)."""
    if at == 0:
        return rhs / Cv
    T = np.maximum(T0.copy(), 0.0)
    # start from above the root so that Newton on the convex function is monotone
    T = np.maximum(T, np.maximum(rhs / Cv, 0.0) ** 1.0)
    T = np.maximum(T, (np.maximum(rhs, 0.0) / at) ** 0.25)
    for _ in range(maxit):
        f = at * T ** 4 + Cv * T - rhs
        df = 4.0 * at * T ** 3 + Cv
        step = f / df
        T -= step
        if np.all(np.abs(step) <= 1e-15 * np.maximum(np.abs(T), 1e-300)):
            break
    return T


def two_stage_step(T, sigma0, dt, L=1.0, a=1.0, c=1.0, Cv=1.0, m=0,
                   bc="neumann", ghost_T=(0.0, 0.0)):
    """(2.8): prediction for U^{n+1} then T^{n+1} = (U^{n+1})^(1/4)."""
    T = np.asarray(T, dtype=np.float64)
    N = T.size
    dx = L / N
    U = T ** 4
    Kn = np.ones(N) if m == 0 else T ** m
    Fint = _face_coeff(Kn, sigma0, m, a, c, from_K=True)
    ghost_U, Fb = _bc_data(bc, ghost_T, sigma0, Kn, a, c)
    pref = 4.0 * T ** 3 / (4.0 * a * T ** 3 + Cv)
    lo, di, up = _diffusion_matrix(Fint, N, dx, bc, Fb)
    rhs = U.copy()
    if bc == "dirichlet":
        rhs[0] += dt * pref[0] * Fb[0] * ghost_U[0] / dx ** 2
        rhs[-1] += dt * pref[-1] * Fb[1] * ghost_U[1] / dx ** 2
    Un1 = _solve_tri(dt * pref * lo, 1.0 + dt * pref * di, dt * pref * up, rhs)
    return np.maximum(Un1, 0.0) ** 0.25


def implicit_step(T, sigma_face, dt, L=1.0, a=1.0, c=1.0, Cv=1.0, q=4,
                  a_time=None, bc="neumann", ghost_T=(0.0, 0.0),
                  sigma_bnd=(1.0, 1.0), tol=1e-13, maxit=100):
    """One step of the fully implicit solver (6.1) (q = 4) or (6.7) (q = 7).

      a_t (T^4 - T_n^4)/dt + Cv (T - T_n)/dt
        = kappa/dx^2 [ (T_{j+1}^q - T_j^q)/sigma_{j+1/2}
                       - (T_j^q - T_{j-1}^q)/sigma_{j-1/2} ],
    kappa = ac/3 for q = 4 (6.1), kappa = 4ac/21 for q = 7 ((6.7) times a).
    T^{n+1} is used in every flux term (in (6.1) one T^n is a misprint).
    `sigma_face` holds sigma at the N-1 interior faces; `sigma_bnd` the
    boundary-face values used with Dirichlet ghosts.  Global Newton with a
    tridiagonal Jacobian.
    """
    Tn = np.asarray(T, dtype=np.float64)
    at = a if a_time is None else a_time
    N = Tn.size
    dx = L / N
    kappa = a * c / 3.0 if q == 4 else 4.0 * a * c / 21.0
    w = kappa / (np.asarray(sigma_face, dtype=np.float64) * dx ** 2)
    wb = (kappa / (sigma_bnd[0] * dx ** 2), kappa / (sigma_bnd[1] * dx ** 2))
    gq = np.asarray(ghost_T, dtype=np.float64) ** q
    Tk = Tn.copy()
    for _ in range(maxit):
        V = Tk ** q
        dV = q * Tk ** (q - 1)
        div = np.zeros(N)
        div[:-1] += w * (V[1:] - V[:-1])
        div[1:] -= w * (V[1:] - V[:-1])
        if bc == "dirichlet":
            div[0] -= wb[0] * (V[0] - gq[0])
            div[-1] += wb[1] * (gq[1] - V[-1])
        F = at * (Tk ** 4 - Tn ** 4) + Cv * (Tk - Tn) - dt * div
        di = 4.0 * at * Tk ** 3 + Cv
        di[:-1] += dt * w * dV[:-1]
        di[1:] += dt * w * dV[1:]
        if bc == "dirichlet":
            di[0] += dt * wb[0] * dV[0]
            di[-1] += dt * wb[1] * dV[-1]
        up = np.zeros(N)
        lo = np.zeros(N)
        up[:-1] = -dt * w * dV[1:]
        lo[1:] = -dt * w * dV[:-1]
        step = _solve_tri(lo, di, up, F)
        Tk = Tk - step
        if np.max(np.abs(step)) <= tol * max(np.max(np.abs(Tk)), 1e-300):
            break
    return Tk


def barenblatt(x, t, q, D, C, x0=0.5):
    """Barenblatt solution of T_t = D (T^q)_xx in 1-D:
    T = tau^(-1/(q+1)) (C - k (x-x0)^2 tau^(-2/(q+1)))_+^(1/(q-1)),
    tau = D t, k = (q-1)/(2q(q+1))."""
    tau = D * t
    al = 1.0 / (q + 1.0)
    k = (q - 1.0) / (2.0 * q * (q + 1.0))
    inner = C - k * (x - x0) ** 2 * tau ** (-2.0 * al)
    return tau ** (-al) * np.maximum(inner, 0.0) ** (1.0 / (q - 1.0))
