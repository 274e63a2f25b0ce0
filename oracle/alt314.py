"""The alternative correction of the remark closing Section 3, (3.14), fully
discrete on the parity grid.

Test infrastructure only: imported by tests/ (and nothing in the product
path); written from the remark's equations, sharing no code with the HIP
library.

The remark keeps the time derivative (1/c) d_t I of (1.1) as the prediction
stage's update (1/c)(I^{n+1*} - I^n)/dt, treats the emission with U^{n+1*},
and then needs no nonlinear solve: (3.14a) is a linear, direction-by-direction
problem for the remainder J^{n+1}, and (3.14b), Cv (T^{n+1} - T^n)/dt =
sigma rho_J^{n+1}, gives T^{n+1} explicitly.  Its printed diffusion limit is
  a (U* - U^n)/dt + Cv (T^{n+1} - T^n)/dt = div( ac/(3 sigma) grad U* ).

Reading (the printed (3.14a) mixes scalings): with
    I^{n+1} = ac U* - (eps/sigma) v.grad(ac U*) + eps^2 J^{n+1},
(1.1) with the time derivative from the prediction and the emission at U*,
    (1/c)(I* - I^n)/dt + (1/eps) v.grad I^{n+1} = (sigma/eps^2)(ac U* - I^{n+1}),
is term by term the printed (3.14a) (the (1/eps) v.grad(ac U*) parts of the
streaming and of the collision term cancel), and its v-average with
(1.1b) is (3.14b).  Written for Jh = (I^{n+1} - ac U*)/eps, the remainder of
the paper's expansion (3.6) taken about U* instead of T^4, it is exactly
    (1/c)(I* - I^n)/dt + (1/eps) v.grad(ac U* + eps Jh) = -(sigma/eps) Jh,
the correction equation of the scheme (the one after (3.10)) with U^{n+1}
replaced by U* and the time derivative by the prediction's.  Its even/odd
parts on the staggered grid are (4.11a,b) with those two replacements:
  nodes:  K_i [ (O*_i - O^n_i)/(c dt) + ac mu (U*_i - U*_{i-1})/(eps^2 dx)
                + mu (E_J,i - E_J,i-1)/(eps dx) ] = -sigma_i O_J,i / eps^2
  cells:  K_j [ (E*_j - E^n_j)/(c dt) + mu (O_J,j+1 - O_J,j)/dx ]
                = -sigma0_j E_J,j / eps
  inflow: (ac U*_1 + eps E_J,1) +- (eps/2)(O_J at the edge node and its
          neighbour) = b, as in (4.6)
with K = (T^n)^m (the prediction's; nothing at the new time level is known
when this stage runs), then
  (3.14b): T^{n+1}_j = T^n_j + dt sigma0_j / (eps K_j Cv) sum_p omega_p E_J,j,p
  projection (4.14): U^{n+1} = (T^{n+1})^4, E^{n+1} = ac U^{n+1} + eps E_J,
                     O^{n+1} = O_J.
Summing the cell rows over the directions gives, per cell and exactly,
  (rho* - rho^n)/(c dt) + Cv (T^{n+1} - T^n)/dt + D_J = 0,
D_J = sum_p omega_p mu_p (O_J,j+1 - O_J,j)/dx: the energy with rho* balances,
the state's energy (with rho^{n+1} = ac U^{n+1} + eps rho_J) does not -- the
remark's "not energy conservative".
"""
import numpy as np

from .ap1d import _index, cell_K, moment, node_K, node_sigma, predict
from .linsolve import XP, coo, solve_refined


def correct_alt(E, O, T, Es, Os, Us, sigma0, mu, bL, bR, ph):
    """E_J (cells), O_J (nodes) of (3.14a) in the parity form above (extended
    precision).  Node rows are multiplied by eps^2 c dt, cell rows by eps c dt."""
    N, P = E.shape
    a, c, Cv, eps, dt, L = ph.ext()
    dx = L / N
    Kc = cell_K(T, ph.m)
    Kn = node_K(Kc)
    sn = node_sigma(sigma0)
    iE, iO = _index(N, P)
    n = N * P + (N + 1) * P
    rows, cols, vals = [], [], []
    rhs = np.zeros(n, dtype=XP)
    v = mu[None, :]

    # nodes i = 1..N-1:
    #   sigma_i c dt O_J,i + K_i eps v c dt (E_J,i - E_J,i-1)/dx
    #     = -K_i eps^2 (O*_i - O^n_i) - K_i ac v c dt (U*_i - U*_{i-1})/dx
    r = iO[1:N]
    Ki, si = Kn[:, None], sn[:, None]
    dU = (Us[1:N] - Us[0:N - 1])[:, None]
    rows += [r, r, r]
    cols += [iO[1:N], iE[1:N], iE[0:N - 1]]
    vals += [np.broadcast_to(si * c * dt, r.shape), Ki * eps * v * c * dt / dx, -Ki * eps * v * c * dt / dx]
    rhs[r.ravel()] = (-Ki * eps ** 2 * (Os[1:N] - O[1:N]) - Ki * a * c * v * c * dt / dx * dU).ravel()

    # inflow relations (4.6) for the state ac U* + eps Jh
    one = np.ones(P, dtype=XP)
    r = iO[0]
    rows += [r, r, r]
    cols += [iE[0], iO[0], iO[1]]
    vals += [one * eps, one * eps / 2, one * eps / 2]
    rhs[r] = bL - a * c * Us[0]
    r = iO[N]
    rows += [r, r, r]
    cols += [iE[N - 1], iO[N - 1], iO[N]]
    vals += [one * eps, -one * eps / 2, -one * eps / 2]
    rhs[r] = bR - a * c * Us[N - 1]

    # cells j = 0..N-1:
    #   sigma0_j c dt E_J,j + K_j eps v c dt (O_J,j+1 - O_J,j)/dx = -K_j eps (E*_j - E^n_j)
    r = iE
    Kj, s0 = Kc[:, None], sigma0[:, None]
    rows += [r, r, r]
    cols += [iE, iO[1:N + 1], iO[0:N]]
    vals += [np.broadcast_to(s0 * c * dt, r.shape), Kj * eps * v * c * dt / dx, -Kj * eps * v * c * dt / dx]
    rhs[r.ravel()] = (-Kj * eps * (Es - E)).ravel()

    A = coo(rows, cols, vals, n)
    x, _, _ = solve_refined(A, rhs)
    return x[:N * P].reshape(N, P), x[N * P:].reshape(N + 1, P)


def alt_step(E, O, T, sigma0, mu, omega, bL, bR, ph):
    """One step with the prediction of Algorithm 2 and the correction (3.14).
    Needs sigma0 > 0 in every cell (the stage divides by the node opacity).
    Returns a dict of binary64 arrays (as ap1d.ap_step)."""
    E = np.asarray(E, dtype=np.float64)
    O = np.asarray(O, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    sigma0 = np.asarray(sigma0, dtype=np.float64)
    N, P = E.shape
    if N < 2 or O.shape != (N + 1, P) or T.shape != (N,) or sigma0.shape != (N,):
        raise ValueError("shape mismatch")
    if not np.all(sigma0 > 0):
        raise ValueError("the alternative correction needs sigma0 > 0")
    Ex, Ox, Tx, sx = (np.asarray(x, dtype=XP) for x in (E, O, T, sigma0))
    mux, omx = np.asarray(mu, dtype=XP), np.asarray(omega, dtype=XP)
    bLx, bRx = np.asarray(bL, dtype=XP), np.asarray(bR, dtype=XP)
    a, c, Cv, eps, dt, L = ph.ext()
    dx = L / N

    Es, Os, Us = predict(Ex, Ox, Tx, sx, mux, omx, bLx, bRx, ph)
    EJ, OJ = correct_alt(Ex, Ox, Tx, Es, Os, Us, sx, mux, bLx, bRx, ph)
    Kc = cell_K(Tx, ph.m)
    rhoJ = moment(EJ, omx)
    Tnew = Tx + dt * sx * rhoJ / (eps * Kc * Cv)            # (3.14b)
    Unew = Tnew ** 4                                         # projection (4.14)
    Enew = a * c * Unew[:, None] + eps * EJ
    f64 = lambda x: np.asarray(x, dtype=np.float64)
    DJ = ((OJ[1:] - OJ[:-1]) * mux) @ omx / dx
    return dict(E=f64(Enew), O=f64(OJ), T=f64(Tnew), U=f64(Unew), E_star=f64(Es), O_star=f64(Os),
                U_star=f64(Us), rho_n=f64(moment(Ex, omx)), rho_star=f64(moment(Es, omx)),
                E_J=f64(EJ), O_J=f64(OJ), D_J=f64(DJ), rho=f64(moment(Enew, omx)))
