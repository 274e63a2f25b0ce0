"""Energy bookkeeping of the AP step (test infrastructure).

(3.12): (1/c) d_t <I> + Cv d_t T + (1/eps) <v . grad I> = 0.  In the parity
variables (4.2) the flux term of cell j is
    D_j = sum_p omega_p mu_p (O_{j+1,p} - O_{j,p}) / dx ,
and the paper shows that its three-stage update is conservative up to the
defect term of (3.13).  For the fully discrete step the same algebra (sum of
(4.13) and of (4.11b) over the directions) gives, per cell, with
rho' = rho^{n+1}, dT = T^{n+1} - T^n, D* from O*, D' from O^{n+1}:

  (rho' - rho^n)/(c dt) + Cv dT/dt + D*
      = [eps^2 K' (D* - D') + Cv (dT/dt) eps^2 (K' - K*)] / (eps^2 K' + c sigma0 dt),

K* = (U*)^(3/4) and K' = (T^{n+1})^3 for sigma/T^3 ((5.3)-(5.5)), K* = K' = 1
when sigma does not depend on T -- then the identity is exactly the fully
discrete form of (3.13), whose defect is eps^2/(c sigma dt + eps^2) times the
change of the flux between prediction and correction.
"""
import numpy as np


def cell_fluxdiv(O, mu, omega, dx):
    return ((O[1:, :] - O[:-1, :]) * mu) @ omega / dx


def total_energy(E, T, omega, dx, c=1.0, Cv=1.0):
    """sum_j dx (rho_j / c + Cv T_j)."""
    return float(np.sum(dx * ((E @ omega) / c + Cv * T)))


def boundary_flux(O, mu, omega):
    """Net outward flux sum_p omega_p mu_p (O_{N} - O_{0}) (node values)."""
    return float((O[-1] - O[0]) @ (mu * omega))


def conservation_terms(res, E_n, T_n, sigma0, mu, omega, ph):
    """Left and right sides of the per-cell identity above."""
    N = T_n.size
    dx = ph.L / N
    c, Cv, eps, dt = ph.c, ph.Cv, ph.eps, ph.dt
    rho_n = E_n @ omega
    rho1 = res["E"] @ omega
    dT = res["T"] - T_n
    Ds = cell_fluxdiv(res["O_star"], mu, omega, dx)
    D1 = cell_fluxdiv(res["O"], mu, omega, dx)
    lhs = (rho1 - rho_n) / (c * dt) + Cv * dT / dt + Ds
    Ks = res["K_star"]
    K1 = np.ones_like(dT) if ph.m == 0 else res["T"] ** ph.m
    rhs = ((eps ** 2 * K1 * (Ds - D1) + Cv * dT / dt * eps ** 2 * (K1 - Ks))
           / (eps ** 2 * K1 + c * sigma0 * dt))
    scale = (np.abs(rho1 / (c * dt)) + np.abs(rho_n / (c * dt))
             + np.abs(Cv * dT / dt) + np.abs(Ds) + np.abs(D1))
    return lhs, rhs, scale
