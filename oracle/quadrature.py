"""Velocity quadrature for the 1-D parity formulation (test infrastructure).

Section 4 averages over v in [-1, 1] with <f> = (1/2) * int_{-1}^{1} f dv and
stores only v > 0 through the even/odd parities (4.2).  The paper leaves the
velocity grid unspecified (remark after (4.5)); the workloads use an N_v-point
Gauss-Legendre rule on [-1, 1].  The parity pairs are its positive nodes,
ordered by increasing mu, with pair weight omega_p equal to the [-1, 1]
Gauss-Legendre weight of +mu_p, so that

    rho = <I> = sum_p omega_p * E_p ,   sum_p omega_p = 1 ,

which is the discrete form of "int_0^1 E dv" used in (4.5c) and (4.13).
"""
import numpy as np


def gauss_legendre_pairs(nv):
    """Return (mu, omega) for the nv/2 parity pairs of an nv-point GL rule."""
    nv = int(nv)
    if nv < 2 or nv % 2:
        raise ValueError("the number of ordinates must be even and >= 2")
    x, w = np.polynomial.legendre.leggauss(nv)
    pos = x > 0
    mu = np.asarray(x[pos], dtype=np.float64)
    omega = np.asarray(w[pos], dtype=np.float64)
    order = np.argsort(mu)
    return mu[order].copy(), omega[order].copy()
