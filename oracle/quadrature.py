"""Velocity quadrature for the parity formulation (test infrastructure).

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


def circle_pairs(nv):
    """Return (mu, eta, omega) for the nv/2 parity pairs of nv equally spaced
    directions on the unit circle (the 2-D workloads).

    The paper is one-dimensional; its 2-D extension needs a direction set.
    Directions theta_k = 2 pi (k + 1/2) / nv, k = 0..nv-1, each carrying the
    weight 1/nv of <f> = (1/2pi) int f dtheta.  Pair p = k < nv/2 holds
    Omega_p = (cos theta_p, sin theta_p) (so eta_p > 0) and its opposite -Omega_p;
    the pair weight is omega_p = 2/nv, sum_p omega_p = 1.  nv must be a multiple
    of 4: then no direction is parallel to an edge (mu_p != 0, eta_p != 0) and
    sum_p omega_p mu_p eta_p = 0, sum_p omega_p mu_p^2 = sum_p omega_p eta_p^2 = 1/2.
    """
    nv = int(nv)
    if nv < 4 or nv % 4:
        raise ValueError("the number of directions must be a positive multiple of 4")
    k = np.arange(nv // 2)
    theta = 2.0 * np.pi * (k + 0.5) / nv
    return np.cos(theta), np.sin(theta), np.full(nv // 2, 2.0 / nv)
