"""One fully discrete AP step on a 2-D rectangle (test infrastructure).

The paper derives and analyses the scheme in one space dimension (Sections 4
and 5) and names several dimensions only as the setting of the diffusion limit
(the D_d of (1.4)).  The 2-D form here is the project's reading of how the
parity discretisation extends ("MAC-staggered parity"):

  * E_p lives at cell centres, the odd parity O_p on cell faces: O^x at the
    x-faces and O^y at the y-faces are the one field O_p sampled at two kinds
    of face, exactly as O sits at the nodes in 1-D;
  * the O-equation (second equation of (4.3), transport direction
    Omega_p = (mu_p, eta_p)) holds at every interior face; at an x-face the
    derivative along x is the compact difference of the two adjacent cells and
    the derivative along y is the mean of the two cells' centred y-differences
    (one-sided at a wall); y-faces likewise with the roles swapped;
  * the E-equation holds in every cell with the discrete divergence
    mu (O^x_right - O^x_left)/dx + eta (O^y_top - O^y_bottom)/dy;
  * at a domain edge the inflow relation of (4.6) is imposed at the centre of
    the adjacent cell, through the two faces of that cell normal to the edge:
    E + s (eps/2)(O_edge + O_opposite) = b, s = +1 when +Omega_p enters the
    domain through that edge and s = -1 when -Omega_p does.

Every other ingredient is Algorithm 2 as in the 1-D oracle: (4.5) in its
K-multiplied form (5.2) for the prediction, the scalar equation (4.13) per
cell, (4.11) with (4.12) for the correction, the projection (4.14).  With
y-periodic boundaries and data that do not depend on y, the step reduces
to the 1-D step with the pairs' x-components as ordinates.

Layout (0-based):
  E[iy, ix, p]    cells, ix = 0..nx-1 along x, iy = 0..ny-1 along y;
  Ox[iy, fx, p]   x-faces, fx = 0..nx; face fx separates cells fx-1 and fx;
  Oy[fy, ix, p]   y-faces, fy = 0..ny; face fy separates cells fy-1 and fy;
  T, sigma0[iy, ix];
  b[e, p]         inflow of the pair's entering direction through edge e:
                  e = 0 (x = 0), 1 (x = Lx), 2 (y = 0), 3 (y = Ly).
With periodic_y the faces fy and fy + ny coincide: Oy[ny] repeats Oy[0] and
the edges 2, 3 carry no inflow.

Readings of points this extension leaves open:
  * sigma at a face: harmonic mean of the two cells, K: arithmetic mean (the
    1-D node rules);
  * the cell-centre odd parity used by the readout I = E +- eps O is the mean
    of the cell's four faces.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .ap1d import cell_K, temperature_equation, newton_temperature
from .linsolve import XP, solve_refined


@dataclass
class Grid2D:
    nx: int
    ny: int
    Lx: float = 1.0
    Ly: float = 1.0
    periodic_y: bool = False

    def check(self):
        if self.nx < 2:
            raise ValueError("the x-direction needs at least two cells")
        if not self.periodic_y and self.ny < 2:
            raise ValueError("the y-direction needs at least two cells (or periodic_y)")


def _harm(a, b):
    den = a + b
    out = np.zeros_like(den)
    nz = den > 0
    out[nz] = 2 * a[nz] * b[nz] / den[nz]
    return out


def _diff(n, i, h, periodic):
    """Centred difference at cell i of an axis of n cells, spacing h, as a list of
    (cell index, weight); one-sided next to a wall, wrapped when periodic."""
    if periodic:
        return [((i + 1) % n, 1 / (2 * h)), ((i - 1) % n, -1 / (2 * h))]
    if i == 0:
        return [(1, 1 / h), (0, -1 / h)]
    if i == n - 1:
        return [(n - 1, 1 / h), (n - 2, -1 / h)]
    return [(i + 1, 1 / (2 * h)), (i - 1, -1 / (2 * h))]


class _Index:
    """Unknown numbering: E (cell-major, pair fastest), then O^x, then O^y."""

    def __init__(self, g, P):
        self.g, self.P = g, P
        self.nE = g.ny * g.nx * P
        self.nOx = g.ny * (g.nx + 1) * P
        self.nOy = (g.ny + 1) * g.nx * P
        self.n = self.nE + self.nOx + self.nOy
        self.p = np.arange(P)

    def E(self, iy, ix):
        return (iy * self.g.nx + ix) * self.P + self.p

    def Ox(self, iy, fx):
        return self.nE + (iy * (self.g.nx + 1) + fx) * self.P + self.p

    def Oy(self, fy, ix):
        return self.nE + self.nOx + (fy * self.g.nx + ix) * self.P + self.p


def face_coefficients(sigma0, Kc, periodic_y):
    """sigma and K at the faces that carry an O-equation.

    Returns (sx, Kx) of shape (ny, nx-1) for the interior x-faces fx = 1..nx-1,
    and (sy, Ky) for the y-faces fy = 1..ny-1 (walls) or fy = 0..ny-1 (periodic;
    face 0 joins cells ny-1 and 0)."""
    sx = _harm(sigma0[:, :-1], sigma0[:, 1:])
    Kx = (Kc[:, :-1] + Kc[:, 1:]) / 2
    if periodic_y:
        below_s, below_K = np.roll(sigma0, 1, axis=0), np.roll(Kc, 1, axis=0)
        sy, Ky = _harm(below_s, sigma0), (below_K + Kc) / 2
    else:
        sy = _harm(sigma0[:-1], sigma0[1:])
        Ky = (Kc[:-1] + Kc[1:]) / 2
    return sx, Kx, sy, Ky


def _operators(g, mu, eta, idx):
    """The sparse pieces shared by both linear systems.

    Gx, Gy: rows = O-equation faces, columns = cell unknowns; row (face, p)
            holds mu_p d_x X + eta_p d_y X at that face (the discretisation of
            Omega_p . grad X described in the module docstring).
    Dv:     rows = cell unknowns, columns = face unknowns; row (cell, p) holds
            mu_p (O^x_right - O^x_left)/dx + eta_p (O^y_top - O^y_bottom)/dy.
    Returned as lists of COO triples in the global numbering."""
    nx, ny, P = g.nx, g.ny, idx.P
    dx, dy = XP(g.Lx) / nx, XP(g.Ly) / ny
    G, Dv = ([], [], []), ([], [], [])

    def add(T, r, c, v):
        T[0].append(r)
        T[1].append(c)
        T[2].append(np.broadcast_to(np.asarray(v, dtype=XP), (P,)))

    # x-faces fx = 1..nx-1
    for iy in range(ny):
        for fx in range(1, nx):
            r = idx.Ox(iy, fx)
            add(G, r, idx.E(iy, fx), mu / dx)
            add(G, r, idx.E(iy, fx - 1), -mu / dx)
            for ix in (fx - 1, fx):
                for jy, w in _diff(ny, iy, dy, g.periodic_y):
                    add(G, r, idx.E(jy, ix), eta * w / 2)
    # y-faces
    fys = range(ny) if g.periodic_y else range(1, ny)
    for fy in fys:
        lo = (fy - 1) % ny
        for ix in range(nx):
            r = idx.Oy(fy, ix)
            add(G, r, idx.E(fy, ix), eta / dy)
            add(G, r, idx.E(lo, ix), -eta / dy)
            for iy in (lo, fy):
                for jx, w in _diff(nx, ix, dx, False):
                    add(G, r, idx.E(iy, jx), mu * w / 2)
    # divergence in every cell
    for iy in range(ny):
        for ix in range(nx):
            r = idx.E(iy, ix)
            add(Dv, r, idx.Ox(iy, ix + 1), mu / dx)
            add(Dv, r, idx.Ox(iy, ix), -mu / dx)
            add(Dv, r, idx.Oy(iy + 1, ix), eta / dy)
            add(Dv, r, idx.Oy(iy, ix), -eta / dy)
    return G, Dv


def _matrix(T, n_rows, n_cols, row0=0, col0=0):
    r = np.concatenate([np.ravel(x) for x in T[0]]) - row0
    c = np.concatenate([np.ravel(x) for x in T[1]]) - col0
    v = np.concatenate([np.ravel(x) for x in T[2]])
    return sp.csr_matrix((v, (r, c)), shape=(n_rows, n_cols), dtype=XP)


def _system(g, E_n, Ox_n, Oy_n, Kc, sigma0, mu, eta, omega, b, ph, fe, co, cell_diag,
            cell_rhs, face_rhs_extra, bc_rhs, coupling):
    """Assemble the common structure of (4.5)/(5.2) and (4.11):

      face rows  (K eps^2 + sigma c dt) O + K c dt fe (Omega . grad X) = K eps^2 O^n + extra
      inflow     fe X_cell + s (eps/2)(O_edge + O_opposite) = bc_rhs
      cell rows  cell_diag X + K co c dt div O - coupling = cell_rhs

    X is E* (fe = 1, co = eps^2) in the prediction and E_J (fe = eps,
    co = eps) in the correction.  Returns (A, rhs, index)."""
    nx, ny = g.nx, g.ny
    P = mu.size
    idx = _Index(g, P)
    a, c, Cv, eps, dt, _ = ph.ext()
    sx, Kx, sy, Ky = face_coefficients(sigma0, Kc, g.periodic_y)
    G, Dv = _operators(g, mu, eta, idx)
    Gm = _matrix(G, idx.n, idx.n)
    Dm = _matrix(Dv, idx.n, idx.n)
    rows, cols, vals = [], [], []
    rhs = np.zeros(idx.n, dtype=XP)
    face_scale = np.zeros(idx.n, dtype=XP)       # K c dt fe multiplying Gm, per face row

    def put(r, cc, v):
        rows.append(r)
        cols.append(cc)
        vals.append(np.broadcast_to(np.asarray(v, dtype=XP), (P,)))

    # O-equation at the interior x-faces
    for iy in range(ny):
        for fx in range(1, nx):
            r = idx.Ox(iy, fx)
            K, s = Kx[iy, fx - 1], sx[iy, fx - 1]
            put(r, r, K * eps ** 2 + s * c * dt)
            face_scale[r] = K * c * dt * fe
            rhs[r] = K * eps ** 2 * Ox_n[iy, fx] + face_rhs_extra[0][iy, fx - 1]
    # O-equation at the y-faces
    fys = range(ny) if g.periodic_y else range(1, ny)
    for fy in fys:
        for ix in range(nx):
            r = idx.Oy(fy, ix)
            k = fy if g.periodic_y else fy - 1
            K, s = Ky[k, ix], sy[k, ix]
            put(r, r, K * eps ** 2 + s * c * dt)
            face_scale[r] = K * c * dt * fe
            rhs[r] = K * eps ** 2 * Oy_n[fy, ix] + face_rhs_extra[1][k, ix]
    # inflow relations, x = 0 and x = Lx
    sgn = np.sign(mu)
    for iy in range(ny):
        for e, fx, fo, ix, s in ((0, 0, 1, 0, sgn), (1, nx, nx - 1, nx - 1, -sgn)):
            r = idx.Ox(iy, fx)
            put(r, idx.E(iy, ix), fe)
            put(r, r, s * eps / 2)
            put(r, idx.Ox(iy, fo), s * eps / 2)
            rhs[r] = bc_rhs(e, iy, ix)
    if g.periodic_y:
        for ix in range(nx):          # the face ny is the face 0
            r = idx.Oy(ny, ix)
            put(r, r, 1.0)
            put(r, idx.Oy(0, ix), -1.0)
    else:
        sgn = np.sign(eta)
        for ix in range(nx):
            for e, fy, fo, iy, s in ((2, 0, 1, 0, sgn), (3, ny, ny - 1, ny - 1, -sgn)):
                r = idx.Oy(fy, ix)
                put(r, idx.E(iy, ix), fe)
                put(r, r, s * eps / 2)
                put(r, idx.Oy(fo, ix), s * eps / 2)
                rhs[r] = bc_rhs(e, iy, ix)
    # E-equation in every cell
    cell_scale = np.zeros(idx.n, dtype=XP)
    for iy in range(ny):
        for ix in range(nx):
            r = idx.E(iy, ix)
            put(r, r, cell_diag[iy, ix])
            cell_scale[r] = Kc[iy, ix] * co * c * dt
            rhs[r] = cell_rhs[iy, ix]
            if coupling is not None:          # -g_cell sum_q omega_q X_q in every row p
                gq = coupling[iy, ix]
                for p in range(P):
                    rows.append(np.full(P, r[p]))
                    cols.append(r)
                    vals.append(-gq * omega)
    A = _matrix((rows, cols, vals), idx.n, idx.n)
    A = A + sp.diags(face_scale, format="csr", dtype=XP) @ Gm + sp.diags(cell_scale, format="csr", dtype=XP) @ Dm
    return A.tocsr(), rhs, idx


def _unpack(x, idx):
    g, P = idx.g, idx.P
    E = x[:idx.nE].reshape(g.ny, g.nx, P)
    Ox = x[idx.nE:idx.nE + idx.nOx].reshape(g.ny, g.nx + 1, P)
    Oy = x[idx.nE + idx.nOx:].reshape(g.ny + 1, g.nx, P)
    return E, Ox, Oy


def _face_gradient(g, X, mu, eta):
    """Omega_p . grad X at the O-equation faces for a cell field X (no pair
    dependence): ((ny, nx-1, P), (faces_y, nx, P)); the same stencil as Gx, Gy."""
    nx, ny = g.nx, g.ny
    dx, dy = XP(g.Lx) / nx, XP(g.Ly) / ny
    d_y = np.zeros((ny, nx), dtype=XP)
    d_x = np.zeros((ny, nx), dtype=XP)
    for iy in range(ny):
        for jy, w in _diff(ny, iy, dy, g.periodic_y):
            d_y[iy] += w * X[jy]
    for ix in range(nx):
        for jx, w in _diff(nx, ix, dx, False):
            d_x[:, ix] += w * X[:, jx]
    gx = (mu[None, None, :] * ((X[:, 1:] - X[:, :-1]) / dx)[:, :, None]
          + eta[None, None, :] * ((d_y[:, :-1] + d_y[:, 1:]) / 2)[:, :, None])
    if g.periodic_y:
        lo = np.roll(X, 1, axis=0)
        dlo = np.roll(d_x, 1, axis=0)
    else:
        lo, dlo = X[:-1], d_x[:-1]
    hi, dhi = (X, d_x) if g.periodic_y else (X[1:], d_x[1:])
    gy = (eta[None, None, :] * ((hi - lo) / dy)[:, :, None]
          + mu[None, None, :] * ((dlo + dhi) / 2)[:, :, None])
    return gx, gy


# --------------------------------------------------------------------------
# Algorithm 2 in 2-D
# --------------------------------------------------------------------------
def predict(g, E, Ox, Oy, T, sigma0, mu, eta, omega, b, ph):
    """Prediction (4.5)/(5.2): U* eliminated with (4.5c) exactly as in 1-D
    (U* = (U^n + beta rho*)/(1 + ac beta)), the rest solved as one linear
    system in (E*, O^x*, O^y*).  Rows multiplied by eps^2 c dt."""
    a, c, Cv, eps, dt, _ = ph.ext()
    m = ph.m
    U = T ** 4
    Kc = cell_K(T, m)
    beta = 4 * sigma0 * dt * T ** (3 - m) / (eps ** 2 * Cv)
    gcpl = sigma0 * c * dt * a * c * beta / (1 + a * c * beta)
    P = mu.size
    diag = Kc * eps ** 2 + sigma0 * c * dt

    def bc(e, iy, ix):
        return b[e]

    nfy = g.ny if g.periodic_y else g.ny - 1
    extra = (np.zeros((g.ny, g.nx - 1, P), dtype=XP), np.zeros((nfy, g.nx, P), dtype=XP))
    rhs_cells = (Kc[:, :, None] * eps ** 2 * E
                 + (sigma0 * c * dt * a * c * U / (1 + a * c * beta))[:, :, None])
    A, rhs, idx = _system(g, E, Ox, Oy, Kc, sigma0, mu, eta, omega, b, ph,
                          fe=XP(1), co=eps ** 2, cell_diag=diag[:, :, None] * np.ones(P, dtype=XP),
                          cell_rhs=rhs_cells, face_rhs_extra=extra, bc_rhs=bc, coupling=gcpl)
    x, _, _ = solve_refined(A, rhs)
    Es, Oxs, Oys = _unpack(x, idx)
    rho = Es @ omega
    Us = (U + beta * rho) / (1 + a * c * beta)
    return Es, Oxs, Oys, Us


def flux_divergence(g, Ox, Oy, mu, eta, omega):
    """D = sum_p omega_p [mu_p (O^x_right - O^x_left)/dx + eta_p (O^y_top - O^y_bottom)/dy]
    per cell (right side of (4.13))."""
    dx, dy = XP(g.Lx) / g.nx, XP(g.Ly) / g.ny
    return (((Ox[:, 1:] - Ox[:, :-1]) * mu) @ omega / dx
            + ((Oy[1:] - Oy[:-1]) * eta) @ omega / dy)


def correct_J(g, E, Ox, Oy, Tnew, sigma0, mu, eta, b, ph):
    """Correction substep 2: (4.11a,b) with (4.12), U^{n+1} = (T^{n+1})^4 and
    K^{n+1}; face rows multiplied by eps^2 c dt, cell rows by eps c dt."""
    a, c, Cv, eps, dt, _ = ph.ext()
    P = mu.size
    U = Tnew ** 4
    Kc = cell_K(Tnew, ph.m)
    sx, Kx, sy, Ky = face_coefficients(sigma0, Kc, g.periodic_y)
    gx, gy = _face_gradient(g, a * c * U, mu, eta)
    extra = (-(Kx * c * dt)[:, :, None] * gx, -(Ky * c * dt)[:, :, None] * gy)
    diag = Kc * eps ** 2 + sigma0 * c * dt
    rhs_cells = Kc[:, :, None] * eps * (E - a * c * U[:, :, None])

    def bc(e, iy, ix):
        return b[e] - a * c * U[iy, ix]

    A, rhs, idx = _system(g, E, Ox, Oy, Kc, sigma0, mu, eta, None, b, ph,
                          fe=eps, co=eps, cell_diag=diag[:, :, None] * np.ones(P, dtype=XP),
                          cell_rhs=rhs_cells, face_rhs_extra=extra, bc_rhs=bc, coupling=None)
    x, _, _ = solve_refined(A, rhs)
    return _unpack(x, idx)


def ap_step(g, E, Ox, Oy, T, sigma0, mu, eta, omega, b, ph, newton_maxit=200):
    """Advance (E, O^x, O^y, T) by one step of Algorithm 2.  Returns a dict of
    every stage (binary64 arrays)."""
    g.check()
    E, Ox, Oy, T, sigma0 = (np.asarray(x, dtype=np.float64) for x in (E, Ox, Oy, T, sigma0))
    nx, ny = g.nx, g.ny
    P = np.asarray(mu).size
    if (E.shape != (ny, nx, P) or Ox.shape != (ny, nx + 1, P) or Oy.shape != (ny + 1, nx, P)
            or T.shape != (ny, nx) or sigma0.shape != (ny, nx)):
        raise ValueError("shape mismatch")
    if ph.m not in (0, 3):
        raise ValueError("opacity law exponent must be 0 or 3")
    Ex, Oxx, Oyx, Tx, sx = (np.asarray(x, dtype=XP) for x in (E, Ox, Oy, T, sigma0))
    mux, etax, omx = (np.asarray(x, dtype=XP) for x in (mu, eta, omega))
    bx = np.asarray(b, dtype=XP).reshape(4, P)

    Es, Oxs, Oys, Us = predict(g, Ex, Oxx, Oyx, Tx, sx, mux, etax, omx, bx, ph)

    rho_n = Ex @ omx
    D = flux_divergence(g, Oxs, Oys, mux, etax, omx)
    Kstar = np.ones_like(Tx) if ph.m == 0 else np.maximum(Us, 0) ** XP(0.75)
    Tnew, its, conv = newton_temperature(Tx.ravel(), rho_n.ravel(), D.ravel(), Kstar.ravel(),
                                         sx.ravel(), ph, maxit=newton_maxit)
    Tnew = Tnew.reshape(ny, nx)
    Tnew = np.where((sx == 0) & (Kstar == 0), Tx, Tnew)

    EJ, OxJ, OyJ = correct_J(g, Ex, Oxx, Oyx, Tnew, sx, mux, etax, bx, ph)

    a, c, _, eps, _, _ = ph.ext()
    Unew = Tnew ** 4
    Enew = a * c * Unew[:, :, None] + eps * EJ
    f64 = lambda x: np.asarray(x, dtype=np.float64)
    return dict(E=f64(Enew), Ox=f64(OxJ), Oy=f64(OyJ), T=f64(Tnew), U=f64(Unew),
                E_star=f64(Es), Ox_star=f64(Oxs), Oy_star=f64(Oys), U_star=f64(Us),
                rho_n=f64(rho_n), rho_star=f64(Es @ omx), D=f64(D), K_star=f64(Kstar),
                E_J=f64(EJ), rho=f64(Enew @ omx),
                newton_its=its.reshape(ny, nx), newton_converged=conv.reshape(ny, nx))


def cell_odd(Ox, Oy):
    """Cell-centre odd parity: the mean of the cell's four face values."""
    return (Ox[:, 1:] + Ox[:, :-1] + Oy[1:] + Oy[:-1]) / 4


def intensity(E, Ox, Oy, eps):
    """Cell-centre I(+Omega_p), I(-Omega_p) = E +- eps O_cell."""
    Oc = cell_odd(Ox, Oy)
    return E + eps * Oc, E - eps * Oc


def total_energy(g, E, T, omega, c=1.0, Cv=1.0):
    """sum over cells of dx dy (rho / c + Cv T)."""
    dx, dy = g.Lx / g.nx, g.Ly / g.ny
    return float(np.sum(dx * dy * ((E @ omega) / c + Cv * T)))


def boundary_outflow(g, Ox, Oy, mu, eta, omega):
    """Net outward flux through the four edges,
    sum_p omega_p [mu_p sum_iy dy (O^x_nx - O^x_0) + eta_p sum_ix dx (O^y_ny - O^y_0)]."""
    dx, dy = g.Lx / g.nx, g.Ly / g.ny
    fx = dy * np.sum((Ox[:, -1] - Ox[:, 0]) * mu, axis=0) @ omega
    fy = dx * np.sum((Oy[-1] - Oy[0]) * eta, axis=0) @ omega
    return float(fx + fy)
