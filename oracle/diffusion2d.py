"""The diffusion limit on a 2-D rectangle (test infrastructure).

As eps -> 0 the AP step must reduce to a discretisation of the nonlinear
diffusion equation of the limit, in d space dimensions
    a d_t T^4 + Cv d_t T = div( ac K <mu^2> / sigma grad T^4 ),   K = T^m,
where <mu^2> = 1/D_d is the second moment of the direction set (1/3 for the
1-D Gauss-Legendre ordinates, 1/2 for directions on the unit circle).  This
module holds the 2-D form of the three-stage scheme (2.7) and of its sigma/T^3
version (2.9) on the AP step's cell-centred grid:

  Stage 1 (prediction, linear):
    (U* - U^n)/dt = 4 T^3/(4 a T^3 + Cv) div(F^n grad U*)
  Stage 2 (correction, one scalar equation per cell):
    a (T^4 - U^n)/dt + Cv (T - T^n)/dt = div(F^n grad U*)
  Stage 3 (projection): U^{n+1} = (T^{n+1})^4,

with the 5-point divergence of face fluxes F_f (U_right - U_left)/h, the face
coefficient F_f = ac <mu^2> K_f / sigma_f (sigma_f harmonic mean and K_f mean of
the two cells, as the AP step's faces), closed edges (zero flux).  The
correction's flux keeps F^n, the limit of the discrete correction (which takes
O* from the prediction).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _harm(a, b):
    return 2.0 * a * b / (a + b)


def _faces(T, sigma0, m, a, c, mu2):
    K = np.ones_like(T) if m == 0 else T ** m
    Fx = a * c * mu2 * 0.5 * (K[:, :-1] + K[:, 1:]) / _harm(sigma0[:, :-1], sigma0[:, 1:])
    Fy = a * c * mu2 * 0.5 * (K[:-1] + K[1:]) / _harm(sigma0[:-1], sigma0[1:])
    return Fx, Fy


def _laplacian(Fx, Fy, dx, dy):
    """Matrix of -div(F grad .) on the cells (row-major, x fastest), closed edges."""
    ny, nx = Fx.shape[0], Fy.shape[1]
    n = nx * ny
    idx = np.arange(n).reshape(ny, nx)
    rows, cols, vals = [], [], []
    diag = np.zeros((ny, nx))
    wx = Fx / dx ** 2
    wy = Fy / dy ** 2
    # x-faces between (iy, ix) and (iy, ix + 1)
    diag[:, :-1] += wx
    diag[:, 1:] += wx
    rows += [idx[:, :-1].ravel(), idx[:, 1:].ravel()]
    cols += [idx[:, 1:].ravel(), idx[:, :-1].ravel()]
    vals += [-wx.ravel(), -wx.ravel()]
    diag[:-1] += wy
    diag[1:] += wy
    rows += [idx[:-1].ravel(), idx[1:].ravel()]
    cols += [idx[1:].ravel(), idx[:-1].ravel()]
    vals += [-wy.ravel(), -wy.ravel()]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def three_stage_step(T, sigma0, dt, Lx=1.0, Ly=1.0, a=1.0, c=1.0, Cv=1.0, m=0, mu2=0.5, maxit=200):
    """One step of (2.7) (m = 0) / (2.9) (m = 3) in 2-D; returns (T^{n+1}, U*)."""
    T = np.asarray(T, dtype=np.float64)
    sigma0 = np.asarray(sigma0, dtype=np.float64)
    ny, nx = T.shape
    dx, dy = Lx / nx, Ly / ny
    U = T ** 4
    Fx, Fy = _faces(T, sigma0, m, a, c, mu2)
    A = _laplacian(Fx, Fy, dx, dy)
    pref = (4.0 * T ** 3 / (4.0 * a * T ** 3 + Cv)).ravel()
    M = sp.identity(nx * ny, format="csr") + dt * sp.diags(pref) @ A
    Us = spla.spsolve(M.tocsc(), U.ravel())
    rhs = a * U.ravel() + Cv * T.ravel() - dt * (A @ Us)
    # a T^4 + Cv T = rhs per cell: Newton from above the root (monotone)
    Tk = np.maximum(np.maximum(T.ravel(), rhs / Cv), (np.maximum(rhs, 0.0) / a) ** 0.25)
    for _ in range(maxit):
        f = a * Tk ** 4 + Cv * Tk - rhs
        step = f / (4.0 * a * Tk ** 3 + Cv)
        Tk = Tk - step
        if np.all(np.abs(step) <= 1e-15 * np.maximum(np.abs(Tk), 1e-300)):
            break
    return Tk.reshape(ny, nx), Us.reshape(ny, nx)
