"""Seeded synthetic workloads for the 1-D AP step (inputs only, no method).

The paper's experiments are analytic set-ups, not datasets; these generators
reproduce the benchmark configurations of this project with the shapes and
value distributions stated below.  Everything is deterministic given the
seed (numpy PCG64, seed 18110000 + configuration number).

  config 1  slab x in [0,1], N = 100, 16 Gauss-Legendre ordinates,
            a = c = Cv = 1, sigma = 1 (m = 0), eps = 1e-2, T = 1e-2,
            I = ac T^4, inflow b = ac at x = 0 (mu > 0), vacuum at x = 1,
            dt = 0.5 dx, 200 steps.
  config 2  N = 4096, 64 ordinates, sigma = sigma0 T^-3 with sigma0 ~ U[0.5, 2]
            i.i.d. per cell, eps in {1, 1e-2, 1e-4}, same initial and inflow
            data, dt = 0.5 dx, 2000 steps.

  config 4  batched ensemble: 4096 independent slabs with N ~ U{64..2048},
            N_v uniform in {8, 16, 32, 64}, eps = 10^U[-5, 0], one sigma0 =
            10^U[-1, 2] per slab with sigma = sigma0 T^-3, the initial and inflow
            data of config 1, dt = 0.5 / N.

  config 5  (one-dimensional analogue of the two-material learned-guess case)
            N = 512, 64 ordinates, sigma in {1, 1000} (m = 0) piecewise
            constant on the cells nearest to 64 seeded sites in [0, 1], each site
            taking either value with probability 1/2, eps = 1e-4, the initial
            and inflow data of config 1, dt = 0.5 dx.

  config 3  2-D square [0,1]^2, 1024 x 1024 cells, 32 equally spaced circle
            directions, two-material opacity: the cell takes the value of the
            nearest of 64 seeded sites (Voronoi), each site sigma in {1, 100}
            with probability 1/2, m = 0, eps = 1e-3, T = 1e-2 and I = ac T^4
            initially, isotropic inflow ac on the edge x = 0, vacuum elsewhere,
            dt = 0.5 dx.
  config 5  the same set-up on 512 x 512 cells, 64 directions, sigma in
            {1, 1000}, eps = 1e-4 (the learned-guess case).

  marshak   dimensional Marshak wave of the paper's last example: eps = 1,
            c = 29.98 cm/ns, a = 0.01372 GJ/(cm^3 keV^4), Cv = 0.3 GJ/(cm^3 keV),
            sigma = 300 / T^3 cm^-1, x in [0, 0.02] cm, T(x, 0) =
            (1 - tanh((x - 0.0024) 1000)) / 2 keV in equilibrium (I = a c T^4),
            T = 1 keV at x = 0 imposed as the isotropic inflow a c 1^4, the
            right-end inflow a c T(0.02, 0)^4; dt in ns (1.6e-12 s = 1.6e-3 ns).

The 2-D direction set is theta_k = 2 pi (k + 1/2)/N_v; the pairs are k < N_v/2
(eta > 0), each with weight 2/N_v.

The velocity grid (Gauss-Legendre pairs: positive nodes by increasing mu,
weight of +mu on [-1, 1], so the weights sum to one) is part of the input:
both the oracle and the GPU library receive these exact binary64 values.
"""
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 18110000


def gauss_legendre_pairs(nv):
    """Positive nodes of the nv-point Gauss-Legendre rule and their weights."""
    x, w = np.polynomial.legendre.leggauss(int(nv))
    pos = x > 0
    order = np.argsort(x[pos])
    return (np.ascontiguousarray(x[pos][order], dtype=np.float64),
            np.ascontiguousarray(w[pos][order], dtype=np.float64))


@dataclass
class Workload:
    name: str
    N: int
    nv: int
    m: int
    eps: float
    dt: float
    steps: int
    a: float = 1.0
    c: float = 1.0
    Cv: float = 1.0
    L: float = 1.0
    mu: np.ndarray = field(default=None, repr=False)
    omega: np.ndarray = field(default=None, repr=False)
    sigma0: np.ndarray = field(default=None, repr=False)
    T: np.ndarray = field(default=None, repr=False)
    E: np.ndarray = field(default=None, repr=False)
    O: np.ndarray = field(default=None, repr=False)
    bL: np.ndarray = field(default=None, repr=False)
    bR: np.ndarray = field(default=None, repr=False)

    @property
    def P(self):
        return self.nv // 2

    def cell_angle_updates(self):
        """N_cells * N_v: the unit of the throughput metric."""
        return self.N * self.nv


def _slab(name, N, nv, m, eps, steps, sigma0, T_in=1e-2, b_hot=1.0, a=1.0, c=1.0, Cv=1.0,
          cfl=0.5, L=1.0):
    mu, om = gauss_legendre_pairs(nv)
    P = nv // 2
    T = np.full(N, T_in, dtype=np.float64)
    E = np.full((N, P), a * c * T_in ** 4, dtype=np.float64)
    O = np.zeros((N + 1, P), dtype=np.float64)
    bL = np.full(P, a * c * b_hot ** 4, dtype=np.float64)
    bR = np.zeros(P, dtype=np.float64)
    dt = cfl * L / N
    return Workload(name=name, N=N, nv=nv, m=m, eps=eps, dt=dt, steps=steps, a=a, c=c, Cv=Cv,
                    L=L, mu=mu, omega=om, sigma0=np.asarray(sigma0, dtype=np.float64),
                    T=T, E=E, O=O, bL=bL, bR=bR)


def config1():
    """1-D, N = 100, GL16, sigma = 1, eps = 1e-2, 200 steps."""
    N = 100
    return _slab("config1", N, 16, 0, 1e-2, 200, np.ones(N))


def config2(eps=1e-2, N=4096, nv=64, steps=2000):
    """1-D, N = 4096, GL64, sigma0 T^-3 with seeded sigma0 ~ U[0.5, 2]."""
    if eps not in (1.0, 1e-2, 1e-4) and (N, nv) == (4096, 64):
        raise ValueError("config 2 is defined for eps in {1, 1e-2, 1e-4}")
    rng = np.random.default_rng(SEED_BASE + 2)
    sigma0 = rng.uniform(0.5, 2.0, 4096)
    if N != 4096:
        sigma0 = np.random.default_rng(SEED_BASE + 2).uniform(0.5, 2.0, N)
    return _slab(f"config2(eps={eps:g})", N, nv, 3, eps, steps, sigma0)


def random_state(N, nv, seed, m=3, eps=1e-2, T_lo=0.05, T_hi=1.0, anisotropy=0.2,
                 scaled=True):
    """A generic state with seeded temperature, opacity and inflow, used to
    exercise every code path (not one of the named configurations).

    With `scaled`, the angular deviation of E from a T^4 follows the scaling of
    the equations, E = acT^4 + eps E_J: its relative size is anisotropy*min(1, eps).
    """
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    mu, om = gauss_legendre_pairs(nv)
    P = nv // 2
    T = rng.uniform(T_lo, T_hi, N)
    dev = anisotropy * (min(1.0, eps) if scaled else 1.0)
    E = (T ** 4)[:, None] * (1.0 + dev * rng.uniform(-1, 1, (N, P)))
    O = 0.1 * rng.normal(size=(N + 1, P)) * np.max(E)
    sigma0 = rng.uniform(0.3, 3.0, N)
    bL = rng.uniform(0.5, 1.5, P)
    bR = rng.uniform(0.0, 0.3, P)
    return Workload(name=f"random(N={N},nv={nv},seed={seed})", N=N, nv=nv, m=m, eps=eps,
                    dt=0.5 / N, steps=1, mu=mu, omega=om, sigma0=sigma0, T=T, E=E, O=O,
                    bL=bL, bR=bR)


@dataclass
class Ensemble:
    """Independent slabs advanced together (packed in instance order)."""
    name: str
    members: list

    def __len__(self):
        return len(self.members)

    def cell_angle_updates(self):
        return sum(w.cell_angle_updates() for w in self.members)

    def packed(self):
        """Concatenated arrays in the packed layout of the batched library."""
        cat = np.concatenate
        return dict(
            mu=cat([w.mu for w in self.members]), omega=cat([w.omega for w in self.members]),
            sigma0=cat([w.sigma0 for w in self.members]), T=cat([w.T for w in self.members]),
            E=cat([w.E.ravel() for w in self.members]), O=cat([w.O.ravel() for w in self.members]),
            bL=cat([w.bL for w in self.members]), bR=cat([w.bR for w in self.members]))


def config4(n=4096, N_lo=64, N_hi=2048, nvs=(8, 16, 32, 64), seed=SEED_BASE + 4):
    """Batched ensemble: n slabs of uneven size, ordinate count, eps and opacity."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(N_lo, N_hi + 1, n)
    nv = rng.choice(np.asarray(nvs), n)
    eps = 10.0 ** rng.uniform(-5.0, 0.0, n)
    s0 = 10.0 ** rng.uniform(-1.0, 2.0, n)
    members = []
    for i in range(n):
        N = int(Ns[i])
        members.append(_slab(f"config4[{i}]", N, int(nv[i]), 3, float(eps[i]), 100,
                             np.full(N, s0[i])))
    return Ensemble(name=f"config4(n={n})", members=members)


def config5_1d(N=512, nv=64, steps=200, seed=SEED_BASE + 5):
    """Two-material slab: sigma in {1, 1000} on seeded nearest-site regions."""
    rng = np.random.default_rng(seed)
    sites = rng.uniform(0.0, 1.0, 64)
    vals = np.where(rng.uniform(0.0, 1.0, 64) < 0.5, 1.0, 1000.0)
    xc = (np.arange(N) + 0.5) / N
    nearest = np.argmin(np.abs(xc[:, None] - sites[None, :]), axis=1)   # ties -> lower index
    return _slab("config5_1d", N, nv, 0, 1e-4, steps, vals[nearest])


def mlp_init(seed=SEED_BASE + 9, scale=1.0):
    """Seeded initial parameters of the 5-64-64-1 guess network (uniform,
    fan-in scaled), float32; biases zero."""
    rng = np.random.default_rng(seed)
    w1 = rng.uniform(-1, 1, (64, 5)) * scale / np.sqrt(5)
    w2 = rng.uniform(-1, 1, (64, 64)) * scale / np.sqrt(64)
    w3 = rng.uniform(-1, 1, 64) * scale / np.sqrt(64)
    th = np.concatenate([w1.ravel(), np.zeros(64), w2.ravel(), np.zeros(64), w3, [0.0]])
    return th.astype(np.float32)


def marshak(N=100, nv=16, dt=1.6e-3, steps=100):
    """Dimensional Marshak wave (eps = 1, units cm, ns, keV, GJ)."""
    a, c, Cv, L = 0.01372, 29.98, 0.3, 0.02
    mu, om = gauss_legendre_pairs(nv)
    P = nv // 2
    xc = (np.arange(N) + 0.5) * (L / N)
    T = 0.5 * (1.0 - np.tanh((xc - 0.0024) * 1000.0))
    E = np.repeat((a * c * T ** 4)[:, None], P, axis=1)
    O = np.zeros((N + 1, P))
    TR = 0.5 * (1.0 - np.tanh((L - 0.0024) * 1000.0))
    return Workload(name=f"marshak(N={N},dt={dt:g}ns)", N=N, nv=nv, m=3, eps=1.0, dt=dt, steps=steps,
                    a=a, c=c, Cv=Cv, L=L, mu=mu, omega=om, sigma0=np.full(N, 300.0), T=T, E=E, O=O,
                    bL=np.full(P, a * c * 1.0), bR=np.full(P, a * c * TR ** 4))


# ---------------------------------------------------------------------------
# 2-D
# ---------------------------------------------------------------------------
def circle_pairs(nv):
    """(mu, eta, omega) of the nv/2 pairs of nv equally spaced directions."""
    k = np.arange(int(nv) // 2)
    th = 2.0 * np.pi * (k + 0.5) / int(nv)
    return np.cos(th), np.sin(th), np.full(k.size, 2.0 / int(nv))


@dataclass
class Workload2D:
    name: str
    nx: int
    ny: int
    nv: int
    m: int
    eps: float
    dt: float
    steps: int
    a: float = 1.0
    c: float = 1.0
    Cv: float = 1.0
    Lx: float = 1.0
    Ly: float = 1.0
    mu: np.ndarray = field(default=None, repr=False)
    eta: np.ndarray = field(default=None, repr=False)
    omega: np.ndarray = field(default=None, repr=False)
    sigma0: np.ndarray = field(default=None, repr=False)   # (ny, nx)
    T: np.ndarray = field(default=None, repr=False)        # (ny, nx)
    E: np.ndarray = field(default=None, repr=False)        # (ny, nx, P)
    Ox: np.ndarray = field(default=None, repr=False)       # (ny, nx+1, P)
    Oy: np.ndarray = field(default=None, repr=False)       # (ny+1, nx, P)
    b: np.ndarray = field(default=None, repr=False)        # (4, P)

    @property
    def P(self):
        return self.nv // 2

    def cell_angle_updates(self):
        return self.nx * self.ny * self.nv


def voronoi_two_material(nx, ny, values, seed, sites=64):
    """Cell field taking, per cell, the value of the nearest of `sites` seeded
    points in [0,1]^2; each site holds values[0] or values[1] with probability 1/2."""
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, (sites, 2))
    val = np.where(rng.uniform(0.0, 1.0, sites) < 0.5, values[0], values[1])
    xc = (np.arange(nx) + 0.5) / nx
    out = np.empty((ny, nx))
    for iy in range(ny):
        yc = (iy + 0.5) / ny
        d2 = (xc[:, None] - pts[None, :, 0]) ** 2 + (yc - pts[None, :, 1]) ** 2
        out[iy] = val[np.argmin(d2, axis=1)]
    return out


def _square(name, n, nv, m, eps, steps, sigma0, T_in=1e-2, b_hot=1.0, a=1.0, c=1.0, Cv=1.0, cfl=0.5):
    mu, eta, om = circle_pairs(nv)
    P = nv // 2
    acT = a * c * T_in ** 4
    b = np.zeros((4, P))
    b[0] = a * c * b_hot ** 4
    return Workload2D(name=name, nx=n, ny=n, nv=nv, m=m, eps=eps, dt=cfl / n, steps=steps, a=a, c=c, Cv=Cv,
                      mu=mu, eta=eta, omega=om, sigma0=np.asarray(sigma0, dtype=np.float64),
                      T=np.full((n, n), T_in), E=np.full((n, n, P), acT),
                      Ox=np.zeros((n, n + 1, P)), Oy=np.zeros((n + 1, n, P)), b=b)


def config3(n=1024, nv=32, steps=500):
    """2-D, 1024^2 cells, 32 directions, Voronoi sigma in {1, 100}, eps = 1e-3."""
    sig = voronoi_two_material(n, n, (1.0, 100.0), SEED_BASE + 3)
    return _square(f"config3(n={n})", n, nv, 0, 1e-3, steps, sig)


def config5(n=512, nv=64, steps=200):
    """2-D, 512^2 cells, 64 directions, Voronoi sigma in {1, 1000}, eps = 1e-4."""
    sig = voronoi_two_material(n, n, (1.0, 1000.0), SEED_BASE + 5)
    return _square(f"config5(n={n})", n, nv, 0, 1e-4, steps, sig)


def random_state_2d(nx, ny, nv, seed, m=3, eps=1e-2, T_lo=0.1, T_hi=1.0, anisotropy=0.2, sigma=(0.5, 2.0)):
    """A generic 2-D state with seeded temperature, opacity and inflow (not one
    of the named configurations); E deviates from a T^4 by anisotropy*min(1, eps)."""
    rng = np.random.default_rng(SEED_BASE + 2000 + seed)
    mu, eta, om = circle_pairs(nv)
    P = nv // 2
    T = rng.uniform(T_lo, T_hi, (ny, nx))
    dev = anisotropy * min(1.0, eps)
    E = (T ** 4)[:, :, None] * (1.0 + dev * rng.uniform(-1, 1, (ny, nx, P)))
    osc = (T ** 4).max() * dev / max(eps, 1e-300) * min(1.0, eps)
    Ox = osc * rng.uniform(-1, 1, (ny, nx + 1, P))
    Oy = osc * rng.uniform(-1, 1, (ny + 1, nx, P))
    sig = rng.uniform(sigma[0], sigma[1], (ny, nx))
    b = rng.uniform(0.0, 1.0, (4, P))
    return Workload2D(name=f"random2d({seed})", nx=nx, ny=ny, nv=nv, m=m, eps=eps, dt=0.5 / max(nx, ny),
                      steps=1, mu=mu, eta=eta, omega=om, sigma0=sig, T=T, E=E, Ox=Ox, Oy=Oy, b=b)
