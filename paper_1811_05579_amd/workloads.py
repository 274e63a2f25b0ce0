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

  marshak   dimensional Marshak wave of the paper's last example: eps = 1,
            c = 29.98 cm/ns, a = 0.01372 GJ/(cm^3 keV^4), Cv = 0.3 GJ/(cm^3 keV),
            sigma = 300 / T^3 cm^-1, x in [0, 0.02] cm, T(x, 0) =
            (1 - tanh((x - 0.0024) 1000)) / 2 keV in equilibrium (I = a c T^4),
            T = 1 keV at x = 0 imposed as the isotropic inflow a c 1^4, the
            right-end inflow a c T(0.02, 0)^4; dt in ns (1.6e-12 s = 1.6e-3 ns).

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
