"""The energy balance of the step, formed on the GPU ((3.12)-(3.13)), against
the oracle.

Every step reports E_tot^n and E_tot^{n+1} (E_tot = sum dx (rho / c + Cv T)),
the outflow through the domain's ends over the step (dt sum_p omega_p mu_p
(O*_{N,p} - O*_{0,p}) with the prediction's fluxes, which the correction's
moment equation uses) and the defect E_tot^{n+1} - E_tot^n + outflow -- the
extra term of (3.13), which vanishes with eps.  The oracle's values are the
same sums of the oracle step's own arrays (oracle/energy.py, oracle/ap2d.py);
the bar is 1e-12 of the largest of the three terms (the arrays themselves
agree at the FP64 bar; the sums add no more than a few ulps of the largest
term).  The full-size 2-D case (a multi-block reduction finished by the last
block) checks E_tot^n against numpy's sum of the same input state.
"""
import numpy as np
import pytest

from oracle import ap2d
from oracle.ap1d import Physics, ap_step
from oracle.energy import boundary_flux, total_energy
from paper_1811_05579_amd import Grte, Grte2D, GrteBatch
from paper_1811_05579_amd.workloads import Ensemble, config1, config2, config3, random_state, random_state_2d

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _ph(w, eps=None):
    return Physics(a=w.a, c=w.c, Cv=w.Cv, eps=w.eps if eps is None else eps, dt=w.dt, L=w.L, m=w.m)


def _expect_1d(w, E, O, T, res):
    dx = w.L / w.N
    eb = total_energy(E, T, w.omega, dx, w.c, w.Cv)
    ea = total_energy(res["E"], res["T"], w.omega, dx, w.c, w.Cv)
    fdt = w.dt * boundary_flux(res["O_star"], w.mu, w.omega)
    return eb, ea, fdt


def _check(label, info, eb, ea, fdt):
    scale = max(abs(eb), abs(ea), abs(fdt))
    got = (info["energy_before"], info["energy_after"], info["boundary_flux_dt"], info["energy_defect"])
    want = (eb, ea, fdt, (ea - eb) + fdt)
    errs = [abs(g - x) / scale for g, x in zip(got, want)]
    print(f"[energy] {label} E_n={eb:.6e} E_n+1={ea:.6e} out*dt={fdt:.3e} defect={want[3]:.3e} "
          f"gpu defect={got[3]:.3e} errs=" + " ".join(f"{e:.1e}" for e in errs), flush=True)
    assert max(errs) <= TOL, (label, errs)


def _step_1d(w, E, O, T, eps=None, fp32=False):
    g = Grte(w.N, w.mu, w.omega, length=w.L, a=w.a, c=w.c, cv=w.Cv, opacity_law=w.m)
    g.set_opacity(w.sigma0)
    g.set_inflow(w.bL, w.bR)
    g.set_storage(fp32)
    g.set_state(E, O, T)
    E0, O0, T0 = g.get_state()           # the stored state (rounded when binary32)
    info = g.step(w.dt, w.eps if eps is None else eps, info=True)
    flags = g.error_flags()
    g.close()
    assert info["status"] == 0, info
    assert not any(flags.values()), flags
    return info, E0, O0, T0


@pytest.mark.parametrize("case", ["config1_cold", "config1_developed", "random_m3_eps1e-4", "random_m0_eps1",
                                  "config2_n512_eps1e-2"])
def test_energy_1d_against_oracle(case):
    if case.startswith("config1"):
        w = config1()
        E, O, T = w.E, w.O, w.T
        if case.endswith("developed"):
            for _ in range(30):
                r = ap_step(E, O, T, w.sigma0, w.mu, w.omega, w.bL, w.bR, _ph(w))
                E, O, T = r["E"], r["O"], r["T"]
    elif case == "random_m3_eps1e-4":
        w = random_state(300, 16, seed=7, m=3, eps=1e-4)
        E, O, T = w.E, w.O, w.T
    elif case == "random_m0_eps1":
        w = random_state(257, 8, seed=8, m=0, eps=1.0)
        E, O, T = w.E, w.O, w.T
    else:
        w = config2(eps=1e-2, N=512)
        E, O, T = w.E, w.O, w.T
    info, E0, O0, T0 = _step_1d(w, E, O, T)
    res = ap_step(E0, O0, T0, w.sigma0, w.mu, w.omega, w.bL, w.bR, _ph(w))
    _check(case, info, *_expect_1d(w, E0, O0, T0, res))


def test_energy_1d_binary32_storage():
    """Binary32 storage: the sums are over the stored state before the step and
    the binary64 result of the step (before it is rounded for storage)."""
    w = random_state(400, 32, seed=9, m=3, eps=1e-2)
    info, E0, O0, T0 = _step_1d(w, w.E, w.O, w.T, fp32=True)
    res = ap_step(E0, O0, T0, w.sigma0, w.mu, w.omega, w.bL, w.bR, _ph(w))
    _check("fp32 storage", info, *_expect_1d(w, E0, O0, T0, res))


def test_defect_vanishes_with_eps():
    """(3.13): the defect is eps^2 / (c sigma dt + eps^2) times the change of the
    flux between prediction and correction, so on well-prepared data (a smooth
    equilibrium profile, inflow in equilibrium with the edges, sigma = 1) it
    falls with eps -- by about eps^2 after a few steps -- while the balance
    itself holds at every eps."""
    w = config1()
    N = w.N
    x = (np.arange(N) + 0.5) / N
    rel = []
    for eps in (1e-1, 1e-2, 1e-3):
        T = 0.5 + 0.3 * np.cos(2 * np.pi * x)
        E = np.repeat((w.a * w.c * T ** 4)[:, None], w.P, 1)
        O = np.zeros((N + 1, w.P))
        bL = np.full(w.P, w.a * w.c * 0.8 ** 4)
        g = Grte(N, w.mu, w.omega, length=w.L, a=w.a, c=w.c, cv=w.Cv, opacity_law=0)
        g.set_opacity(np.ones(N))
        g.set_inflow(bL, bL)
        g.set_state(E, O, T)
        for _ in range(6):
            info = g.step(w.dt, eps, info=True)
            assert info["status"] == 0, info
        g.close()
        scale = max(abs(info["energy_before"]), abs(info["energy_after"]), abs(info["boundary_flux_dt"]))
        rel.append(abs(info["energy_defect"]) / scale)
    print("[energy] |defect| / scale after 6 steps at eps = 1e-1, 1e-2, 1e-3:", rel, flush=True)
    assert rel[1] < 0.1 * rel[0] and rel[2] < 0.1 * rel[1], rel


def test_energy_batched_against_oracle():
    ms = []
    for q, (N, nv, m, eps) in enumerate([(2, 2, 0, 1.0), (37, 16, 3, 1e-2), (200, 8, 0, 1e-4),
                                          (300, 32, 3, 1e-3), (513, 16, 0, 1e-1)]):
        w = random_state(N, nv, seed=100 + q, m=m, eps=eps)
        w.dt = 0.5 / N
        ms.append(w)
    ens = Ensemble("energy", ms)
    b = GrteBatch(ens.members)
    pk = ens.packed()
    b.set_opacity(pk["sigma0"])
    b.set_inflow(pk["bL"], pk["bR"])
    b.set_state(pk["E"], pk["O"], pk["T"])
    b.error_flags(clear=True)
    st, infos = b.step(info=True)
    flags = b.error_flags()
    b.close()
    assert st == 0, infos
    assert not any(flags.values()), flags
    for w, inf in zip(ens.members, infos):
        res = ap_step(w.E, w.O, w.T, w.sigma0, w.mu, w.omega, w.bL, w.bR, _ph(w))
        _check(f"batch {w.name} N={w.N} P={w.P}", inf, *_expect_1d(w, w.E, w.O, w.T, res))


def _ctx2d(w):
    g = Grte2D(w.nx, w.ny, w.mu, w.eta, w.omega, lx=w.Lx, ly=w.Ly, a=w.a, c=w.c, cv=w.Cv, opacity_law=w.m)
    g.set_opacity(w.sigma0)
    g.set_inflow(w.b)
    return g


@pytest.mark.parametrize("nx,ny,nv,m,eps,seed", [(12, 9, 8, 0, 1.0, 1), (16, 11, 16, 3, 1e-2, 2),
                                                 (20, 14, 32, 0, 1e-3, 4)])
def test_energy_2d_against_oracle(nx, ny, nv, m, eps, seed):
    w = random_state_2d(nx, ny, nv, seed, m=m, eps=eps)
    g = _ctx2d(w)
    g.set_state(w.E, w.Ox, w.Oy, w.T)
    info = g.step(w.dt, w.eps, info=True)
    g.close()
    assert info["status"] == 0, info
    grid = ap2d.Grid2D(w.nx, w.ny, w.Lx, w.Ly)
    ph = Physics(a=w.a, c=w.c, Cv=w.Cv, eps=w.eps, dt=w.dt, m=w.m)
    r = ap2d.ap_step(grid, w.E, w.Ox, w.Oy, w.T, w.sigma0, w.mu, w.eta, w.omega, w.b, ph)
    eb = ap2d.total_energy(grid, w.E, w.T, w.omega, w.c, w.Cv)
    ea = ap2d.total_energy(grid, r["E"], r["T"], w.omega, w.c, w.Cv)
    fdt = w.dt * ap2d.boundary_outflow(grid, r["Ox_star"], r["Oy_star"], w.mu, w.eta, w.omega)
    _check(f"2-D {nx}x{ny} P={w.P} m={m} eps={eps}", info, eb, ea, fdt)


def test_energy_2d_full_size_reduction():
    """1024 x 1024 cells: the device reduction (1024 blocks, finished by the last
    block) gives E_tot^n of the input state as numpy sums it, and E_tot^{n+1}
    of the returned state.  (The defect of a cold start with a hot inflow is
    not small: the first steps carry the transient of the inflow spike.)"""
    w = config3()
    g = _ctx2d(w)
    g.set_state(w.E, w.Ox, w.Oy, w.T)
    info = g.step(w.dt, w.eps, info=True)
    E1, Ox1, Oy1, T1 = g.get_state()
    g.close()
    assert info["status"] == 0, info
    grid = ap2d.Grid2D(w.nx, w.ny, w.Lx, w.Ly)
    eb = ap2d.total_energy(grid, w.E, w.T, w.omega, w.c, w.Cv)
    ea = ap2d.total_energy(grid, E1, T1, w.omega, w.c, w.Cv)
    print(f"[energy] config3 gpu {info['energy_before']:.15e} {info['energy_after']:.15e} "
          f"numpy {eb:.15e} {ea:.15e} out*dt {info['boundary_flux_dt']:.3e} defect {info['energy_defect']:.3e}",
          flush=True)
    assert abs(info["energy_before"] - eb) <= 1e-13 * abs(eb)
    assert abs(info["energy_after"] - ea) <= 1e-13 * abs(ea)
    assert np.isfinite(info["boundary_flux_dt"]) and np.isfinite(info["energy_defect"])
    assert info["energy_defect"] == (info["energy_after"] - info["energy_before"]) + info["boundary_flux_dt"]
