"""Parity of the 2-D HIP path (through the C ABI) with the 2-D CPU oracle.

Every case feeds the same seeded state to one GPU step and one oracle step and
compares T, E, O^x, O^y and the stages E*, U*, D element by element: max
|gpu - oracle| / max |oracle| per array within the FP64 bar of fp64_bar.py
(1e-12 up to a c beta = 1e6).  Grids span several 256-thread tiles with a
ragged tail; the pair counts cover 4 to 32 pairs.  At the full size of the
1024 x 1024 workload, where no direct solve is possible, the step is checked
through properties that hold at any size: the conservation identity of the
full step in every cell (normwise: the solves meet a relative tolerance on
the whole grid, so cells far below the grid's largest values carry errors at
that global level), and the scalar equation (4.13) in sampled cells.
"""
import numpy as np
import pytest

from fp64_bar import FLOOR, STIFF, bars, sensitivity, stiffness
from oracle import ap2d
from oracle.ap1d import Physics
from paper_1811_05579_amd import Grte2D, GrteError
from paper_1811_05579_amd.workloads import (Workload2D, circle_pairs, config3, random_state_2d,
                                            voronoi_two_material, _square)

pytestmark = pytest.mark.gpu


def _rel(x, y):
    den = np.max(np.abs(y))
    return float(np.max(np.abs(x - y)) / den) if den > 0 else float(np.max(np.abs(x)))


def _ctx(w):
    g = Grte2D(w.nx, w.ny, w.mu, w.eta, w.omega, lx=w.Lx, ly=w.Ly, a=w.a, c=w.c, cv=w.Cv, opacity_law=w.m)
    g.set_opacity(w.sigma0)
    g.set_inflow(w.b)
    return g


def _ph(w):
    return Physics(a=w.a, c=w.c, Cv=w.Cv, eps=w.eps, dt=w.dt, m=w.m)


def gpu_step(g, w, E, Ox, Oy, T):
    g.set_state(E, Ox, Oy, T)
    info = g.step(w.dt, w.eps, info=True)
    Eg, Oxg, Oyg, Tg = g.get_state()
    return dict(E=Eg, Ox=Oxg, Oy=Oyg, T=Tg, E_star=g.get_stage("E_star"), U_star=g.get_stage("U_star"),
                D=g.get_stage("D"), rho_n=g.get_stage("rho_n")), info


def oracle_step(w, E, Ox, Oy, T):
    grid = ap2d.Grid2D(w.nx, w.ny, w.Lx, w.Ly)
    return ap2d.ap_step(grid, E, Ox, Oy, T, w.sigma0, w.mu, w.eta, w.omega, w.b, _ph(w))


KEYS = ("T", "E", "Ox", "Oy", "E_star", "U_star", "D", "rho_n")


def oracle_with_bars(w, E, Ox, Oy, T, keys=KEYS):
    """The oracle's step and the FP64 bar per array (fp64_bar.py: 1e-12 up to
    a stiffness a c beta of 1e6, above it ten times the oracle's measured
    one-ulp sensitivity)."""
    grid = ap2d.Grid2D(w.nx, w.ny, w.Lx, w.Ly)
    step = lambda E_, X_, Y_, T_, s_: ap2d.ap_step(grid, E_, X_, Y_, T_, s_, w.mu, w.eta, w.omega, w.b, _ph(w))
    if stiffness(w, T) <= STIFF:
        return step(E, Ox, Oy, T, w.sigma0), {k: FLOOR for k in keys}
    o, sens = sensitivity(step, [E, Ox, Oy, T, w.sigma0], keys)
    return o, bars(w, T, keys, sens)


def _compare(w, r, o, T, bar, keys=KEYS):
    errs = {k: _rel(r[k], o[k]) for k in keys}
    print(w.name, f"a c beta {stiffness(w, T):.1e}", {k: f"{v:.2e}/{bar[k]:.0e}" for k, v in errs.items()},
          flush=True)
    for k, e in errs.items():
        assert e <= bar[k], (k, e, bar[k])
    return errs


CASES = [  # nx, ny, nv, m, eps, seed
    (12, 9, 8, 0, 1.0, 1),
    (16, 11, 16, 3, 1e-2, 2),
    (10, 13, 8, 3, 1e-4, 3),
    (20, 14, 32, 0, 1e-3, 4),
    (7, 6, 64, 0, 1e-4, 5),
    (9, 17, 4, 3, 1.0, 6),
    (5, 4, 128, 3, 1e-2, 7),      # 64 pairs: one cell per wavefront
    (37, 29, 8, 0, 1e-2, 8),      # 1073 cells x 4 pairs: 17 tiles, ragged
]


@pytest.mark.parametrize("narrow", [True, False])
@pytest.mark.parametrize("nx,ny,nv,m,eps,seed", CASES)
def test_one_step_matches_oracle(nx, ny, nv, m, eps, seed, narrow):
    """Both storages of the Krylov vectors: binary32 where the solve allows it
    (the default) and binary64 throughout."""
    w = random_state_2d(nx, ny, nv, seed, m=m, eps=eps)
    g = _ctx(w)
    g.set_krylov_storage(narrow)
    r, info = gpu_step(g, w, w.E, w.Ox, w.Oy, w.T)
    g.close()
    assert info["status"] == 0, info
    assert info["pred_converged"] and info["corr_converged"], info
    # the correction's blocks are diagonal: binary32 whenever allowed
    assert info["corr_narrow"] == int(narrow), info
    if not narrow:
        assert info["pred_narrow"] == 0, info
    elif stiffness(w, w.T) < 1e3:
        # the prediction keeps binary64 vectors only where a cell's block inverse
        # is near singular: 1 - g sum_p omega_p / d_p >= 1 / (1 + a c beta) of
        # (4.5c), above 1e-8 on these mild states
        assert info["pred_narrow"] == 1, info
    o, bar = oracle_with_bars(w, w.E, w.Ox, w.Oy, w.T)
    _compare(w, r, o, w.T, bar)


def _two_material(n, nv, sig, eps, seed):
    s = voronoi_two_material(n, n, sig, seed)
    return _square(f"two-material({n}, {nv}, {sig}, {eps:g})", n, nv, 0, eps, 3, s)


@pytest.mark.parametrize("n,nv,sig,eps", [(24, 32, (1.0, 100.0), 1e-3), (16, 64, (1.0, 1000.0), 1e-4)])
def test_cold_start_two_material_steps(n, nv, sig, eps):
    """The workload shape (Voronoi opacity, cold start, hot inflow at x = 0) on a
    small grid: three consecutive steps, each compared from the same state."""
    w = _two_material(n, nv, sig, eps, 18110000 + 3)
    g = _ctx(w)
    E, Ox, Oy, T = w.E, w.Ox, w.Oy, w.T
    for k in range(3):
        r, info = gpu_step(g, w, E, Ox, Oy, T)
        assert info["status"] == 0, info
        o, bar = oracle_with_bars(w, E, Ox, Oy, T)
        _compare(w, r, o, T, bar)
        E, Ox, Oy, T = r["E"], r["Ox"], r["Oy"], r["T"]
    g.close()


@pytest.mark.parametrize("eps", [1.0, 1e-3])
def test_free_streaming_uniform_state(eps):
    """sigma = 0: T unchanged bit for bit; a uniform state whose inflow matches
    on all four edges is a fixed point."""
    nx, ny, nv = 19, 13, 16
    mu, eta, om = circle_pairs(nv)
    P = nv // 2
    rng = np.random.default_rng(7)
    fp, fm = rng.uniform(0.1, 1.0, P), rng.uniform(0.1, 1.0, P)
    E = np.broadcast_to((fp + fm) / 2, (ny, nx, P)).copy()
    Oc = (fp - fm) / (2 * eps)
    Ox = np.broadcast_to(Oc, (ny, nx + 1, P)).copy()
    Oy = np.broadcast_to(Oc, (ny + 1, nx, P)).copy()
    ent = lambda s: np.where(s > 0, fp, fm)
    b = np.stack([ent(mu), ent(-mu), ent(eta), ent(-eta)])
    T = rng.uniform(0.2, 1.0, (ny, nx))
    w = Workload2D(name="free", nx=nx, ny=ny, nv=nv, m=0, eps=eps, dt=0.05, steps=1, mu=mu, eta=eta, omega=om,
                   sigma0=np.zeros((ny, nx)), T=T, E=E, Ox=Ox, Oy=Oy, b=b)
    g = _ctx(w)
    r, info = gpu_step(g, w, E, Ox, Oy, T)
    g.close()
    assert info["status"] == 0, info
    assert np.array_equal(r["T"], T)
    assert _rel(r["E"], E) < 1e-13
    # O^{n+1} = O^n - (c dt / eps) grad E_J when sigma = 0: an error of E_J at the
    # solver's relative tolerance reaches O amplified by c dt / (eps h)
    EJ = np.max(np.abs(E - (T ** 4)[:, :, None])) / eps
    amp = w.c * w.dt / (eps * min(1.0 / nx, 1.0 / ny))
    bar = max(1e-12, 10 * 1e-14 * amp * EJ / np.max(np.abs(Ox)))
    assert _rel(r["Ox"], Ox) < bar and _rel(r["Oy"], Oy) < bar, (bar, _rel(r["Ox"], Ox), _rel(r["Oy"], Oy))


def test_full_size_step_properties():
    """Two steps of the 1024 x 1024, 32-direction two-material workload from its
    cold start: both solves converge, and the outputs satisfy the conservation
    identity of the full step in every cell and (4.13) in sampled cells."""
    w = config3()
    g = _ctx(w)
    E, Ox, Oy, T = w.E, w.Ox, w.Oy, w.T
    c, Cv, eps, dt, a = w.c, w.Cv, w.eps, w.dt, w.a
    dx, dy = w.Lx / w.nx, w.Ly / w.ny
    mu, eta, om = w.mu, w.eta, w.omega
    for k in range(2):
        r, info = gpu_step(g, w, E, Ox, Oy, T)
        print("config3 step", k, info, flush=True)
        assert info["status"] == 0, info
        Dv = lambda X, Y: (((X[:, 1:] - X[:, :-1]) * mu) @ om / dx + ((Y[1:] - Y[:-1]) * eta) @ om / dy)
        D1 = Dv(r["Ox"], r["Oy"])
        Ds = r["D"]
        rho_n, rho1 = E @ om, r["E"] @ om
        dT = r["T"] - T
        lhs = (rho1 - rho_n) / (c * dt) + Cv * dT / dt + Ds
        rhs = (eps ** 2 * (Ds - D1)) / (eps ** 2 + c * w.sigma0 * dt)      # m = 0: K = K* = 1
        scale = (np.abs(rho1 / (c * dt)) + np.abs(rho_n / (c * dt)) + np.abs(Cv * dT / dt)
                 + np.abs(Ds) + np.abs(D1))
        dev = np.abs(lhs - rhs)
        print("identity: max dev", dev.max(), "max scale", scale.max(), flush=True)
        assert dev.max() <= 1e-12 * scale.max()
        # (4.13) in sampled cells, from the stages
        rng = np.random.default_rng(k)
        iy, ix = rng.integers(0, w.ny, 4096), rng.integers(0, w.nx, 4096)
        s0 = w.sigma0[iy, ix]
        Tn, Tk = T[iy, ix], r["T"][iy, ix]
        lin = Cv * (eps ** 2 + c * s0 * dt)
        G = a * c * s0 * dt * Tk ** 4 + lin * (Tk - Tn) - s0 * dt * (r["rho_n"][iy, ix] - c * dt * Ds[iy, ix])
        assert np.max(np.abs(G) / (lin * np.maximum(Tk, 1e-300))) < 1e-13
        # the same sum over the pairs in another order (lane butterfly vs numpy)
        np.testing.assert_allclose(r["rho_n"], rho_n, rtol=1e-13, atol=0)
        assert np.all(r["T"] > 0)
        E, Ox, Oy, T = r["E"], r["Ox"], r["Oy"], r["T"]
    g.close()


U32 = 2.0 ** -24


def test_fp32_storage_round_trip_and_step_against_oracle():
    """Binary32 storage: the stored state is E = a c T^4 + fl32(E - a c T^4) and
    fl32(O); one step from that state equals the oracle's step from it (T at the
    FP64 bar: the arithmetic is binary64), with E and O rounded once more on
    storing (<= 2 u32 of the array's largest deviation)."""
    w = random_state_2d(16, 11, 16, 2, m=3, eps=1e-2)
    g = _ctx(w)
    g.set_storage(True)
    g.set_state(w.E, w.Ox, w.Oy, w.T)
    E, Ox, Oy, T = g.get_state()
    # the library forms a c T^4 as (a c T^2) T^2
    T2 = w.T * w.T
    base = ((w.a * w.c) * T2 * T2)[:, :, None]
    assert np.array_equal(E, base + (w.E - base).astype(np.float32).astype(np.float64))
    assert np.array_equal(Ox, w.Ox.astype(np.float32).astype(np.float64))
    assert np.array_equal(Oy, w.Oy.astype(np.float32).astype(np.float64))
    assert np.array_equal(T, w.T)
    info = g.step(w.dt, w.eps, info=True)
    assert info["status"] == 0, info
    E1, Ox1, Oy1, T1 = g.get_state()
    g.close()
    o, bar = oracle_with_bars(w, E, Ox, Oy, T, keys=("T",))
    assert _rel(T1, o["T"]) <= bar["T"]
    dev = o["E"] - w.a * w.c * (o["T"] ** 4)[:, :, None]
    assert np.max(np.abs(E1 - o["E"])) <= 2 * U32 * np.max(np.abs(dev)) + 1e-12 * np.max(np.abs(o["E"]))
    for k, x in (("Ox", Ox1), ("Oy", Oy1)):
        assert np.max(np.abs(x - o[k])) <= 2 * U32 * np.max(np.abs(o[k])), k


def test_fp32_storage_full_size_against_fp64_storage():
    """Five steps of the 1024 x 1024 workload from its cold start with binary32
    and with binary64 storage: the trajectories stay close (the error the
    stored rounding adds, reported per output)."""
    w = config3()
    res = []
    for f32 in (False, True):
        g = _ctx(w)
        g.set_storage(f32)
        g.set_state(w.E, w.Ox, w.Oy, w.T)
        for _ in range(5):
            info = g.step(w.dt, w.eps, info=True)
            assert info["status"] == 0, info
        res.append(g.get_state())
        g.close()
    (E0, X0, Y0, T0), (E1, X1, Y1, T1) = res
    errs = {"T": _rel(T1, T0), "E": _rel(E1, E0), "Ox": _rel(X1, X0), "Oy": _rel(Y1, Y0),
            "rho": _rel(E1 @ w.omega, E0 @ w.omega)}
    print("config3, 5 steps, binary32 vs binary64 storage:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert errs["T"] < 1e-6 and errs["rho"] < 1e-6
    assert errs["E"] < 1e-5 and errs["Ox"] < 1e-5 and errs["Oy"] < 1e-5


def test_binary32_krylov_full_size_against_binary64_krylov():
    """Three steps of the 1024 x 1024 workload from its cold start with the
    Krylov vectors in binary32 (passes of binary32 iterations inside binary64
    true-residual restarts) and in binary64 throughout: both meet the same
    binary64 residual tolerance, so the states agree to the solves' accuracy
    (many column tiles, 16,384 block partials per inner product summed in one
    launch, several passes per solve)."""
    w = config3()
    res, infos = [], []
    for narrow in (False, True):
        g = _ctx(w)
        g.set_storage(False)
        g.set_krylov_storage(narrow)
        g.set_state(w.E, w.Ox, w.Oy, w.T)
        for _ in range(3):
            info = g.step(w.dt, w.eps, info=True)
            assert info["status"] == 0, info
            assert info["pred_converged"] and info["corr_converged"], info
            assert info["corr_narrow"] == int(narrow), info
        infos.append(info)
        res.append(g.get_state())
        g.close()
    (E0, X0, Y0, T0), (E1, X1, Y1, T1) = res
    errs = {"T": _rel(T1, T0), "E": _rel(E1, E0), "Ox": _rel(X1, X0), "Oy": _rel(Y1, Y0)}
    print("config3, 3 steps, binary32 vs binary64 Krylov vectors:", {k: f"{v:.2e}" for k, v in errs.items()},
          "iterations", [(i["pred_iters"], i["corr_iters"]) for i in infos], flush=True)
    for k, v in errs.items():
        assert v < 1e-10, (k, v)


def test_full_size_one_level_reduction_against_two_levels():
    """On the 1024 x 1024 workload an inner product has 16,384 block partials
    (vector updates) or 4096 (operator products).  By default one block of
    1024 threads sums them all; with a first level of 2048 they are summed by
    blocks of 2048 partials and then one block.  The two steps differ only in
    the order of the binary64 sums, so they agree to the solves' accuracy."""
    w = config3()
    res, infos = [], []
    for shape in (None, (4, 2048)):
        g = _ctx(w)
        if shape is not None:
            g.set_launch_shape(*shape)
        r, info = gpu_step(g, w, w.E, w.Ox, w.Oy, w.T)
        g.close()
        assert info["status"] == 0, info
        assert info["pred_converged"] and info["corr_converged"], info
        res.append(r)
        infos.append(info)
    errs = {k: _rel(res[1][k], res[0][k]) for k in ("T", "E", "Ox", "Oy", "E_star", "D")}
    print("config3, one level vs two levels:", {k: f"{v:.2e}" for k, v in errs.items()},
          "iterations", [(i["pred_iters"], i["corr_iters"]) for i in infos], flush=True)
    for k, v in errs.items():
        assert v < 1e-10, (k, v)


@pytest.mark.parametrize("kind,steps", [("none", 1), ("multigrid", 1), ("multigrid", 2), ("chebyshev", 4)])
def test_isotropic_correction_variants_agree(kind, steps):
    """The isotropic correction only changes the preconditioner: three
    cold-start steps of a two-material grid give the same state with every
    variant (within the solver tolerance's effect) and match the oracle."""
    w = _two_material(40, 32, (1.0, 100.0), 1e-3, 18110000 + 3)
    out = []
    for k, st in (("chebyshev", 19), (kind, steps)):
        g = _ctx(w)
        g.set_isotropic_correction(k, st)
        g.set_state(w.E, w.Ox, w.Oy, w.T)
        for _ in range(3):
            info = g.step(w.dt, w.eps, info=True)
            assert info["status"] == 0, info
        out.append(g.get_state())
        g.close()
    for a, b in zip(out[0], out[1]):
        assert _rel(b, a) < 1e-10


@pytest.mark.parametrize("nx,ny,steps", [(75, 41, 10), (75, 41, 5), (33, 70, 2), (33, 70, 1), (64, 32, 10),
                                         (33, 70, 12), (75, 41, 19), (64, 32, 20), (33, 70, 28)])
def test_tiled_chebyshev_equals_per_step(nx, ny, steps):
    """The isotropic correction's Chebyshev steps in tiled launches (32 x 32
    cells per block plus a halo of the launch's stencil steps, at most 9 per
    launch, chained through the stored iterate and direction) give the
    per-step launches' map to the bit: two steps of an optically thick state
    on grids of whole and ragged tiles leave identical states and iteration
    counts, for one launch (up to 10 steps) and two or three (12 to 28)."""
    w = random_state_2d(nx, ny, 16, 40 + steps, m=0, eps=1e-3, sigma=(1.0, 100.0))
    out = []
    for kind in ("chebyshev", "chebyshev-per-step"):
        g = _ctx(w)
        g.set_isotropic_correction(kind, steps)
        g.set_state(w.E, w.Ox, w.Oy, w.T)
        its = []
        for _ in range(2):
            info = g.step(w.dt, w.eps, info=True)
            assert info["status"] == 0, info
            its.append((info["pred_iters"], info["corr_iters"]))
        out.append((g.get_state(), its))
        g.close()
    print(w.name, steps, "iterations", out[0][1], out[1][1], flush=True)
    assert out[0][1] == out[1][1]
    for a, b in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, b)


def test_step_independent_of_convergence_check_batches():
    """The host reads the convergence flag after batches of iterations sized
    from the previous solve; iterations enqueued past convergence do nothing,
    so a context with that history and a fresh one (batches of eight) take
    the same step from the same state, to the bit."""
    w = _two_material(40, 32, (1.0, 100.0), 1e-3, 18110000 + 3)
    g = _ctx(w)
    g.set_state(w.E, w.Ox, w.Oy, w.T)
    for _ in range(3):
        assert g.step(w.dt, w.eps, info=True)["status"] == 0
    s1 = g.get_state()
    i_hist = g.step(w.dt, w.eps, info=True)
    s_hist = g.get_state()
    g.close()
    f = _ctx(w)
    f.set_state(*s1)
    i_fresh = f.step(w.dt, w.eps, info=True)
    s_fresh = f.get_state()
    f.close()
    assert (i_hist["pred_iters"], i_hist["corr_iters"]) == (i_fresh["pred_iters"], i_fresh["corr_iters"])
    for a, b in zip(s_hist, s_fresh):
        assert np.array_equal(a, b)


def test_isotropic_correction_arguments():
    """Step counts outside 1..64 and unknown kinds are rejected."""
    w = random_state_2d(8, 8, 8, 1)
    g = _ctx(w)
    for steps in (0, 65):
        with pytest.raises(GrteError):
            g.set_isotropic_correction("chebyshev", steps)
    with pytest.raises(ValueError):
        g.set_isotropic_correction("jacobi", 4)
    g.close()


@pytest.mark.parametrize("fp32", [False, True])
def test_intensity_readout_2d(fp32):
    """I(+-Omega_p) at the cell centres from the library equals the oracle's
    readout (E +- eps times the mean of the four face values of O)."""
    w = _two_material(20, 16, (1.0, 100.0), 1e-2, 18110000 + 3)
    g = _ctx(w)
    g.set_storage(fp32)
    g.set_state(w.E, w.Ox, w.Oy, w.T)
    for _ in range(3):
        g.step(w.dt, w.eps)
    E, Ox, Oy, T = g.get_state()
    I = g.get_intensity(w.eps)
    g.close()
    ip, im = ap2d.intensity(E, Ox, Oy, w.eps)
    scale = np.max(np.abs(ip))
    assert np.max(np.abs(I[:, :, :w.P] - ip)) <= 4e-16 * scale
    assert np.max(np.abs(I[:, :, w.P:] - im)) <= 4e-16 * scale


@pytest.mark.parametrize("m", [0, 3])
def test_gpu_step_reaches_the_diffusion_limit(m):
    """The asymptotic-preserving property on the GPU path, at a grid the
    transport oracle cannot reach: a compact bump on 48 x 48 cells with 16
    directions, sigma = 1, zero inflow, dt = 0.1 dx; after six steps the GPU
    solution tends to the 2-D three-stage scheme (2.7)/(2.9) (<mu^2> = 1/2) at
    the rate eps^2."""
    from oracle.diffusion2d import three_stage_step
    n, nv = 48, 16
    mu, eta, om = circle_pairs(nv)
    P = nv // 2
    xc = (np.arange(n) + 0.5) / n
    T0 = np.maximum(1 - 40 * ((xc[None, :] - 0.5) ** 2 + (xc[:, None] - 0.5) ** 2), 0.0)
    diffs = []
    for eps in (1e-2, 1e-3, 1e-4):
        w = Workload2D(name=f"bump({eps:g})", nx=n, ny=n, nv=nv, m=m, eps=eps, dt=0.1 / n, steps=6, mu=mu, eta=eta,
                       omega=om, sigma0=np.ones((n, n)), T=T0.copy(), E=np.repeat((T0 ** 4)[:, :, None], P, 2),
                       Ox=np.zeros((n, n + 1, P)), Oy=np.zeros((n + 1, n, P)), b=np.zeros((4, P)))
        g = _ctx(w)
        g.set_state(w.E, w.Ox, w.Oy, w.T)
        Td = T0.copy()
        for _ in range(6):
            info = g.step(w.dt, eps, info=True)
            assert info["status"] == 0, info
            Td, _ = three_stage_step(Td, np.ones((n, n)), w.dt, m=m, mu2=0.5)
        T = g.get_state()[3]
        g.close()
        diffs.append(float(np.max(np.abs(T - Td))))
    print("max |T_gpu - T_(2.7)|:", diffs, flush=True)
    assert diffs[2] < 1e-5, diffs
    assert diffs[0] / diffs[1] > 50 and diffs[1] / diffs[2] > 50, diffs


@pytest.mark.parametrize("nx,ny,pairs", [
    (2, 2, ([0.6], [0.8], [1.0])),                      # smallest grid, one pair
    (3, 2, ([-0.28, 0.8], [0.96, 0.6], [0.5, 0.5])),    # two user pairs, one with mu < 0
    (2, 5, ([0.6], [0.8], [1.0])),
])
def test_degenerate_sizes_match_oracle(nx, ny, pairs):
    """The smallest grids (every cell an edge cell, corner cells on both kinds of
    edge) and user-supplied direction pairs, P = 1 and 2."""
    mu, eta, om = (np.asarray(x, dtype=np.float64) for x in pairs)
    P = mu.size
    rng = np.random.default_rng(nx * 10 + ny)
    T = rng.uniform(0.3, 1.0, (ny, nx))
    E = (T ** 4)[:, :, None] * rng.uniform(0.9, 1.1, (ny, nx, P))
    Ox = rng.uniform(-0.1, 0.1, (ny, nx + 1, P))
    Oy = rng.uniform(-0.1, 0.1, (ny + 1, nx, P))
    w = Workload2D(name=f"tiny({nx}x{ny}, P={P})", nx=nx, ny=ny, nv=2 * P, m=3, eps=1e-2, dt=0.1, steps=1, mu=mu,
                   eta=eta, omega=om, sigma0=rng.uniform(0.5, 2.0, (ny, nx)), T=T, E=E, Ox=Ox, Oy=Oy,
                   b=rng.uniform(0.0, 1.0, (4, P)))
    g = _ctx(w)
    r, info = gpu_step(g, w, E, Ox, Oy, T)
    g.close()
    assert info["status"] == 0, info
    o, bar = oracle_with_bars(w, E, Ox, Oy, T)
    _compare(w, r, o, T, bar)


def test_iteration_cap_holds_for_the_whole_solve():
    """With a cap of 5 Krylov iterations the stiff cold-start step stops at the cap
    (over all restarts) and reports that it did not converge."""
    w = _two_material(24, 32, (1.0, 100.0), 1e-3, 18110000 + 3)
    g = _ctx(w)
    g.set_solver(1e-14, 5)
    g.set_state(w.E, w.Ox, w.Oy, w.T)
    first = g.step(w.dt, w.eps, info=True)
    assert first["pred_iters"] <= 5 and first["corr_iters"] <= 5, first
    info = g.step(w.dt, w.eps, info=True)  # the spike step (R15) needs the most iterations
    g.close()
    assert info["pred_iters"] <= 5 and info["corr_iters"] <= 5, info
    assert info["status"] == -4 and not info["pred_converged"], info


@pytest.mark.parametrize("case,shape", [("random", (1, 4)), ("two_material", (1, 2)), ("random", (3, 1))])
def test_many_block_two_level_path_against_oracle(case, shape):
    """A launch shape of one or three items per thread and a first reduction
    level of one to four partials makes these grids run many blocks whose
    partial sums are reduced in two levels (the default shape sums any count
    of partials in one block of 1024 threads); the step still matches the
    oracle and the default shape's step."""
    if case == "random":
        w = random_state_2d(37, 29, 8, 8, m=0, eps=1e-2)
    else:
        w = _two_material(24, 32, (1.0, 100.0), 1e-3, 18110000 + 3)
    ref_g = _ctx(w)
    r_def, _ = gpu_step(ref_g, w, w.E, w.Ox, w.Oy, w.T)
    ref_g.close()
    g = _ctx(w)
    g.set_launch_shape(*shape)
    r, info = gpu_step(g, w, w.E, w.Ox, w.Oy, w.T)
    g.close()
    assert info["status"] == 0, info
    nblk = -(-w.nx * w.ny * w.P // (256 * shape[0]))
    print(f"{w.name}: {nblk} blocks, first level of {shape[1]}", flush=True)
    assert nblk > shape[1]
    o, bar = oracle_with_bars(w, w.E, w.Ox, w.Oy, w.T)
    _compare(w, r, o, w.T, bar)
    for k in ("T", "E", "Ox", "Oy"):
        assert _rel(r[k], r_def[k]) <= 2 * bar[k], k


def test_64x64_two_material_cold_start_against_oracle():
    """The workload shape of the 1024^2 run (two-material Voronoi opacity
    sigma in {1, 100}, eps = 1e-3, 32 directions, cold start, hot inflow) on
    64 x 64 cells: four 32 x 32 tiles of the isotropic correction with their
    halos, 1024 Krylov blocks; one step against the oracle."""
    w = _two_material(64, 32, (1.0, 100.0), 1e-3, 18110000 + 3)
    g = _ctx(w)
    r, info = gpu_step(g, w, w.E, w.Ox, w.Oy, w.T)
    g.close()
    assert info["status"] == 0, info
    o, bar = oracle_with_bars(w, w.E, w.Ox, w.Oy, w.T)
    _compare(w, r, o, w.T, bar)


def test_40x40_two_material_developed_state_against_oracle():
    """The same workload shape on 40 x 40 cells (2 x 2 tiles, ragged): ten GPU
    steps from the cold start (the heated cells of the sigma = 100 material
    are then stiff, a c beta above 1e6), then one GPU step and one oracle
    step from that GPU state."""
    w = _two_material(40, 32, (1.0, 100.0), 1e-3, 18110000 + 3)
    g = _ctx(w)
    g.set_state(w.E, w.Ox, w.Oy, w.T)
    for _ in range(10):
        assert g.step(w.dt, w.eps, info=True)["status"] == 0
    E, Ox, Oy, T = g.get_state()
    r, info = gpu_step(g, w, E, Ox, Oy, T)
    g.close()
    assert info["status"] == 0, info
    o, bar = oracle_with_bars(w, E, Ox, Oy, T)
    _compare(w, r, o, T, bar)
