"""The discrete diffusion limit on the GPU (grte_diff_*) against the oracle
(oracle/diffusion1d.py): the three-stage scheme (2.7)/(2.9) in every variant
and the two-stage counter-example (2.8).

  * one step from seeded states, both opacity laws, both boundary kinds, both
    correction fluxes for sigma0/T^3, a_time = 0, ragged sizes up to 4096:
    T and U* within 1e-12 (relative to the largest value) of the oracle;
  * a 50-step trajectory within 1e-10;
  * the front: from compactly supported data the three-stage scheme spreads the
    support, the two-stage scheme leaves it where it was (remark after (2.8));
  * porous-medium limit (a_time = 0): the GPU scheme converges to the
    Barenblatt closed form under refinement;
  * the limit of the alternative correction (3.14): one step against the
    oracle, and its properties -- total energy sum(a T^4 + Cv T) drifts where the
    three-stage scheme keeps it to rounding; on the cold-start front with a hot
    boundary it blows up at the hyperbolic time step (conditional stability)
    where the three-stage scheme stays positive.
"""
import numpy as np
import pytest

from oracle.diffusion1d import barenblatt, semi_cor_step, three_stage_step, two_stage_step
from paper_1811_05579_amd import GrteDiff

pytestmark = pytest.mark.gpu


def _rel(x, y):
    return float(np.max(np.abs(x - y)) / np.max(np.abs(y)))


def _state(N, seed):
    """Smooth seeded temperature (a few sines) and rough opacity.  (With
    per-cell random temperatures and the (U*)^{3/4} correction flux the
    correction can ask a cell for more energy than it has: a c T^4 + Cv T = rhs
    then has no real root, and both implementations report it.)"""
    rng = np.random.default_rng(18110000 + 700 + seed)
    x = (np.arange(N) + 0.5) / N
    T = 0.55 + sum(rng.uniform(-0.12, 0.12) * np.sin(2 * np.pi * (k + 1) * x + rng.uniform(0, 6.3))
                   for k in range(3))
    sigma0 = rng.uniform(0.3, 3.0, N)
    return T, sigma0


CASES = [  # (N, m, bc, corr_K, a_time, scheme)
    (2, 0, "neumann", "old", None, 0), (37, 0, "dirichlet", "old", None, 0),
    (256, 3, "dirichlet", "old", None, 0), (257, 3, "dirichlet", "predicted", None, 0),
    (1000, 3, "neumann", "predicted", None, 0), (513, 0, "neumann", "old", 0.0, 0),
    (700, 3, "dirichlet", "old", 0.0, 0), (4096, 3, "dirichlet", "old", None, 0),
    (300, 0, "dirichlet", "old", None, 1), (129, 3, "neumann", "old", None, 1),
    (333, 0, "dirichlet", "old", None, 2), (2048, 3, "neumann", "old", None, 2),
]


@pytest.mark.parametrize("N,m,bc,ck,at,scheme", CASES)
def test_one_step_matches_oracle(N, m, bc, ck, at, scheme):
    T, sigma0 = _state(N, N + m)
    ghost = (1.0, 0.1)
    dt = 0.5 / N
    g = GrteDiff(N, opacity_law=m, boundary=bc, ghost=ghost)
    g.set_opacity(sigma0)
    g.set_state(T)
    info = g.step(dt, scheme=scheme, corr_K=ck, a_time=at, info=True)
    assert info["status"] == 0
    Tg, Ug = g.get_state()
    if scheme == 0:
        To, Uo = three_stage_step(T, sigma0, dt, m=m, a_time=at, bc=bc, ghost_T=ghost, corr_K=ck)
        assert _rel(Ug, Uo) <= 1e-12
    elif scheme == 1:
        To = two_stage_step(T, sigma0, dt, m=m, bc=bc, ghost_T=ghost)
    else:
        To, Uo = semi_cor_step(T, sigma0, dt, m=m, bc=bc, ghost_T=ghost)
        assert _rel(Ug, Uo) <= 1e-12
    assert _rel(Tg, To) <= 1e-12
    g.close()


def test_trajectory_matches_oracle():
    N, m = 200, 3
    T, sigma0 = _state(N, 5)
    dt = 0.5 / N
    g = GrteDiff(N, opacity_law=m, boundary="dirichlet", ghost=(1.0, 0.0))
    g.set_opacity(sigma0)
    g.set_state(T)
    for _ in range(50):
        T = three_stage_step(T, sigma0, dt, m=m, bc="dirichlet", ghost_T=(1.0, 0.0))[0]
        g.step(dt)
    assert _rel(g.get_state()[0], T) <= 1e-10
    g.close()


def test_three_stage_moves_the_front_two_stage_does_not():
    N = 200
    x = (np.arange(N) + 0.5) / N
    T0 = np.where(np.abs(x - 0.5) < 0.1, 1.0, 0.0)
    supports = []
    for scheme in (GrteDiff.THREE_STAGE, GrteDiff.TWO_STAGE):
        g = GrteDiff(N, opacity_law=0)
        g.set_opacity(np.ones(N))
        g.set_state(T0)
        for _ in range(20):
            g.step(0.5 / N, scheme=scheme)
        T = g.get_state()[0]
        supports.append(int(np.count_nonzero(T > 0)))
        g.close()
    assert supports[0] > np.count_nonzero(T0) + 10
    assert supports[1] == np.count_nonzero(T0)


def test_porous_medium_limit_converges_to_barenblatt():
    q, D, Cb, t0, t1 = 4, 1.0 / 3.0, 0.05, 0.01, 0.05
    errs = []
    for N in (50, 100, 200):
        x = (np.arange(N) + 0.5) / N
        g = GrteDiff(N, opacity_law=0)
        g.set_opacity(np.ones(N))
        g.set_state(barenblatt(x, t0, q, D, Cb))
        dt = 0.1 / N
        steps = int(round((t1 - t0) / dt))
        for _ in range(steps):
            g.step(dt, a_time=0.0)
        T = g.get_state()[0]
        errs.append(np.sum(np.abs(T - barenblatt(x, t0 + steps * dt, q, D, Cb))) / N)
        g.close()
    assert errs[0] > errs[1] > errs[2] and errs[2] < 5e-3



@pytest.mark.parametrize("m", [0, 3])
def test_semi_cor_limit_is_not_energy_conservative(m):
    """Closed ends: sum(a T^4 + Cv T) is kept to rounding by the three-stage
    scheme and drifts with the (3.14) limit (its update conserves the sum with
    U* in place of (T^{n+1})^4), as the paper states."""
    N = 400
    T, sigma0 = _state(N, 40 + m)
    dt = 0.5 / N
    res = {}
    for scheme in (0, 2):
        g = GrteDiff(N, opacity_law=m, boundary="neumann")
        g.set_opacity(sigma0)
        g.set_state(T)
        for _ in range(20):
            g.step(dt, scheme=scheme)
        Tg = g.get_state()[0]
        g.close()
        res[scheme] = abs(np.sum(Tg ** 4 + Tg) - np.sum(T ** 4 + T)) / np.sum(T ** 4 + T)
    assert res[0] < 1e-13 and res[2] > 1e-6, res


def test_semi_cor_limit_blows_up_on_the_front_at_the_hyperbolic_step():
    """Cold start (T = 0.01), hot boundary (ghost T = 1), sigma = 1, dt = 0.5 dx:
    the (3.14) limit loses positivity and overflows within a few steps (its T
    update is explicit in the flux of U*), the three-stage scheme does not."""
    N = 100
    dt = 0.5 / N
    out = {}
    for scheme in (0, 2):
        g = GrteDiff(N, opacity_law=0, boundary="dirichlet", ghost=(1.0, 0.01))
        g.set_opacity(np.ones(N))
        g.set_state(np.full(N, 0.01))
        ok = True
        for _ in range(20):
            g.step(dt, scheme=scheme)
            Tg = g.get_state()[0]
            if not np.all(np.isfinite(Tg)) or Tg.min() < 0:
                ok = False
                break
        g.close()
        out[scheme] = ok
    assert out[0] and not out[2], out
