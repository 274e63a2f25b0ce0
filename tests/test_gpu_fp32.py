"""Binary32 storage of the intensity state against the FP64 oracle.

With grte_set_storage(ctx, 1) the stored E is the binary32 deviation from
a c T^4 and O is binary32; all arithmetic and T stay binary64.  The state is
rounded once when stored and once per step, so every output is off by a
small multiple of the binary32 unit roundoff u = 2^-24 of the quantity
rounded (E - a c T^4, O), propagated by one stable step.  Bounds checked
here (max |x - oracle| / max |oracle| per output):

  one step from the same state      T <= 1e-10; E, rho, I, O <= 16 u
  config 1, 200 steps               T, rho <= 1e-9; E, I <= 1e-8; O <= 16 u
  config-2 runs (N = 256), 60 steps T <= 1e-8; E, rho, I, O <= 64 u

(I = E +- eps (O_j + O_{j+1}) / 2 is the cell-centre intensity.)  Storage
round trip: the state read back is exactly a c T^4 + fl32(E - a c T^4) up to
the rounding of that sum.
"""
import numpy as np
import pytest

from oracle.ap1d import Physics, ap_step
from paper_1811_05579_amd import Grte
from paper_1811_05579_amd.workloads import config1, config2, random_state

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


def _rel(x, y):
    return float(np.max(np.abs(x - y)) / np.max(np.abs(y)))


def _ctx(w):
    g = Grte(w.N, w.mu, w.omega, length=w.L, a=w.a, c=w.c, cv=w.Cv, opacity_law=w.m)
    g.set_opacity(w.sigma0)
    g.set_inflow(w.bL, w.bR)
    g.set_storage(True)
    g.set_state(w.E, w.O, w.T)
    return g


def _I(E, O, eps):
    Oc = 0.5 * (O[:-1] + O[1:])
    return np.concatenate([E + eps * Oc, E - eps * Oc], axis=1)


def _ph(w):
    return Physics(a=w.a, c=w.c, Cv=w.Cv, eps=w.eps, dt=w.dt, L=w.L, m=w.m)


def test_storage_round_trip():
    w = random_state(130, 8, seed=4, m=3, eps=1e-2)
    g = _ctx(w)
    E, O, T = g.get_state()
    base = w.a * w.c * (w.T * w.T) * (w.T * w.T)
    Eexp = base[:, None] + (w.E - base[:, None]).astype(np.float32).astype(np.float64)
    assert np.array_equal(T, w.T)
    assert np.max(np.abs(E - Eexp)) <= 2 * np.finfo(float).eps * np.max(np.abs(w.E))
    assert np.array_equal(O, w.O.astype(np.float32).astype(np.float64))
    g.close()


@pytest.mark.parametrize("N,nv,seed,m,eps", [(200, 16, 1, 3, 1e-2), (200, 16, 2, 0, 1.0), (300, 32, 3, 3, 1e-4)])
def test_one_step_against_oracle(N, nv, seed, m, eps):
    w = random_state(N, nv, seed=seed, m=m, eps=eps)
    o = ap_step(w.E, w.O, w.T, w.sigma0, w.mu, w.omega, w.bL, w.bR, _ph(w))
    g = _ctx(w)
    assert g.step(w.dt, w.eps, info=True)["status"] == 0
    E, O, T = g.get_state()
    assert _rel(T, o["T"]) <= 1e-10
    assert _rel(E, o["E"]) <= 16 * U32
    assert _rel(E @ w.omega, o["E"] @ w.omega) <= 16 * U32
    assert _rel(O, o["O"]) <= 16 * U32
    assert _rel(_I(E, O, w.eps), _I(o["E"], o["O"], w.eps)) <= 16 * U32
    g.close()


def test_config1_trajectory_against_oracle():
    w = config1()
    ph = _ph(w)
    E, O, T = w.E, w.O, w.T
    g = _ctx(w)
    for _ in range(200):
        r = ap_step(E, O, T, w.sigma0, w.mu, w.omega, w.bL, w.bR, ph)
        E, O, T = r["E"], r["O"], r["T"]
        g.step(w.dt, w.eps)
    Eg, Og, Tg = g.get_state()
    assert _rel(Tg, T) <= 1e-9
    assert _rel(Eg @ w.omega, E @ w.omega) <= 1e-9
    assert _rel(Eg, E) <= 1e-8
    assert _rel(_I(Eg, Og, w.eps), _I(E, O, w.eps)) <= 1e-8
    assert _rel(Og, O) <= 16 * U32
    g.close()


@pytest.mark.parametrize("eps", [1.0, 1e-2, 1e-4])
def test_config2_runs_against_oracle(eps):
    w = config2(eps=eps, N=256, nv=16)
    ph = _ph(w)
    E, O, T = w.E, w.O, w.T
    g = _ctx(w)
    for _ in range(60):
        r = ap_step(E, O, T, w.sigma0, w.mu, w.omega, w.bL, w.bR, ph)
        E, O, T = r["E"], r["O"], r["T"]
        assert g.step(w.dt, w.eps, info=True)["status"] == 0
    Eg, Og, Tg = g.get_state()
    assert _rel(Tg, T) <= 1e-8
    for x, y in ((Eg, E), (Eg @ w.omega, E @ w.omega), (Og, O), (_I(Eg, Og, w.eps), _I(E, O, w.eps))):
        assert _rel(x, y) <= 64 * U32
    g.close()


# ---------------------------------------------------------------------------
# batched slabs (grte_batch_set_storage)

def _batch32(members):
    from paper_1811_05579_amd import GrteBatch
    from paper_1811_05579_amd.workloads import Ensemble
    ens = Ensemble("fp32", members)
    b = GrteBatch(ens.members)
    pk = ens.packed()
    b.set_opacity(pk["sigma0"])
    b.set_inflow(pk["bL"], pk["bR"])
    b.set_storage(True)
    b.set_state(pk["E"], pk["O"], pk["T"])
    return b, pk


# wavefront tiles (N <= 256) and work-group tiles, both opacity laws, eps 1 .. 1e-4
BATCH_CASES = [(64, 8, 3, 1e-2, 11), (200, 16, 0, 1.0, 12), (300, 32, 3, 1e-4, 13), (1000, 16, 3, 1e-2, 14),
               (37, 4, 0, 1e-2, 15)]


def _batch_members():
    ms = []
    for N, nv, m, eps, seed in BATCH_CASES:
        w = random_state(N, nv, seed=seed, m=m, eps=eps)
        w.dt = 0.5 / N
        ms.append(w)
    return ms


def test_batch_storage_round_trip():
    ms = _batch_members()
    b, pk = _batch32(ms)
    E, O, T = b.get_state()
    assert np.array_equal(T, pk["T"])
    assert np.array_equal(O, pk["O"].astype(np.float32).astype(np.float64))
    for w, (Ei, _, _) in zip(ms, b.split(E, O, T)):
        base = w.a * w.c * (w.T * w.T) * (w.T * w.T)
        Eexp = base[:, None] + (w.E - base[:, None]).astype(np.float32).astype(np.float64)
        assert np.max(np.abs(Ei - Eexp)) <= 2 * np.finfo(float).eps * np.max(np.abs(w.E))
    b.close()


def test_batch_one_step_against_oracle_and_single_path():
    """Every slab of a binary32 batched step against the FP64 oracle (the
    single-slab bounds: T <= 1e-10, E, O <= 16 u) and against the single-slab
    binary32 path from the same stored state (the two compute the same
    binary64 step with different tile partitions, then round once: T within
    1e-11, E and O within 4 u)."""
    ms = _batch_members()
    b, _ = _batch32(ms)
    st, infos = b.step(info=True)
    assert st == 0
    parts = b.split(*b.get_state())
    for w, (Eb, Ob, Tb) in zip(ms, parts):
        o = ap_step(w.E, w.O, w.T, w.sigma0, w.mu, w.omega, w.bL, w.bR, _ph(w))
        assert _rel(Tb, o["T"]) <= 1e-10, w.name
        assert _rel(Eb, o["E"]) <= 16 * U32, w.name
        assert _rel(Ob, o["O"]) <= 16 * U32, w.name
        g = _ctx(w)
        assert g.step(w.dt, w.eps, info=True)["status"] == 0
        Es, Os, Ts = g.get_state()
        g.close()
        assert _rel(Tb, Ts) <= 1e-11, w.name
        assert _rel(Eb, Es) <= 4 * U32, w.name
        assert _rel(Ob, Os) <= 4 * U32, w.name
    b.close()


def test_batch_ensemble_fp32_against_fp64():
    """64 slabs of the batched ensemble, 20 steps with binary32 storage against
    20 steps of the binary64 batched path (itself the oracle's step to the FP64
    bar): per output, max over slabs of the relative error.  Bounds:
    T <= 1e-7, E and the moment rho <= 256 u, O <= 1e-4 (O is the difference of
    two nearly equal intensities over eps; in the stiffest slabs its size is
    ~1e-6 of E's, so its binary32 rounding is relative to that small scale)."""
    from paper_1811_05579_amd import GrteBatch
    from paper_1811_05579_amd.workloads import config4
    ens = config4(n=64)
    pk = ens.packed()
    out = {}
    for fp32 in (False, True):
        b = GrteBatch(ens.members)
        b.set_opacity(pk["sigma0"])
        b.set_inflow(pk["bL"], pk["bR"])
        b.set_storage(fp32)
        b.set_state(pk["E"], pk["O"], pk["T"])
        for _ in range(20):
            st, _ = b.step(info=True)
            assert st == 0
        out[fp32] = b.split(*b.get_state())
        b.close()
    worst = {"T": 0.0, "E": 0.0, "rho": 0.0, "O": 0.0}
    for w, (E1, O1, T1), (E0, O0, T0) in zip(ens.members, out[True], out[False]):
        worst["T"] = max(worst["T"], _rel(T1, T0))
        worst["E"] = max(worst["E"], _rel(E1, E0))
        worst["rho"] = max(worst["rho"], _rel(E1 @ w.omega, E0 @ w.omega))
        worst["O"] = max(worst["O"], _rel(O1, O0))
    print("batched binary32 vs binary64, 20 steps, worst over 64 slabs: "
          + " ".join(f"{k}={v:.1e}" for k, v in worst.items()))
    assert worst["T"] <= 1e-7
    assert worst["E"] <= 256 * U32 and worst["rho"] <= 256 * U32
    assert worst["O"] <= 1e-4
