"""The C-ABI library loads, exports every symbol include/grte.h declares, and
its host-only logic behaves (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grte.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(grte(?:2d)?_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1811_05579_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1811_05579_amd import build
        build.build()
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_1811_05579_amd import _lib
    assert sorted(_lib._SIGS) == _declared()


def _gl_reference(nv, dps=40):
    """Gauss-Legendre pairs by Newton iteration at 40 digits (mpmath)."""
    import mpmath
    mpmath.mp.dps = dps
    xs, ws = [], []
    for k in range(1, nv // 2 + 1):
        x = mpmath.cos(mpmath.pi * (k - mpmath.mpf(1) / 4) / (nv + mpmath.mpf(1) / 2))
        for _ in range(60):
            p = mpmath.legendre(nv, x)
            dp = nv * (x * p - mpmath.legendre(nv - 1, x)) / (x * x - 1)
            x -= p / dp
        dp = nv * (x * mpmath.legendre(nv, x) - mpmath.legendre(nv - 1, x)) / (x * x - 1)
        xs.append(float(x))
        ws.append(float(2 / ((1 - x * x) * dp * dp)))
    return np.array(xs[::-1]), np.array(ws[::-1])


@pytest.mark.parametrize("nv", [2, 8, 16, 32, 64, 128])
def test_gauss_legendre_correctly_rounded(lib, nv):
    P = nv // 2
    mu = np.zeros(P)
    om = np.zeros(P)
    assert lib.grte_gauss_legendre(nv, mu.ctypes.data, om.ctypes.data) == 0
    xe, we = _gl_reference(nv)
    assert np.all(np.abs(mu - xe) <= np.spacing(xe))
    assert np.all(np.abs(om - we) <= np.spacing(we))
    # numpy leggauss (used by the workload generator) agrees to ~1e-11
    x, w = np.polynomial.legendre.leggauss(nv)
    assert np.max(np.abs(w[x > 0] - we) / we) < 1e-10


def test_invalid_arguments_rejected_before_device_work(lib):
    from paper_1811_05579_amd._lib import Problem
    mu = np.array([0.5])
    om = np.array([1.0])
    h = ctypes.c_void_p()
    for pb in (Problem(1, 1, 1.0, 1.0, 1.0, 1.0, 0),      # N < 2
               Problem(8, 1, 1.0, 1.0, 1.0, 1.0, 2),      # opacity law
               Problem(8, 1, -1.0, 1.0, 1.0, 1.0, 0),     # length
               Problem(8, 1, 1.0, 0.0, 1.0, 1.0, 0)):     # a
        assert lib.grte_create(ctypes.byref(pb), mu.ctypes.data, om.ctypes.data, ctypes.byref(h)) == -1
    big = Problem(5000, 1, 1.0, 1.0, 1.0, 1.0, 0)
    assert lib.grte_create(ctypes.byref(big), mu.ctypes.data, om.ctypes.data, ctypes.byref(h)) == -5
    bad_mu = np.array([-0.5])
    ok = Problem(8, 1, 1.0, 1.0, 1.0, 1.0, 0)
    assert lib.grte_create(ctypes.byref(ok), bad_mu.ctypes.data, om.ctypes.data, ctypes.byref(h)) == -1
    assert lib.grte_gauss_legendre(7, mu.ctypes.data, om.ctypes.data) == -1
    assert lib.grte_step(None, 1.0, 1.0, None) == -1
    assert lib.grte_set_acceleration(None, 1) == -1
    assert lib.grte_set_profiling(None, 1) == -1
    assert lib.grte_get_pred_history(None, None, 0, None) == -1
    assert lib.grte_destroy(None) == 0
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.grte_status_string(s)


def test_batch_invalid_arguments_rejected_before_device_work(lib):
    from paper_1811_05579_amd._lib import Instance
    mu = np.array([0.5, 0.5])
    om = np.array([1.0, 1.0])
    h = ctypes.c_void_p()

    def create(*insts):
        arr = (Instance * len(insts))(*insts)
        return lib.grte_batch_create(len(insts), arr, mu.ctypes.data, om.ctypes.data, ctypes.byref(h))

    good = Instance(8, 1, 0, 1.0, 1.0, 1.0, 1.0, 0.01, 1.0)
    assert create(good, Instance(1, 1, 0, 1.0, 1.0, 1.0, 1.0, 0.01, 1.0)) == -1     # N < 2
    assert create(good, Instance(8, 1, 2, 1.0, 1.0, 1.0, 1.0, 0.01, 1.0)) == -1     # opacity law
    assert create(good, Instance(8, 1, 0, 1.0, 1.0, 1.0, 1.0, 0.0, 1.0)) == -1      # dt
    assert create(good, Instance(8, 1, 0, 1.0, 1.0, 1.0, 1.0, 0.01, -1.0)) == -1    # eps
    assert create(good, Instance(4096, 1, 0, 1.0, 1.0, 1.0, 1.0, 0.01, 1.0)) == -5  # N > 2048
    assert lib.grte_batch_create(0, None, mu.ctypes.data, om.ctypes.data, ctypes.byref(h)) == -1
    bad = np.array([0.5, -0.5])
    arr = (Instance * 2)(good, good)
    assert lib.grte_batch_create(2, arr, bad.ctypes.data, om.ctypes.data, ctypes.byref(h)) == -1
    assert lib.grte_batch_step(None, None) == -1
    assert lib.grte_batch_set_acceleration(None, 0) == -1
    assert lib.grte_batch_set_storage(None, 1) == -1
    assert lib.grte_batch_tune(None, 1, None) == -1
    assert lib.grte_batch_destroy(None) == 0


def test_group_step_invalid_arguments(lib):
    from paper_1811_05579_amd._lib import StepInfo
    dt = np.array([0.1])
    ep = np.array([1.0])
    assert lib.grte_step_group(None, 1, dt.ctypes.data, ep.ctypes.data, None) == -1
    hs = (ctypes.c_void_p * 1)(None)
    assert lib.grte_step_group(hs, 1, dt.ctypes.data, ep.ctypes.data, None) == -1
    assert lib.grte_step_group(hs, 0, dt.ctypes.data, ep.ctypes.data, None) == -1
    hs5 = (ctypes.c_void_p * 5)()
    d5 = np.full(5, 0.1)
    assert lib.grte_step_group(hs5, 5, d5.ctypes.data, d5.ctypes.data, None) == -5


def test_diffusion_invalid_arguments(lib):
    from paper_1811_05579_amd._lib import DiffProblem
    h = ctypes.c_void_p()
    for pb in (DiffProblem(1, 1.0, 1.0, 1.0, 1.0, 0, 0, 0.0, 0.0),     # N < 2
               DiffProblem(8, 1.0, 1.0, 1.0, 1.0, 1, 0, 0.0, 0.0),     # opacity law
               DiffProblem(8, 1.0, 1.0, 1.0, 1.0, 0, 2, 0.0, 0.0),     # boundary kind
               DiffProblem(8, 1.0, 1.0, 1.0, 1.0, 0, 1, -1.0, 0.0)):   # ghost T < 0
        assert lib.grte_diff_create(ctypes.byref(pb), ctypes.byref(h)) == -1
    big = DiffProblem(5000, 1.0, 1.0, 1.0, 1.0, 0, 0, 0.0, 0.0)
    assert lib.grte_diff_create(ctypes.byref(big), ctypes.byref(h)) == -5
    assert lib.grte_diff_step(None, 0.1, 0, 0, -1.0, None) == -1
    assert lib.grte_diff_destroy(None) == 0


def test_2d_host_checks(lib):
    """grte2d_* argument checks that return before any device work."""
    from paper_1811_05579_amd._lib import Problem2D
    mu, eta, om = (np.zeros(4) for _ in range(3))
    assert lib.grte2d_circle_directions(8, mu.ctypes.data, eta.ctypes.data, om.ctypes.data) == 0
    for bad in (2, 6, 130):
        assert lib.grte2d_circle_directions(bad, mu.ctypes.data, eta.ctypes.data, om.ctypes.data) == -1
    h = ctypes.c_void_p()
    for nx, ny, P in ((1, 4, 4), (4, 1, 4), (4, 4, 3), (4, 4, 128), (4, 4, 0)):
        pb = Problem2D(nx, ny, P, 1.0, 1.0, 1.0, 1.0, 1.0, 0)
        assert lib.grte2d_create(ctypes.byref(pb), mu.ctypes.data, eta.ctypes.data, om.ctypes.data,
                                 ctypes.byref(h)) == -5
    pb = Problem2D(4, 4, 4, 1.0, 1.0, 1.0, 1.0, 1.0, 2)
    assert lib.grte2d_create(ctypes.byref(pb), mu.ctypes.data, eta.ctypes.data, om.ctypes.data,
                             ctypes.byref(h)) == -1
    # a direction parallel to an edge (eta = 0) or a zero weight is rejected
    pb = Problem2D(4, 4, 4, 1.0, 1.0, 1.0, 1.0, 1.0, 0)
    mu[:], eta[:], om[:] = 0.5, 0.0, 0.25
    assert lib.grte2d_create(ctypes.byref(pb), mu.ctypes.data, eta.ctypes.data, om.ctypes.data,
                             ctypes.byref(h)) == -1
    assert lib.grte2d_create(None, mu.ctypes.data, eta.ctypes.data, om.ctypes.data, ctypes.byref(h)) == -1
    for f in ("grte2d_step",):
        assert getattr(lib, f)(None, 0.1, 0.1, None) == -1
    assert lib.grte2d_set_solver(None, 1e-14, 10) == -1
    assert lib.grte2d_set_inflow(None, None) == -1
    assert lib.grte2d_set_opacity(None, None, 0) == -1
    assert lib.grte2d_get_stage(None, 0, None, 0) == -1
    assert lib.grte2d_get_intensity(None, 1.0, None, 0) == -1
    assert lib.grte_get_intensity(None, 1.0, None, 0) == -1
    for kind in range(4):
        assert lib.grte2d_set_isotropic_correction(None, kind, 10) == -1
    assert lib.grte_set_launch(None, 0) == -1
    assert lib.grte2d_destroy(None) == 0


def test_2d_directions_match_numpy(lib):
    from oracle.quadrature import circle_pairs
    for nv in (4, 8, 32, 64, 128):
        P = nv // 2
        mu, eta, om = np.zeros(P), np.zeros(P), np.zeros(P)
        assert lib.grte2d_circle_directions(nv, mu.ctypes.data, eta.ctypes.data, om.ctypes.data) == 0
        m2, e2, o2 = circle_pairs(nv)
        np.testing.assert_allclose(mu, m2, rtol=0, atol=2.3e-16)
        np.testing.assert_allclose(eta, e2, rtol=0, atol=2.3e-16)
        assert np.array_equal(om, o2)
