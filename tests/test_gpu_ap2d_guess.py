"""The learned Newton guess on the 2-D step (the two-material learned-guess
case, at a reduced grid so that the test trains in seconds).

* an unusable network (its guesses worse than T^n by residual) leaves every
  step bit-identical to plain Newton;
* trained on (state, converged T) rows that the 2-D solver itself logged, the
  network lowers the Newton iterations of the same runs, with T equal to the
  plain method's within the 1e-6 relative bound.
"""
import numpy as np
import pytest
import torch

from paper_1811_05579_amd import Grte2D, Mlp
from paper_1811_05579_amd.workloads import _square, mlp_init, voronoi_two_material

pytestmark = pytest.mark.gpu


def _case(n, nv, sig, eps, seed):
    s = voronoi_two_material(n, n, sig, seed)
    return _square(f"two-material({n}, {nv}, {sig}, {eps:g})", n, nv, 0, eps, 1, s)


def _run(w, K, model=None, log=None, tol=1e-10):
    g = Grte2D(w.nx, w.ny, w.mu, w.eta, w.omega, lx=w.Lx, ly=w.Ly, a=w.a, c=w.c, cv=w.Cv, opacity_law=w.m)
    g.set_opacity(w.sigma0)
    g.set_inflow(w.b)
    g.set_state(w.E, w.Ox, w.Oy, w.T)
    if model is not None:
        g.set_guess(model, tol)
    its = started = 0
    buf = torch.empty((w.nx * w.ny, 6), dtype=torch.float32, device="cuda") if log is not None else None
    for _ in range(K):
        d = g.step(w.dt, w.eps, info=True)
        assert d["status"] == 0, d
        its += d["newton_total_iters"]
        started += d["guess_started"] + d["guess_accepted"]
        if log is not None:
            g.log_pairs(buf)
            log.append(buf.clone())
    T = g.get_state()[3]
    g.close()
    return its, started, T


CASES = [(96, 64, (1.0, 1000.0), 1e-4, 18110000 + 5), (96, 32, (1.0, 100.0), 1e-3, 18110000 + 3)]


def test_unusable_guess_falls_back_to_plain_newton():
    w = _case(*CASES[0])
    m = Mlp()
    th = mlp_init().copy()
    th[-1] = 1e30                      # output bias: T^n exp(huge) is not finite
    m.set_params(th)
    m.set_norm(np.array([0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 0, 1], dtype=np.float32))
    its0, _, T0 = _run(w, 6)
    its1, started, T1 = _run(w, 6, model=m)
    assert started == 0
    assert its1 == its0
    assert np.array_equal(T0, T1)
    m.close()


def test_learned_guess_gain_2d():
    K = 30
    logs, plain = [], []
    ws = [_case(*c) for c in CASES]
    for w in ws:
        plain.append(_run(w, K, log=logs))
    rows = torch.cat(logs)
    keep = rows[:, 5] != 0           # cells with sigma0 > 0 and a change of T
    rows = rows[keep]
    perm = torch.randperm(rows.shape[0], generator=torch.Generator().manual_seed(1234)).cuda()
    rows = rows[perm].contiguous()
    m = Mlp()
    m.set_params(mlp_init())
    m.fit_norm(rows)
    losses = []
    for lr in (1e-3, 1e-3, 1e-3, 5e-4, 5e-4, 2e-4, 1e-4, 5e-5):
        losses.append(m.train(rows, steps=1000, batch=4096, lr=lr))
    assert losses[-1][-200:].mean() < 0.01 * losses[0][0]
    for w, (its0, _, T0) in zip(ws, plain):
        its1, started, T1 = _run(w, K, model=m)
        rel = float(np.max(np.abs(T1 - T0) / T0))
        print(w.name, "Newton iterations", its0, "->", its1, "guess used in", started, "cells; T rel", rel,
              flush=True)
        assert rel < 1e-6
        assert its1 <= its0
        assert started > 0
    m.close()
