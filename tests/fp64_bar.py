"""The FP64 bar of one AP step against the oracle, per output array
(max |gpu - oracle| / max |oracle|).

  a c beta <= 1e6   1e-12, the target, for every array.
  a c beta >  1e6   max(1e-12, FACTOR * s), s measured, per array.

a c beta is the stiffness of (4.5c): the ratio between the material coupling
and the net isotropic absorption of an optically thick cell.  Above 1e6 the
step's answer is itself ill-conditioned: the temperature equation (4.13)
balances a c sigma dt T^4 against sigma dt (rho^n - c dt D), D a second
difference of E*, and that balance passes any rounding of its inputs on to
T, E and O amplified.  s is that amplification measured on the oracle: the
largest relative change of the array when every binary64 input of the step
(E^n, O^n, T^n, sigma0) moves by one ulp, up or down at random, over TRIALS
independent draws.  No binary64 computation of the step can be expected
closer to the exact answer than s.  The GPU path rounds its own
intermediates (rho*, D, E*, the node fluxes) once each, which acts like a
further one-ulp perturbation at each stage; FACTOR = 10 covers those stages
and the spread of the random draws.  (On the six stiffest slabs of the
batched ensemble, a c beta 2e9 to 7e9, s reaches 2e-11 in T, 1e-10 in E and
2e-10 in O; the GPU's errors there are 0.2 to 5 times s.)
"""
import numpy as np

STIFF = 1e6
FACTOR = 10.0
TRIALS = 4
FLOOR = 1e-12


def stiffness(w, T, eps=None, dt=None):
    eps = w.eps if eps is None else eps
    dt = w.dt if dt is None else dt
    beta = 4 * w.sigma0 * dt * np.asarray(T) ** (3 - w.m) / (eps ** 2 * w.Cv)
    return float(np.max(w.a * w.c * beta))


def _rel(x, y):
    den = np.max(np.abs(y))
    return float(np.max(np.abs(x - y)) / den) if den > 0 else float(np.max(np.abs(x)))


def sensitivity(step, inputs, keys, trials=TRIALS, seed=0):
    """Run step(*inputs) (a dict of output arrays) and measure, per key, the
    largest relative change of the output when each binary64 input array is
    moved by one ulp up or down at random, over `trials` draws.  Returns
    (the unperturbed output, {key: s})."""
    base = step(*inputs)
    rng = np.random.default_rng(seed)
    worst = {k: 0.0 for k in keys}
    for _ in range(trials):
        pert = [np.nextafter(np.asarray(x, dtype=np.float64),
                             rng.choice([-np.inf, np.inf], size=np.shape(x))) for x in inputs]
        r = step(*pert)
        for k in keys:
            worst[k] = max(worst[k], _rel(r[k], base[k]))
    return base, worst


def bars(w, T, keys, sens=None, eps=None, dt=None):
    """{key: bar}: FLOOR below the stiffness STIFF, else max(FLOOR, FACTOR * s)
    with s from `sens` (required above STIFF)."""
    if stiffness(w, T, eps, dt) <= STIFF:
        return {k: FLOOR for k in keys}
    if sens is None:
        raise ValueError("a stiff state needs the measured sensitivity (fp64_bar.sensitivity)")
    return {k: max(FLOOR, FACTOR * sens[k]) for k in keys}


def fp64_bar(w, T, eps=None, dt=None):
    """The bar of a state below the stiffness STIFF (1e-12); a stiff state has
    per-array bars from its measured sensitivity (bars())."""
    if stiffness(w, T, eps, dt) > STIFF:
        raise ValueError("stiff state: use bars() with the measured sensitivity")
    return FLOOR
