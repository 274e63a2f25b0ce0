"""MI355X (gfx950) library for the asymptotic-preserving step of the gray
radiative transfer equation (Tang, Wang & Zhang, arXiv 1811.05579, Algorithm 2
and Section 5).

The Python layer only marshals arguments into the C ABI of include/grte.h;
every stage of the step runs in the HIP kernels of csrc/grte.hip (one
slab), csrc/batch.hip (many slabs in one persistent launch) and csrc/ap2d.hip
(a 2-D rectangle).  Arrays may
be numpy arrays (host memory, copied by the library) or torch CUDA tensors
(device memory, borrowed for the call).
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import (BatchInfo, BatchTuning, DiffProblem, GrteError, Instance, Problem, Problem2D, StepInfo,
                   StepInfo2D, check, load)

__all__ = ["Grte", "Grte2D", "GrteBatch", "GrteDiff", "GrteError", "Mlp", "circle_directions",
           "gauss_legendre", "load", "step_group"]


def gauss_legendre(nv):
    """Gauss-Legendre parity pairs computed by the library (host routine)."""
    lib = load()
    P = nv // 2
    mu = np.zeros(P)
    om = np.zeros(P)
    check("grte_gauss_legendre", lib.grte_gauss_legendre(int(nv), mu.ctypes.data, om.ctypes.data))
    return mu, om


def _ptr(x, n, name):
    """(pointer, on_device) for a float64 numpy array or torch tensor of n elements."""
    if hasattr(x, "data_ptr"):
        import torch
        if x.dtype != torch.float64 or not x.is_contiguous() or x.numel() != n:
            raise ValueError(f"{name}: need a contiguous float64 tensor of {n} elements")
        return ctypes.c_void_p(x.data_ptr()), int(x.is_cuda)
    a = np.ascontiguousarray(x, dtype=np.float64)
    if a.size != n:
        raise ValueError(f"{name}: need {n} elements, got {a.size}")
    return a, 0


def _addr(a):
    return a if isinstance(a, ctypes.c_void_p) else ctypes.c_void_p(a.ctypes.data)


class Grte:
    """One AP solver context (owns its device memory)."""

    def __init__(self, nx, mu, omega, length=1.0, a=1.0, c=1.0, cv=1.0, opacity_law=0):
        self._lib = load()
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        omega = np.ascontiguousarray(omega, dtype=np.float64)
        if mu.shape != omega.shape or mu.ndim != 1:
            raise ValueError("mu and omega must be 1-D arrays of equal length")
        self.N, self.P = int(nx), int(mu.size)
        pb = Problem(self.N, self.P, float(length), float(a), float(c), float(cv), int(opacity_law))
        h = ctypes.c_void_p()
        check("grte_create", self._lib.grte_create(ctypes.byref(pb), mu.ctypes.data,
                                                   omega.ctypes.data, ctypes.byref(h)))
        self._h = h
        self._keep = []

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.grte_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        """Use a torch.cuda.Stream (or a raw hipStream_t integer, 0 = null stream)."""
        raw = getattr(stream, "cuda_stream", stream)
        check("grte_set_stream", self._lib.grte_set_stream(self._h, ctypes.c_void_p(int(raw))))

    def set_solver(self, pred_tol=1e-15, pred_maxit=200, newton_maxit=100):
        check("grte_set_solver", self._lib.grte_set_solver(self._h, float(pred_tol), int(pred_maxit),
                                                           int(newton_maxit)))

    def set_acceleration(self, mode):
        """'chebyshev' (default) or 'richardson' for the prediction iteration."""
        modes = {"richardson": 0, "chebyshev": 1}
        if mode not in modes:
            raise ValueError(f"acceleration must be one of {sorted(modes)}")
        check("grte_set_acceleration", self._lib.grte_set_acceleration(self._h, modes[mode]))

    def pred_history(self):
        """max|z| / max|rho| of each update of the last prediction solve."""
        out = np.zeros(1024)
        n = ctypes.c_int(0)
        check("grte_get_pred_history", self._lib.grte_get_pred_history(
            self._h, out.ctypes.data, out.size, ctypes.byref(n)))
        return out[:n.value].copy()

    def set_opacity(self, sigma0):
        p, dev = _ptr(sigma0, self.N, "sigma0")
        check("grte_set_opacity", self._lib.grte_set_opacity(self._h, _addr(p), dev))

    def set_inflow(self, b_left, b_right):
        bl = np.ascontiguousarray(b_left, dtype=np.float64)
        br = np.ascontiguousarray(b_right, dtype=np.float64)
        if bl.size != self.P or br.size != self.P:
            raise ValueError("inflow arrays need P entries")
        check("grte_set_inflow", self._lib.grte_set_inflow(self._h, bl.ctypes.data, br.ctypes.data))

    def set_state(self, E, O, T):
        pe, d1 = _ptr(E, self.N * self.P, "E")
        po, d2 = _ptr(O, (self.N + 1) * self.P, "O")
        pt, d3 = _ptr(T, self.N, "T")
        if not (d1 == d2 == d3):
            raise ValueError("E, O, T must all be host arrays or all device tensors")
        check("grte_set_state", self._lib.grte_set_state(self._h, _addr(pe), _addr(po), _addr(pt), d1))

    def get_state(self, out=None):
        """Return (E (N,P), O (N+1,P), T (N,)) as numpy arrays, or fill the torch
        tensors passed in `out`."""
        if out is not None:
            E, O, T = out
            pe, d = _ptr(E, self.N * self.P, "E")
            po, _ = _ptr(O, (self.N + 1) * self.P, "O")
            pt, _ = _ptr(T, self.N, "T")
            check("grte_get_state", self._lib.grte_get_state(self._h, _addr(pe), _addr(po), _addr(pt), d))
            return out
        E = np.empty((self.N, self.P))
        O = np.empty((self.N + 1, self.P))
        T = np.empty(self.N)
        check("grte_get_state", self._lib.grte_get_state(self._h, E.ctypes.data, O.ctypes.data,
                                                         T.ctypes.data, 0))
        return E, O, T

    def get_stage(self, name):
        n = {"E_star": self.N * self.P, "O_star": (self.N + 1) * self.P}.get(name, self.N)
        out = np.empty(n)
        check("grte_get_stage", self._lib.grte_get_stage(self._h, _lib.STAGES[name], out.ctypes.data, 0))
        if name == "E_star":
            return out.reshape(self.N, self.P)
        if name == "O_star":
            return out.reshape(self.N + 1, self.P)
        return out

    def get_intensity(self, eps):
        """Cell-centre intensities (N, 2P): columns p = I(+mu_p), P + p = I(-mu_p)."""
        out = np.empty((self.N, 2 * self.P))
        check("grte_get_intensity", self._lib.grte_get_intensity(self._h, float(eps), out.ctypes.data, 0))
        return out

    def set_profiling(self, on=True):
        """True or 1: time every step; k >= 2: every k-th step; False or 0: off."""
        k = int(on) if not isinstance(on, bool) else int(on)
        check("grte_set_profiling", self._lib.grte_set_profiling(self._h, k))

    def read_timing(self):
        """{stage: (total_ms, launches)} from the library's HIP events."""
        n = len(_lib.TIMING)
        ms = np.zeros(n)
        cnt = np.zeros(n, dtype=np.int32)
        check("grte_read_timing", self._lib.grte_read_timing(self._h, ms.ctypes.data, cnt.ctypes.data))
        return {k: (float(ms[v]), int(cnt[v])) for k, v in _lib.TIMING.items()}

    def reference_step(self, dt, eps, tol=1e-14, maxit=500):
        """One step of the iterative implicit reference solver (6.6); returns
        its diagnostics (dict with 'status')."""
        inf = _lib.ReferenceInfo()
        st = self._lib.grte_reference_step(self._h, float(dt), float(eps), float(tol), int(maxit),
                                           ctypes.byref(inf))
        if st not in (0, -4):
            check("grte_reference_step", st)
        d = {k: getattr(inf, k) for k, _ in _lib.ReferenceInfo._fields_}
        d["status"] = st
        return d

    def set_launch(self, cooperative=True):
        """Cooperative (default) or ordinary launch of the prediction kernel; the
        ordinary one is faster but assumes no other work holds the device."""
        check("grte_set_launch", self._lib.grte_set_launch(self._h, int(bool(cooperative))))

    def set_storage(self, fp32):
        """Store E (as its deviation from a c T^4) and O in binary32 (True) or
        binary64 (False); arithmetic stays binary64."""
        check("grte_set_storage", self._lib.grte_set_storage(self._h, int(bool(fp32))))

    def set_correction(self, kind="conservative"):
        """Correction stage: 'conservative' (Algorithm 2) or 'alt' (the
        remark's alternative (3.14), grte_set_correction)."""
        kinds = {"conservative": 0, "alt": 1}
        if kind not in kinds:
            raise ValueError(f"correction kind: one of {sorted(kinds)}")
        check("grte_set_correction", self._lib.grte_set_correction(self._h, kinds[kind]))

    def error_flags(self, clear=False):
        """Error flags OR-ed over the steps since the last clear (grte_get_error_flags):
        a dict of booleans keyed by 'sync', 'pred_noconv', 'newton', 'negative_root'."""
        f = ctypes.c_int()
        check("grte_get_error_flags", self._lib.grte_get_error_flags(self._h, ctypes.byref(f), int(bool(clear))))
        return {k: bool(f.value & b) for k, b in _lib.ERRF.items()}

    def set_guess(self, model, accept_tol=1e-10):
        """Learned initial guess for the temperature solve (None: Newton from T^n)."""
        h = model._h if model is not None else None
        check("grte_set_guess", self._lib.grte_set_guess(self._h, h, float(accept_tol)))

    def log_pairs(self, rows):
        """Write the last step's training rows into the float32 CUDA tensor
        `rows` (shape (>= N, 6)); returns the number of rows written."""
        _check_rows(rows, self.N)
        n = ctypes.c_longlong()
        check("grte_log_pairs", self._lib.grte_log_pairs(self._h, ctypes.c_void_p(rows.data_ptr()),
                                                         rows.shape[0], ctypes.byref(n)))
        return int(n.value)

    def step(self, dt, eps, info=False):
        """One AP step.  With info=True, synchronise and return the step
        diagnostics (dict, including 'status'); otherwise only enqueue."""
        if info:
            si = StepInfo()
            st = self._lib.grte_step(self._h, float(dt), float(eps), ctypes.byref(si))
            if st not in (0, -4):
                check("grte_step", st)
            d = si.as_dict()
            d["status"] = st
            return d
        check("grte_step", self._lib.grte_step(self._h, float(dt), float(eps), None))
        return None


def _check_rows(rows, n_min=1):
    import torch
    if (not isinstance(rows, torch.Tensor) or rows.dtype != torch.float32 or not rows.is_cuda
            or rows.dim() != 2 or rows.shape[1] != 6 or not rows.is_contiguous() or rows.shape[0] < n_min):
        raise ValueError("rows: need a contiguous float32 CUDA tensor of shape (n, 6)")


class Mlp:
    """Learned Newton initial guess (5 -> 64 -> 64 -> 1, gelu); parameters and
    training live on the GPU (grte_mlp_*)."""

    N_PARAM = 4609
    N_NORM = 12

    def __init__(self):
        self._lib = load()
        h = ctypes.c_void_p()
        check("grte_mlp_create", self._lib.grte_mlp_create(ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.grte_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        raw = getattr(stream, "cuda_stream", stream)
        check("grte_mlp_set_stream", self._lib.grte_mlp_set_stream(self._h, ctypes.c_void_p(int(raw))))

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.size != self.N_PARAM:
            raise ValueError(f"need {self.N_PARAM} parameters")
        check("grte_mlp_set_params", self._lib.grte_mlp_set_params(self._h, th.ctypes.data))

    def get_params(self):
        """(binary32 master parameters, their bfloat16 bit patterns as uint16)."""
        th = np.empty(self.N_PARAM, dtype=np.float32)
        bf = np.empty(self.N_PARAM, dtype=np.uint16)
        check("grte_mlp_get_params", self._lib.grte_mlp_get_params(self._h, th.ctypes.data, bf.ctypes.data))
        return th, bf

    def set_norm(self, norm):
        nm = np.ascontiguousarray(norm, dtype=np.float32)
        check("grte_mlp_set_norm", self._lib.grte_mlp_set_norm(self._h, nm.ctypes.data))

    def get_norm(self):
        nm = np.empty(self.N_NORM, dtype=np.float32)
        check("grte_mlp_get_norm", self._lib.grte_mlp_get_norm(self._h, nm.ctypes.data))
        return nm

    def fit_norm(self, rows):
        _check_rows(rows, 2)
        check("grte_mlp_fit_norm", self._lib.grte_mlp_fit_norm(self._h, ctypes.c_void_p(rows.data_ptr()),
                                                               rows.shape[0]))

    def grad(self, rows):
        """(loss, gradient) of the mean squared error over all rows."""
        _check_rows(rows)
        g = np.empty(self.N_PARAM, dtype=np.float32)
        loss = ctypes.c_float()
        check("grte_mlp_grad", self._lib.grte_mlp_grad(self._h, ctypes.c_void_p(rows.data_ptr()), rows.shape[0],
                                                       g.ctypes.data, ctypes.byref(loss)))
        return float(loss.value), g

    def train(self, rows, steps, batch=4096, lr=1e-3):
        """Adam steps on minibatches of consecutive rows; returns the loss history."""
        _check_rows(rows)
        hist = np.empty(int(steps), dtype=np.float32)
        check("grte_mlp_train", self._lib.grte_mlp_train(self._h, ctypes.c_void_p(rows.data_ptr()), rows.shape[0],
                                                         int(steps), int(batch), ctypes.c_float(lr),
                                                         hist.ctypes.data))
        return hist

    def train_noalloc(self, rows, steps, batch=4096, lr=1e-3, history=True):
        """The same training through grte_mlp_train_noalloc (no device
        allocation: a fixed workspace, at most 16384 rows per minibatch and
        65536 recorded steps); returns the loss history (None if history=False)."""
        _check_rows(rows)
        hist = np.empty(int(steps), dtype=np.float32) if history else None
        check("grte_mlp_train_noalloc",
              self._lib.grte_mlp_train_noalloc(self._h, ctypes.c_void_p(rows.data_ptr()), rows.shape[0], int(steps),
                                               int(batch), ctypes.c_float(lr),
                                               hist.ctypes.data if history else None))
        return hist

    def predict(self, rows):
        """Network outputs y (float32 CUDA tensor) for the feature columns of rows."""
        import torch
        _check_rows(rows)
        y = torch.empty(rows.shape[0], dtype=torch.float32, device=rows.device)
        check("grte_mlp_predict", self._lib.grte_mlp_predict(self._h, ctypes.c_void_p(rows.data_ptr()),
                                                             rows.shape[0], ctypes.c_void_p(y.data_ptr())))
        return y


def step_group(ctxs, dts, epss, info=False):
    """One AP step of several Grte contexts with one launch of each kernel
    (grte_step_group); ordered on the first context's stream."""
    n = len(ctxs)
    lib = load()
    hs = (ctypes.c_void_p * n)(*[c._h for c in ctxs])
    dt = np.ascontiguousarray(dts, dtype=np.float64)
    ep = np.ascontiguousarray(epss, dtype=np.float64)
    if dt.size != n or ep.size != n:
        raise ValueError("one dt and one eps per context")
    if not info:
        check("grte_step_group", lib.grte_step_group(hs, n, dt.ctypes.data, ep.ctypes.data, None))
        return None
    arr = (StepInfo * n)()
    st = lib.grte_step_group(hs, n, dt.ctypes.data, ep.ctypes.data, arr)
    if st not in (0, -4):
        check("grte_step_group", st)
    out = [a.as_dict() for a in arr]
    for d in out:
        d["status"] = st
    return out


class GrteBatch:
    """Many independent slabs advanced by one persistent launch per step.

    `members` is a sequence of objects with attributes N, P, m, L, a, c, Cv,
    dt, eps, mu, omega (e.g. workloads.Workload); arrays are exchanged in the
    packed layout of include/grte.h (instances concatenated in order)."""

    def __init__(self, members):
        self._lib = load()
        n = len(members)
        arr = (Instance * n)()
        for i, w in enumerate(members):
            arr[i] = Instance(int(w.N), int(w.P), int(w.m), float(w.L), float(w.a), float(w.c),
                              float(w.Cv), float(w.dt), float(w.eps))
        mu = np.ascontiguousarray(np.concatenate([w.mu for w in members]), dtype=np.float64)
        om = np.ascontiguousarray(np.concatenate([w.omega for w in members]), dtype=np.float64)
        h = ctypes.c_void_p()
        check("grte_batch_create", self._lib.grte_batch_create(n, arr, mu.ctypes.data, om.ctypes.data,
                                                               ctypes.byref(h)))
        self._h = h
        self.n = n
        self.Ns = [int(w.N) for w in members]
        self.Ps = [int(w.P) for w in members]
        tot = [ctypes.c_longlong() for _ in range(4)]
        check("grte_batch_sizes", self._lib.grte_batch_sizes(self._h, *[ctypes.byref(t) for t in tot]))
        self.n_cells, self.n_E, self.n_O, self.n_pairs = (int(t.value) for t in tot)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.grte_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        raw = getattr(stream, "cuda_stream", stream)
        check("grte_batch_set_stream", self._lib.grte_batch_set_stream(self._h, ctypes.c_void_p(int(raw))))

    def set_solver(self, pred_tol=1e-15, pred_maxit=200, newton_maxit=100):
        check("grte_batch_set_solver", self._lib.grte_batch_set_solver(
            self._h, float(pred_tol), int(pred_maxit), int(newton_maxit)))

    def set_storage(self, fp32):
        """Binary32 intensity storage (True) or binary64 (False) for every instance."""
        check("grte_batch_set_storage", self._lib.grte_batch_set_storage(self._h, 1 if fp32 else 0))

    def set_acceleration(self, mode):
        """'chebyshev' (default) or 'richardson' for every instance's prediction."""
        modes = {"richardson": 0, "chebyshev": 1}
        if mode not in modes:
            raise ValueError(f"acceleration must be one of {sorted(modes)}")
        check("grte_batch_set_acceleration", self._lib.grte_batch_set_acceleration(self._h, modes[mode]))

    def set_opacity(self, sigma0):
        p, dev = _ptr(sigma0, self.n_cells, "sigma0")
        check("grte_batch_set_opacity", self._lib.grte_batch_set_opacity(self._h, _addr(p), dev))

    def set_inflow(self, b_left, b_right):
        bl = np.ascontiguousarray(b_left, dtype=np.float64)
        br = np.ascontiguousarray(b_right, dtype=np.float64)
        if bl.size != self.n_pairs or br.size != self.n_pairs:
            raise ValueError("inflow arrays need one entry per pair of every instance")
        check("grte_batch_set_inflow", self._lib.grte_batch_set_inflow(self._h, bl.ctypes.data,
                                                                       br.ctypes.data))

    def set_state(self, E, O, T):
        pe, d1 = _ptr(E, self.n_E, "E")
        po, d2 = _ptr(O, self.n_O, "O")
        pt, d3 = _ptr(T, self.n_cells, "T")
        if not (d1 == d2 == d3):
            raise ValueError("E, O, T must all be host arrays or all device tensors")
        check("grte_batch_set_state", self._lib.grte_batch_set_state(self._h, _addr(pe), _addr(po),
                                                                     _addr(pt), d1))

    def get_state(self):
        """Packed (E, O, T) as numpy arrays."""
        E = np.empty(self.n_E)
        O = np.empty(self.n_O)
        T = np.empty(self.n_cells)
        check("grte_batch_get_state", self._lib.grte_batch_get_state(self._h, E.ctypes.data, O.ctypes.data,
                                                                     T.ctypes.data, 0))
        return E, O, T

    def split(self, E, O, T):
        """Per-instance views (E (N,P), O (N+1,P), T (N,)) of packed arrays."""
        out, oe, oo, ot = [], 0, 0, 0
        for N, P in zip(self.Ns, self.Ps):
            out.append((E[oe:oe + N * P].reshape(N, P), O[oo:oo + (N + 1) * P].reshape(N + 1, P),
                        T[ot:ot + N]))
            oe += N * P
            oo += (N + 1) * P
            ot += N
        return out

    def step(self, info=False):
        """One step of every instance; with info=True synchronise and return
        (status, list of per-instance dicts)."""
        if not info:
            check("grte_batch_step", self._lib.grte_batch_step(self._h, None))
            return None
        arr = (BatchInfo * self.n)()
        st = self._lib.grte_batch_step(self._h, arr)
        if st not in (0, -4):
            check("grte_batch_step", st)
        return st, [{k: getattr(a, k) for k, _ in BatchInfo._fields_} for a in arr]

    def error_flags(self, clear=False):
        """Error flags OR-ed over the steps since the last clear (grte_batch_get_error_flags)."""
        f = ctypes.c_int()
        check("grte_batch_get_error_flags",
              self._lib.grte_batch_get_error_flags(self._h, ctypes.byref(f), int(bool(clear))))
        return {k: bool(f.value & b) for k, b in _lib.ERRF.items()}

    def tune(self, trials=2):
        t = BatchTuning()
        check("grte_batch_tune", self._lib.grte_batch_tune(self._h, int(trials), ctypes.byref(t)))
        return {"wave_max_n": t.wave_max_n, "grid": t.grid, "step_ms": t.step_ms}

    def set_tuning(self, wave_max_n, grid):
        t = BatchTuning(int(wave_max_n), int(grid), 0.0)
        check("grte_batch_set_tuning", self._lib.grte_batch_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self):
        t = BatchTuning()
        check("grte_batch_get_tuning", self._lib.grte_batch_get_tuning(self._h, ctypes.byref(t)))
        return {"wave_max_n": t.wave_max_n, "grid": t.grid}

    def use_graph(self, on=True):
        check("grte_batch_use_graph", self._lib.grte_batch_use_graph(self._h, int(bool(on))))

    def set_profiling(self, on=True):
        check("grte_batch_set_profiling", self._lib.grte_batch_set_profiling(self._h, int(bool(on))))

    def read_timing(self):
        ms = ctypes.c_double()
        cnt = ctypes.c_int()
        check("grte_batch_read_timing", self._lib.grte_batch_read_timing(self._h, ctypes.byref(ms),
                                                                         ctypes.byref(cnt)))
        return float(ms.value), int(cnt.value)

    def read_timing2(self):
        """(summed step ms, summed prediction-solve kernel ms, steps) of the
        profiled steps since the last read."""
        ms = ctypes.c_double()
        ks = ctypes.c_double()
        cnt = ctypes.c_int()
        check("grte_batch_read_timing2", self._lib.grte_batch_read_timing2(self._h, ctypes.byref(ms),
                                                                           ctypes.byref(ks), ctypes.byref(cnt)))
        return float(ms.value), float(ks.value), int(cnt.value)


class GrteDiff:
    """Discrete nonlinear diffusion limit: three-stage (2.7)/(2.9) or two-stage
    (2.8) scheme on the GPU (grte_diff_*)."""

    THREE_STAGE, TWO_STAGE = 0, 1

    def __init__(self, nx, length=1.0, a=1.0, c=1.0, cv=1.0, opacity_law=0, boundary="neumann",
                 ghost=(0.0, 0.0)):
        self._lib = load()
        bc = {"neumann": 0, "dirichlet": 1}[boundary]
        pb = DiffProblem(int(nx), float(length), float(a), float(c), float(cv), int(opacity_law), bc,
                         float(ghost[0]), float(ghost[1]))
        h = ctypes.c_void_p()
        check("grte_diff_create", self._lib.grte_diff_create(ctypes.byref(pb), ctypes.byref(h)))
        self._h = h
        self.N = int(nx)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.grte_diff_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_opacity(self, sigma0):
        p, dev = _ptr(sigma0, self.N, "sigma0")
        check("grte_diff_set_opacity", self._lib.grte_diff_set_opacity(self._h, _addr(p), dev))

    def set_state(self, T):
        p, dev = _ptr(T, self.N, "T")
        check("grte_diff_set_state", self._lib.grte_diff_set_state(self._h, _addr(p), dev))

    def get_state(self):
        """(T, U* of the last prediction) as numpy arrays."""
        T = np.empty(self.N)
        U = np.empty(self.N)
        check("grte_diff_get_state", self._lib.grte_diff_get_state(self._h, T.ctypes.data, U.ctypes.data, 0))
        return T, U

    def step(self, dt, scheme=0, corr_K="old", a_time=None, info=False):
        ck = {"old": 0, "predicted": 1}[corr_K]
        at = -1.0 if a_time is None else float(a_time)
        if not info:
            check("grte_diff_step", self._lib.grte_diff_step(self._h, float(dt), int(scheme), ck, at, None))
            return None
        its = ctypes.c_int()
        st = self._lib.grte_diff_step(self._h, float(dt), int(scheme), ck, at, ctypes.byref(its))
        if st not in (0, -4):
            check("grte_diff_step", st)
        return {"status": st, "newton_max_iters": int(its.value)}


def circle_directions(nv):
    """The nv/2 direction pairs of nv equally spaced circle directions, computed
    by the library (host routine): (mu, eta, omega)."""
    lib = load()
    P = nv // 2
    mu, eta, om = np.zeros(P), np.zeros(P), np.zeros(P)
    check("grte2d_circle_directions", lib.grte2d_circle_directions(int(nv), mu.ctypes.data, eta.ctypes.data,
                                                                   om.ctypes.data))
    return mu, eta, om


class Grte2D:
    """AP solver context on a 2-D rectangle (staggered parity: E in the cells,
    O on the x- and y-faces).  Arrays: E (ny, nx, P), Ox (ny, nx+1, P),
    Oy (ny+1, nx, P), T and sigma0 (ny, nx), inflow b (4, P) for the edges
    x = 0, x = lx, y = 0, y = ly."""

    def __init__(self, nx, ny, mu, eta, omega, lx=1.0, ly=1.0, a=1.0, c=1.0, cv=1.0, opacity_law=0):
        self._lib = load()
        mu, eta, omega = (np.ascontiguousarray(x, dtype=np.float64) for x in (mu, eta, omega))
        if not (mu.shape == eta.shape == omega.shape) or mu.ndim != 1:
            raise ValueError("mu, eta and omega must be 1-D arrays of equal length")
        self.nx, self.ny, self.P = int(nx), int(ny), int(mu.size)
        self.N = self.nx * self.ny
        pb = Problem2D(self.nx, self.ny, self.P, float(lx), float(ly), float(a), float(c), float(cv),
                       int(opacity_law))
        h = ctypes.c_void_p()
        check("grte2d_create", self._lib.grte2d_create(ctypes.byref(pb), mu.ctypes.data, eta.ctypes.data,
                                                       omega.ctypes.data, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.grte2d_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sizes(self):
        return (self.N * self.P, self.ny * (self.nx + 1) * self.P, (self.ny + 1) * self.nx * self.P, self.N)

    def set_stream(self, stream):
        raw = getattr(stream, "cuda_stream", stream)
        check("grte2d_set_stream", self._lib.grte2d_set_stream(self._h, ctypes.c_void_p(int(raw))))

    def set_solver(self, tol=1e-14, maxit=2000):
        check("grte2d_set_solver", self._lib.grte2d_set_solver(self._h, float(tol), int(maxit)))

    def set_launch_shape(self, items_per_thread=4, first_level=2048):
        """Krylov kernels' items per thread and the two-level reduction threshold
        (grte2d_set_launch_shape)."""
        check("grte2d_set_launch_shape",
              self._lib.grte2d_set_launch_shape(self._h, int(items_per_thread), int(first_level)))

    def set_krylov_storage(self, narrow=True):
        """Binary32 Krylov vectors where the solve allows them (True, the
        default) or binary64 always (grte2d_set_krylov_storage)."""
        check("grte2d_set_krylov_storage", self._lib.grte2d_set_krylov_storage(self._h, int(bool(narrow))))

    def set_opacity(self, sigma0):
        p, dev = _ptr(sigma0, self.N, "sigma0")
        check("grte2d_set_opacity", self._lib.grte2d_set_opacity(self._h, _addr(p), dev))

    def set_inflow(self, b):
        b = np.ascontiguousarray(b, dtype=np.float64)
        if b.size != 4 * self.P:
            raise ValueError("inflow: need 4 * P values (edges x=0, x=lx, y=0, y=ly)")
        check("grte2d_set_inflow", self._lib.grte2d_set_inflow(self._h, b.ctypes.data))

    def set_state(self, E, Ox, Oy, T):
        nE, nX, nY, nT = self.sizes()
        pe, d1 = _ptr(E, nE, "E")
        px, d2 = _ptr(Ox, nX, "Ox")
        py, d3 = _ptr(Oy, nY, "Oy")
        pt, d4 = _ptr(T, nT, "T")
        if not (d1 == d2 == d3 == d4):
            raise ValueError("E, Ox, Oy, T must all be host arrays or all device tensors")
        check("grte2d_set_state", self._lib.grte2d_set_state(self._h, _addr(pe), _addr(px), _addr(py),
                                                             _addr(pt), d1))

    def get_state(self):
        """(E, Ox, Oy, T) as numpy arrays."""
        E = np.empty((self.ny, self.nx, self.P))
        Ox = np.empty((self.ny, self.nx + 1, self.P))
        Oy = np.empty((self.ny + 1, self.nx, self.P))
        T = np.empty((self.ny, self.nx))
        check("grte2d_get_state", self._lib.grte2d_get_state(self._h, E.ctypes.data, Ox.ctypes.data,
                                                             Oy.ctypes.data, T.ctypes.data, 0))
        return E, Ox, Oy, T

    def set_storage(self, fp32):
        """Store E (as its deviation from a c T^4), O^x and O^y in binary32 (True) or
        binary64 (False) between steps; arithmetic stays binary64."""
        check("grte2d_set_storage", self._lib.grte2d_set_storage(self._h, int(bool(fp32))))

    def set_guess(self, model, accept_tol=1e-10):
        """Learned initial guess for the temperature solve (None: Newton from T^n)."""
        h = model._h if model is not None else None
        check("grte2d_set_guess", self._lib.grte2d_set_guess(self._h, h, float(accept_tol)))

    def log_pairs(self, rows):
        """Write the last step's training rows into the float32 CUDA tensor `rows`
        (shape (>= nx*ny, 6)); returns the number of rows written."""
        _check_rows(rows, self.N)
        n = ctypes.c_longlong()
        check("grte2d_log_pairs", self._lib.grte2d_log_pairs(self._h, ctypes.c_void_p(rows.data_ptr()),
                                                             rows.shape[0], ctypes.byref(n)))
        return int(n.value)

    def set_isotropic_correction(self, kind="chebyshev", steps=None):
        """The prediction preconditioner's isotropic (diffusion) correction:
        'none', 'chebyshev' (steps: Chebyshev steps, default 19), 'multigrid'
        (steps: Jacobi sweeps before and after each coarse correction, default 2)
        or 'chebyshev-per-step' (the same map as 'chebyshev', one launch per step)."""
        kinds = {"none": 0, "chebyshev": 1, "multigrid": 2, "chebyshev-per-step": 3}
        if kind not in kinds:
            raise ValueError(f"kind must be one of {sorted(kinds)}")
        if steps is None:
            steps = 2 if kind == "multigrid" else 19
        check("grte2d_set_isotropic_correction",
              self._lib.grte2d_set_isotropic_correction(self._h, kinds[kind], int(steps)))

    def set_profiling(self, on=True):
        check("grte2d_set_profiling", self._lib.grte2d_set_profiling(self._h, int(bool(on))))

    def read_timing(self):
        """(total ms, launches) of the timed operator-kernel launches."""
        ms, n = ctypes.c_double(), ctypes.c_int()
        check("grte2d_read_timing", self._lib.grte2d_read_timing(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def get_intensity(self, eps):
        """Cell-centre intensities (ny, nx, 2P): [..., p] = I(+Omega_p), [..., P + p] = I(-Omega_p)."""
        out = np.empty((self.ny, self.nx, 2 * self.P))
        check("grte2d_get_intensity", self._lib.grte2d_get_intensity(self._h, float(eps), out.ctypes.data, 0))
        return out

    def get_stage(self, name):
        shape = (self.ny, self.nx, self.P) if name == "E_star" else (self.ny, self.nx)
        out = np.empty(shape)
        check("grte2d_get_stage", self._lib.grte2d_get_stage(self._h, _lib.STAGES2D[name], out.ctypes.data, 0))
        return out

    def step(self, dt, eps, info=False):
        """One AP step; returns the diagnostics (dict with 'status') when info=True.
        The step synchronises its stream either way (convergence checks)."""
        si = StepInfo2D()
        st = self._lib.grte2d_step(self._h, float(dt), float(eps), ctypes.byref(si))
        if st not in (0, -4):
            check("grte2d_step", st)
        if not info:
            if st != 0:
                check("grte2d_step", st)
            return None
        d = si.as_dict()
        d["status"] = st
        return d
