"""ctypes declarations of the C ABI in include/grte.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrte.so")

c_int, c_double, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
c_double_p = ctypes.POINTER(ctypes.c_double)

GRTE_OK = 0
STATUS = {0: "GRTE_OK", -1: "GRTE_E_INVAL", -2: "GRTE_E_NOMEM", -3: "GRTE_E_HIP",
          -4: "GRTE_E_NOCONV", -5: "GRTE_E_UNSUPPORTED"}
STAGES = {"E_star": 0, "O_star": 1, "U_star": 2, "D": 3, "rho": 4}
TIMING = {"step": 0, "predict": 1}


class Problem(ctypes.Structure):
    _fields_ = [("nx", c_int), ("npairs", c_int), ("length", c_double), ("a", c_double),
                ("c", c_double), ("cv", c_double), ("opacity_law", c_int)]


class StepInfo(ctypes.Structure):
    _fields_ = [("pred_iters", c_int), ("pred_converged", c_int), ("newton_max_iters", c_int),
                ("newton_failed", c_int), ("kstar_clamped", c_int), ("negative_root", c_int),
                ("sync_error", c_int), ("guess_accepted", c_int), ("guess_rejected", c_int),
                ("newton_total_iters", c_int), ("guess_started", c_int), ("pred_floor_stop", c_int),
                ("energy_before", c_double), ("energy_after", c_double), ("boundary_flux_dt", c_double),
                ("energy_defect", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ERRF = {"sync": 1, "pred_noconv": 2, "newton": 4, "negative_root": 8}


class Instance(ctypes.Structure):
    _fields_ = [("nx", c_int), ("npairs", c_int), ("opacity_law", c_int), ("length", c_double),
                ("a", c_double), ("c", c_double), ("cv", c_double), ("dt", c_double),
                ("eps", c_double)]


class DiffProblem(ctypes.Structure):
    _fields_ = [("nx", c_int), ("length", c_double), ("a", c_double), ("c", c_double), ("cv", c_double),
                ("opacity_law", c_int), ("boundary", c_int), ("ghost_left", c_double),
                ("ghost_right", c_double)]


class ReferenceInfo(ctypes.Structure):
    _fields_ = [("picard_iters", c_int), ("converged", c_int), ("pred_max_iters", c_int),
                ("pred_failed", c_int), ("sync_error", c_int)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("pred_iters", c_int), ("pred_converged", c_int), ("newton_max_iters", c_int),
                ("newton_failed", c_int), ("kstar_clamped", c_int), ("negative_root", c_int),
                ("pred_floor_stop", c_int), ("energy_before", c_double), ("energy_after", c_double),
                ("boundary_flux_dt", c_double), ("energy_defect", c_double)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("wave_max_n", c_int), ("grid", c_int), ("step_ms", c_double)]


class Problem2D(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("npairs", c_int), ("lx", c_double), ("ly", c_double),
                ("a", c_double), ("c", c_double), ("cv", c_double), ("opacity_law", c_int)]


class StepInfo2D(ctypes.Structure):
    _fields_ = [("pred_iters", c_int), ("pred_converged", c_int), ("pred_residual", c_double),
                ("corr_iters", c_int), ("corr_converged", c_int), ("corr_residual", c_double),
                ("newton_max_iters", c_int), ("newton_failed", c_int), ("kstar_clamped", c_int),
                ("negative_root", c_int), ("newton_total_iters", c_int), ("guess_accepted", c_int),
                ("guess_rejected", c_int), ("guess_started", c_int), ("pred_floor_stop", c_int),
                ("corr_floor_stop", c_int), ("energy_before", c_double), ("energy_after", c_double),
                ("boundary_flux_dt", c_double), ("energy_defect", c_double), ("pred_narrow", c_int),
                ("corr_narrow", c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


STAGES2D = {"E_star": 0, "U_star": 1, "D": 2, "rho_n": 3}

c_ll_p = ctypes.POINTER(ctypes.c_longlong)

_SIGS = {
    "grte_gauss_legendre": (c_int, [c_int, c_void_p, c_void_p]),
    "grte_create": (c_int, [ctypes.POINTER(Problem), c_void_p, c_void_p, ctypes.POINTER(c_void_p)]),
    "grte_destroy": (c_int, [c_void_p]),
    "grte_set_stream": (c_int, [c_void_p, c_void_p]),
    "grte_set_opacity": (c_int, [c_void_p, c_void_p, c_int]),
    "grte_set_inflow": (c_int, [c_void_p, c_void_p, c_void_p]),
    "grte_set_state": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    "grte_get_state": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    "grte_step": (c_int, [c_void_p, c_double, c_double, ctypes.POINTER(StepInfo)]),
    "grte_step_group": (c_int, [ctypes.POINTER(c_void_p), c_int, c_void_p, c_void_p,
                                ctypes.POINTER(StepInfo)]),
    "grte_get_stage": (c_int, [c_void_p, c_int, c_void_p, c_int]),
    "grte_get_intensity": (c_int, [c_void_p, c_double, c_void_p, c_int]),
    "grte_set_solver": (c_int, [c_void_p, c_double, c_int, c_int]),
    "grte_set_acceleration": (c_int, [c_void_p, c_int]),
    "grte_get_pred_history": (c_int, [c_void_p, c_void_p, c_int, c_void_p]),
    "grte_set_profiling": (c_int, [c_void_p, c_int]),
    "grte_read_timing": (c_int, [c_void_p, c_void_p, c_void_p]),
    "grte_status_string": (ctypes.c_char_p, [c_int]),
    "grte_mlp_create": (c_int, [ctypes.POINTER(c_void_p)]),
    "grte_mlp_destroy": (c_int, [c_void_p]),
    "grte_mlp_set_stream": (c_int, [c_void_p, c_void_p]),
    "grte_mlp_set_params": (c_int, [c_void_p, c_void_p]),
    "grte_mlp_get_params": (c_int, [c_void_p, c_void_p, c_void_p]),
    "grte_mlp_set_norm": (c_int, [c_void_p, c_void_p]),
    "grte_mlp_get_norm": (c_int, [c_void_p, c_void_p]),
    "grte_mlp_fit_norm": (c_int, [c_void_p, c_void_p, ctypes.c_longlong]),
    "grte_mlp_grad": (c_int, [c_void_p, c_void_p, ctypes.c_longlong, c_void_p, c_void_p]),
    "grte_mlp_train": (c_int, [c_void_p, c_void_p, ctypes.c_longlong, c_int, c_int, ctypes.c_float,
                               c_void_p]),
    "grte_mlp_predict": (c_int, [c_void_p, c_void_p, ctypes.c_longlong, c_void_p]),
    "grte_mlp_train_noalloc": (c_int, [c_void_p, c_void_p, ctypes.c_longlong, c_int, c_int, ctypes.c_float,
                                       c_void_p]),
    "grte_set_guess": (c_int, [c_void_p, c_void_p, c_double]),
    "grte_set_storage": (c_int, [c_void_p, c_int]),
    "grte_set_launch": (c_int, [c_void_p, c_int]),
    "grte_get_error_flags": (c_int, [c_void_p, ctypes.POINTER(c_int), c_int]),
    "grte_set_correction": (c_int, [c_void_p, c_int]),
    "grte_batch_get_error_flags": (c_int, [c_void_p, ctypes.POINTER(c_int), c_int]),
    "grte_reference_step": (c_int, [c_void_p, c_double, c_double, c_double, c_int,
                                    ctypes.POINTER(ReferenceInfo)]),
    "grte_log_pairs": (c_int, [c_void_p, c_void_p, ctypes.c_longlong, ctypes.POINTER(ctypes.c_longlong)]),
    "grte_diff_create": (c_int, [ctypes.POINTER(DiffProblem), ctypes.POINTER(c_void_p)]),
    "grte_diff_destroy": (c_int, [c_void_p]),
    "grte_diff_set_stream": (c_int, [c_void_p, c_void_p]),
    "grte_diff_set_opacity": (c_int, [c_void_p, c_void_p, c_int]),
    "grte_diff_set_state": (c_int, [c_void_p, c_void_p, c_int]),
    "grte_diff_get_state": (c_int, [c_void_p, c_void_p, c_void_p, c_int]),
    "grte_diff_step": (c_int, [c_void_p, c_double, c_int, c_int, c_double, ctypes.POINTER(c_int)]),
    "grte_batch_create": (c_int, [c_int, ctypes.POINTER(Instance), c_void_p, c_void_p,
                                  ctypes.POINTER(c_void_p)]),
    "grte_batch_destroy": (c_int, [c_void_p]),
    "grte_batch_sizes": (c_int, [c_void_p, c_ll_p, c_ll_p, c_ll_p, c_ll_p]),
    "grte_batch_set_stream": (c_int, [c_void_p, c_void_p]),
    "grte_batch_set_solver": (c_int, [c_void_p, c_double, c_int, c_int]),
    "grte_batch_set_acceleration": (c_int, [c_void_p, c_int]),
    "grte_batch_set_storage": (c_int, [c_void_p, c_int]),
    "grte_batch_set_opacity": (c_int, [c_void_p, c_void_p, c_int]),
    "grte_batch_set_inflow": (c_int, [c_void_p, c_void_p, c_void_p]),
    "grte_batch_set_state": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    "grte_batch_get_state": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    "grte_batch_step": (c_int, [c_void_p, ctypes.POINTER(BatchInfo)]),
    "grte_batch_tune": (c_int, [c_void_p, c_int, ctypes.POINTER(BatchTuning)]),
    "grte_batch_set_tuning": (c_int, [c_void_p, ctypes.POINTER(BatchTuning)]),
    "grte_batch_get_tuning": (c_int, [c_void_p, ctypes.POINTER(BatchTuning)]),
    "grte_batch_use_graph": (c_int, [c_void_p, c_int]),
    "grte_batch_set_profiling": (c_int, [c_void_p, c_int]),
    "grte_batch_read_timing": (c_int, [c_void_p, ctypes.POINTER(c_double), ctypes.POINTER(c_int)]),
    "grte_batch_read_timing2": (c_int, [c_void_p, ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                        ctypes.POINTER(c_int)]),
    "grte2d_circle_directions": (c_int, [c_int, c_void_p, c_void_p, c_void_p]),
    "grte2d_create": (c_int, [ctypes.POINTER(Problem2D), c_void_p, c_void_p, c_void_p,
                              ctypes.POINTER(c_void_p)]),
    "grte2d_destroy": (c_int, [c_void_p]),
    "grte2d_set_stream": (c_int, [c_void_p, c_void_p]),
    "grte2d_set_solver": (c_int, [c_void_p, c_double, c_int]),
    "grte2d_set_launch_shape": (c_int, [c_void_p, c_int, c_int]),
    "grte2d_set_krylov_storage": (c_int, [c_void_p, c_int]),
    "grte2d_set_opacity": (c_int, [c_void_p, c_void_p, c_int]),
    "grte2d_set_inflow": (c_int, [c_void_p, c_void_p]),
    "grte2d_set_state": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    "grte2d_get_state": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    "grte2d_step": (c_int, [c_void_p, c_double, c_double, ctypes.POINTER(StepInfo2D)]),
    "grte2d_get_stage": (c_int, [c_void_p, c_int, c_void_p, c_int]),
    "grte2d_get_intensity": (c_int, [c_void_p, c_double, c_void_p, c_int]),
    "grte2d_set_profiling": (c_int, [c_void_p, c_int]),
    "grte2d_set_isotropic_correction": (c_int, [c_void_p, c_int, c_int]),
    "grte2d_set_guess": (c_int, [c_void_p, c_void_p, c_double]),
    "grte2d_set_storage": (c_int, [c_void_p, c_int]),
    "grte2d_log_pairs": (c_int, [c_void_p, c_void_p, ctypes.c_longlong, ctypes.POINTER(ctypes.c_longlong)]),
    "grte2d_read_timing": (c_int, [c_void_p, ctypes.POINTER(c_double), ctypes.POINTER(c_int)]),
}

_lib = None


def load():
    """Load libgrte.so from the package directory; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1811_05579_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class GrteError(RuntimeError):
    def __init__(self, call, status):
        msg = load().grte_status_string(status).decode()
        super().__init__(f"{call} -> {STATUS.get(status, status)} ({msg})")
        self.status = status


def check(call, status):
    if status != GRTE_OK:
        raise GrteError(call, status)
    return status
