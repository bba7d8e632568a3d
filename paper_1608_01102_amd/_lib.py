"""ctypes view of libstfas.so (include/stfas.h, include/stfas_ops.h).

Loads the in-tree HIP library and fails loudly when it is missing: there is
no CPU fallback."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstfas.so")

c_int32, c_int64, c_double, c_size_t, c_void_p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                   ctypes.c_size_t, ctypes.c_void_p)

STFAS_OK, STFAS_E_INVALID, STFAS_E_NOMEM, STFAS_E_DEVICE, STFAS_E_NONFINITE = range(5)
STFAS_FP64, STFAS_MIXED = 0, 1


class StfasProblem(ctypes.Structure):
    _fields_ = [
        ("dim", c_int32), ("n", c_int32 * 3), ("num_steps", c_int32),
        ("dt", c_double), ("r", c_double), ("K", c_double), ("beta", c_double),
        ("ao_iters", c_int32),
        ("eps_stfas", c_double), ("eps_admm", c_double),
        ("max_admm", c_int32), ("max_vcycles", c_int32), ("metric_levels", c_int32),
        ("poisson_rtol", c_double),
        ("fixed_counts", c_int32), ("precision", c_int32),
        ("scgs_omega", c_double),
        ("density_op", c_int32),
        ("al_tol", c_double),
        ("scgs_lm", c_double),
        ("velocity_op", c_int32),
        ("scgs_local", c_int32),
    ]


class StfasStats(ctypes.Structure):
    _fields_ = [
        ("admm_iters", c_int32), ("vcycles", c_int32), ("converged", c_int32),
        ("objective", c_double), ("objective_l2", c_double), ("reg_term", c_double),
        ("kkt_res_inf", c_double), ("visual_diff", c_double), ("seconds", c_double),
        ("multiplier_updates", c_int32),
    ]


class StfasState(ctypes.Structure):
    _fields_ = [("v", c_void_p), ("pbar", c_void_p), ("u", c_void_p), ("p", c_void_p)]


_SIGS = {
    "stfas_workspace_bytes": (c_size_t, [ctypes.POINTER(StfasProblem)]),
    "stfas_create": (c_int32, [ctypes.POINTER(StfasProblem), c_void_p, ctypes.POINTER(c_void_p)]),
    "stfas_create_in": (c_int32, [ctypes.POINTER(StfasProblem), c_void_p, c_void_p, c_size_t,
                                  ctypes.POINTER(c_void_p)]),
    "stfas_solve": (c_int32, [c_void_p, c_void_p, c_int32, ctypes.POINTER(c_int32), c_void_p, c_void_p,
                              ctypes.POINTER(StfasStats)]),
    "stfas_lbfgs": (c_int32, [c_void_p, c_void_p, c_int32, ctypes.POINTER(c_int32), c_void_p, c_void_p,
                              c_int32, ctypes.c_double, ctypes.POINTER(c_int32), ctypes.POINTER(ctypes.c_double)]),
    "stfas_step_forward": (c_int32, [ctypes.POINTER(StfasProblem), c_void_p, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_void_p]),
    "stfas_step_backward": (c_int32, [ctypes.POINTER(StfasProblem), c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "stfas_step_backward_u": (c_int32, [ctypes.POINTER(StfasProblem), c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "stfas_step_forward_noalloc": (c_int32, [ctypes.POINTER(StfasProblem), c_void_p, c_void_p, c_void_p, c_void_p,
                                             c_void_p, c_void_p, c_void_p]),
    "stfas_step_work_bytes": (c_size_t, [ctypes.POINTER(StfasProblem)]),
    "stfas_step_vcycles": (c_int32, [ctypes.POINTER(StfasProblem)]),
    "stfas_destroy": (None, [c_void_p]),
    "stfas_status_string": (ctypes.c_char_p, [c_int32]),
    "stfas_build_info": (ctypes.c_char_p, []),
    "stfas_num_levels": (c_int32, [c_void_p]),
    "stfas_level_cells": (c_int64, [c_void_p, c_int32]),
    "stfas_level_faces": (c_int64, [c_void_p, c_int32]),
    "stfas_op_advect": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "stfas_op_advect_T": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "stfas_op_advect_dv_T": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_double,
                                       c_void_p]),
    "stfas_op_upwind": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_int32)]),
    "stfas_op_upwind_adj": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "stfas_op_self_advect": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "stfas_op_self_advect_T": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_double, c_void_p]),
    "stfas_op_project": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_int32)]),
    "stfas_op_metric": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "stfas_op_kkt_residual": (c_int32, [c_void_p, c_int32, StfasState, c_void_p, StfasState, StfasState]),
    "stfas_op_scgs_sweep": (c_int32, [c_void_p, c_int32, StfasState, c_void_p, StfasState]),
    "stfas_op_restrict": (c_int32, [c_void_p, c_int32, StfasState, StfasState]),
    "stfas_op_prolong": (c_int32, [c_void_p, c_int32, StfasState, c_double, StfasState]),
    "stfas_op_nso": (c_int32, [c_void_p, StfasState, c_void_p, ctypes.POINTER(c_int32), ctypes.POINTER(c_double)]),
    "stfas_op_ao": (c_int32, [c_void_p, c_void_p, c_int32, ctypes.POINTER(c_int32), c_void_p, c_void_p, c_void_p,
                              c_void_p, ctypes.POINTER(c_double)]),
    "stfas_trace_enable": (c_int32, [c_void_p, c_int32, c_int32]),
    "stfas_trace_read": (c_int32, [c_void_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_double),
                                   ctypes.POINTER(c_double), ctypes.POINTER(c_double)]),
}

EXPORTED = tuple(_SIGS)

_lib = None


def load():
    """Load libstfas.so (built by build.py); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1608_01102_amd/build.py "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class StfasError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = load().stfas_status_string(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")


def check(status, where):
    if status != STFAS_OK:
        raise StfasError(status, where)
