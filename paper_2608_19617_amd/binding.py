"""ctypes binding of the C ABI declared in include/lbm.h.

Argument marshalling only: every step of the solver runs in the HIP library.
Importing this module loads liblbmadj.so and fails loudly if it is missing.
"""

import ctypes
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbmadj.so")

LBM_OK, LBM_E_INVALID, LBM_E_NOMEM, LBM_E_HIP, LBM_E_UNSTABLE, LBM_E_STATE = range(6)
LBM_D2Q9, LBM_D3Q19 = 0, 1
LBM_F64, LBM_F32, LBM_F16S = 0, 1, 2
LBM_WALL, LBM_VELOCITY, LBM_PRESSURE = 0, 1, 2
LBM_S_LINEAR, LBM_S_PAPER = 0, 1
LBM_J_PRESSURE_DROP, LBM_J_DISSIPATION_PLUS_DP, LBM_J_DRAG, LBM_J_WAKE = 0, 1, 2, 3

STATUS_NAMES = {0: "LBM_OK", 1: "LBM_E_INVALID", 2: "LBM_E_NOMEM", 3: "LBM_E_HIP",
                4: "LBM_E_UNSTABLE", 5: "LBM_E_STATE"}

EXPORTED = ["lbm_workspace_bytes", "lbm_init", "lbm_set_gamma", "lbm_reset", "lbm_forward",
            "lbm_window_history", "lbm_adjoint", "lbm_adjoint_full", "lbm_window_replay",
            "lbm_set_wake_reference", "lbm_wake_mean_velocity", "lbm_get_state",
            "lbm_set_state", "lbm_get_fields", "lbm_timing", "lbm_set_blocking", "lbm_set_blocking_3d",
            "lbm_set_adjoint_blocking", "lbm_set_adjoint_blocking_3d", "lbm_last_error", "lbm_destroy",
            "lbm_design_workspace_bytes", "lbm_design_init", "lbm_design_map", "lbm_design_chain",
            "lbm_design_update", "lbm_design_destroy", "lbm_design_map_noalloc"]


class lbm_config(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("tau", ctypes.c_double), ("c_smag", ctypes.c_double),
        ("prec", ctypes.c_int), ("s_map", ctypes.c_int), ("s_q", ctypes.c_double),
        ("periodic_x", ctypes.c_int), ("periodic_y", ctypes.c_int), ("periodic_z", ctypes.c_int),
        ("west", ctypes.POINTER(ctypes.c_int)), ("east", ctypes.POINTER(ctypes.c_int)),
        ("u_in", ctypes.POINTER(ctypes.c_double)),
        ("rho_out", ctypes.c_double), ("rho_init", ctypes.c_double), ("u_init_mode", ctypes.c_int),
        ("window_len", ctypes.c_int), ("sample_every", ctypes.c_int), ("max_windows", ctypes.c_int),
        ("eps", ctypes.c_double),
        ("objective", ctypes.c_int), ("monitor", ctypes.c_int),
        ("sec_in_x", ctypes.c_int), ("sec_in_lo", ctypes.c_int), ("sec_in_hi", ctypes.c_int),
        ("sec_out_x", ctypes.c_int), ("sec_out_lo", ctypes.c_int), ("sec_out_hi", ctypes.c_int),
        ("ckpt_every", ctypes.c_int),
        ("full_history", ctypes.c_int),
        ("force_box", ctypes.c_int * 6), ("drag_ref", ctypes.c_double), ("meas_box", ctypes.c_int * 6),
    ]


class lbm_fwd_report(ctypes.Structure):
    _fields_ = [
        ("steps_done", ctypes.c_long), ("windows_done", ctypes.c_int), ("converged", ctypes.c_int),
        ("w_eff", ctypes.c_int), ("J_eff", ctypes.c_double), ("monitor", ctypes.c_double),
        ("rel_change", ctypes.c_double), ("unstable", ctypes.c_int),
    ]


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"HIP library {_LIB_PATH} is missing: build it with "
            "`python -c 'import __graft_entry__; __graft_entry__.build()'` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    D = ctypes.POINTER(ctypes.c_double)
    lib.lbm_workspace_bytes.argtypes = [ctypes.POINTER(lbm_config), ctypes.POINTER(ctypes.c_size_t)]
    lib.lbm_init.argtypes = [ctypes.POINTER(lbm_config), P, P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    lib.lbm_set_gamma.argtypes = [P, P]
    lib.lbm_reset.argtypes = [P]
    lib.lbm_forward.argtypes = [P, ctypes.c_long, ctypes.c_int, ctypes.POINTER(lbm_fwd_report)]
    lib.lbm_window_history.argtypes = [P, D, D, D, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.lbm_adjoint.argtypes = [P, ctypes.c_int, P, D]
    lib.lbm_adjoint_full.argtypes = [P, P, D]
    lib.lbm_window_replay.argtypes = [P, P, D]
    lib.lbm_set_wake_reference.argtypes = [P, P]
    lib.lbm_wake_mean_velocity.argtypes = [P, P]
    lib.lbm_get_state.argtypes = [P, D, ctypes.POINTER(ctypes.c_long)]
    lib.lbm_set_state.argtypes = [P, D, ctypes.c_long]
    lib.lbm_get_fields.argtypes = [P, P]
    lib.lbm_timing.argtypes = [P, ctypes.c_int, D]
    lib.lbm_set_blocking.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.lbm_set_adjoint_blocking.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.lbm_set_blocking_3d.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.lbm_set_adjoint_blocking_3d.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.lbm_last_error.argtypes = []
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_destroy.argtypes = [P]
    lib.lbm_destroy.restype = None
    dbl, i = ctypes.c_double, ctypes.c_int
    lib.lbm_design_workspace_bytes.argtypes = [i, i, i, dbl, ctypes.POINTER(ctypes.c_size_t)]
    lib.lbm_design_init.argtypes = [i, i, i, dbl, P, P, P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    lib.lbm_design_map.argtypes = [P, P, dbl, dbl, P, D]
    lib.lbm_design_chain.argtypes = [P, P, dbl, dbl, P, P, P]
    lib.lbm_design_update.argtypes = [P, P, P, P, dbl, dbl, dbl, dbl, dbl, P, D, D]
    lib.lbm_design_destroy.argtypes = [P]
    lib.lbm_design_map_noalloc.argtypes = [i, i, i, dbl, P, P, P, dbl, dbl, P, P, P]
    lib.lbm_design_destroy.restype = None
    for name in EXPORTED:
        if name not in ("lbm_last_error", "lbm_destroy", "lbm_design_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


lib = _load()


def check(status):
    """Raises LbmError with the library's message for a non-OK status."""
    if status != LBM_OK:
        raise LbmError(status, lib.lbm_last_error().decode())
    return status
