"""ctypes declarations of the C ABI in include/dda.h.

Loading fails loudly when ``libdda.so`` has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdda.so")

DDA_OK = 0
DDA_ERR_INVALID_ARG = -1
DDA_ERR_OOM = -2
DDA_ERR_HIP = -3
DDA_ERR_STATE = -4
DDA_ERR_UNSUPPORTED_DIMS = -5
DDA_ERR_NO_DEVICE = -6
DDA_ERR_IO = -7
DDA_WARN_NOT_CONVERGED = 1
DDA_WARN_MKD_GE_1 = 2

DDA_ALPHA_CM = 0
DDA_ALPHA_CM_RR = 1
DDA_ALPHA_LDR = 2

DDA_FP64 = 1
DDA_FP32 = 2

DDA_SOLVE_FP64 = 0
DDA_SOLVE_FP32_REFINE = 1

DDA_GUESS_ZERO = 0
DDA_GUESS_USER = 1
DDA_GUESS_PREV = 2
DDA_GUESS_NN = 3
DDA_GUESS_PREV_SHIFT = 4
DDA_GUESS_PROJECT = 5

DDA_SOLVER_BICGSTAB = 0
DDA_SOLVER_BICGSTAB2 = 1

DDA_DEVICE_PTRS = 1
DDA_NO_GRAPH = 2
DDA_NO_FALLBACK = 4


class dda_wave(C.Structure):
    _fields_ = [("khat", C.c_double * 3), ("e0", C.c_double * 6), ("target", C.c_int32), ("pad_", C.c_int32)]


class dda_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("guess", C.c_int32), ("prec", C.c_int32),
                ("flags", C.c_uint32), ("graph_iters", C.c_int32), ("history", C.c_int32),
                ("restart_every", C.c_int32), ("solver", C.c_int32)]


class dda_solve_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("matvecs", C.c_int32), ("outer", C.c_int32), ("status", C.c_int32),
                ("rel_resid", C.c_double), ("guess_resid", C.c_double)]


class dda_nn_config(C.Structure):
    _fields_ = [("width", C.c_int32), ("depth", C.c_int32), ("seed", C.c_int32), ("reserved", C.c_int32)]


class dda_nn_train_opts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double), ("weight_decay", C.c_double),
                ("reserved", C.c_int32 * 4)]


# name -> (restype, argtypes); every symbol declared in include/dda.h
P = C.c_void_p
D = C.POINTER(C.c_double)
SIGNATURES = {
    "dda_version": (C.c_char_p, []),
    "dda_create": (C.c_int32, [C.POINTER(P), C.c_int32, P]),
    "dda_destroy": (C.c_int32, [P]),
    "dda_last_error": (C.c_char_p, [P]),
    "dda_set_target": (C.c_int32, [P, C.POINTER(C.c_int32), P, C.c_int32, D, C.c_double, C.c_int32, D]),
    "dda_add_target": (C.c_int32, [P, C.POINTER(C.c_int32), P, C.c_int32, D, C.c_double, C.c_int32, D,
                                   C.POINTER(C.c_int32)]),
    "dda_target_info": (C.c_int32, [P, C.c_int32, C.POINTER(C.c_int64), D]),
    "dda_build_green_fft": (C.c_int32, [P, C.c_uint32]),
    "dda_set_anisotropic": (C.c_int32, [P, C.c_int32, C.c_int32, D, D]),
    "dda_solve": (C.c_int32, [P, C.c_int32, C.POINTER(dda_wave), C.POINTER(dda_solve_opts), P, P,
                              C.POINTER(dda_solve_stats)]),
    "dda_solve_field": (C.c_int32, [P, C.c_int32, C.POINTER(dda_wave), C.POINTER(dda_solve_opts), P, P, P,
                                    C.POINTER(dda_solve_stats)]),
    "dda_matvec": (C.c_int32, [P, C.c_int32, C.c_int32, D, P, P, C.c_uint32, C.c_uint32]),
    "dda_matvec_noalloc": (C.c_int32, [P, C.c_int32, C.c_int32, P, P, P, C.c_uint32]),
    "dda_inverse_polarizability": (C.c_int32, [P, C.c_int32, C.POINTER(dda_wave), D]),
    "dda_cross_sections": (C.c_int32, [P, C.c_int32, D]),
    "dda_cross_sections_phi": (C.c_int32, [P, C.c_int32, C.c_int32, D, D]),
    "dda_scattering_moments": (C.c_int32, [P, C.c_int32, C.c_int32, D, D, D]),
    "dda_scattering_quadrature": (C.c_int32, [C.c_double, C.c_double, D, C.c_int32, C.POINTER(C.c_int32), D, D]),
    "dda_orientation_samples": (C.c_int32, [D, C.POINTER(C.c_int32), D, D, D, D]),
    "dda_phi_coefficients": (C.c_int32, [C.c_double, C.c_double, C.c_double, C.c_int32, D, D, D, D, D]),
    "dda_amplitudes": (C.c_int32, [P, C.c_int32, C.c_int32, D, D, D]),
    "dda_amplitudes_per_rhs": (C.c_int32, [P, C.c_int32, C.c_int32, D, D, D]),
    "dda_near_field": (C.c_int32, [P, C.c_int32, C.c_int32, D, D, D]),
    "dda_polarization": (C.c_int32, [C.c_int32, D, C.c_double, D, D]),
    "dda_mueller": (C.c_int32, [C.c_int32, D, D, D, D, D, D]),
    "dda_lab_frame": (C.c_int32, [C.c_double, C.c_double, C.c_double, D, D, D]),
    "dda_orientation_waves": (C.c_int32, [C.c_double, C.c_double, C.c_double, D, D, D, C.c_int32,
                                          C.POINTER(dda_wave)]),
    "dda_scattering_frame": (C.c_int32, [C.c_int32, D, D, D, D, D]),
    "dda_autotune": (C.c_int32, [P, C.c_int32, C.c_char_p]),
    "dda_last_timing": (C.c_int32, [P, D, D, D]),
    "dda_last_guess_ms": (C.c_int32, [P, D]),
    "dda_get_shape": (C.c_int32, [P, C.c_int32, C.c_uint32, C.POINTER(C.c_int32)]),
    "dda_set_shape": (C.c_int32, [P, C.c_int32, C.c_uint32, C.POINTER(C.c_int32)]),
    "dda_profile_matvec": (C.c_int32, [P, C.c_int32, C.c_int32, C.c_uint32, C.c_int32, D, D]),
    "dda_nn_create": (C.c_int32, [P, C.POINTER(dda_nn_config), C.POINTER(P)]),
    "dda_nn_destroy": (C.c_int32, [P]),
    "dda_nn_num_params": (C.c_int64, [P]),
    "dda_nn_num_samples": (C.c_int32, [P]),
    "dda_nn_layer_info": (C.c_int32, [P, C.POINTER(C.c_int32)]),
    "dda_nn_get_params": (C.c_int32, [P, C.POINTER(C.c_float)]),
    "dda_nn_set_params": (C.c_int32, [P, C.POINTER(C.c_float)]),
    "dda_set_guess_model": (C.c_int32, [P, P]),
    "dda_nn_record": (C.c_int32, [P, P]),
    "dda_nn_train": (C.c_int32, [P, P, C.POINTER(dda_nn_train_opts), D]),
    "dda_nn_save": (C.c_int32, [P, C.c_char_p]),
    "dda_nn_load": (C.c_int32, [P, C.c_char_p]),
    "dda_nn_forward_backward": (C.c_int32, [P, C.c_int32, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                            P, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_float), D]),
    "dda_nn_profile": (C.c_int32, [P, C.c_int32, C.c_int32, C.c_int32, D, D, D]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libdda.so and declare its functions; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_1002_1505_amd.build` "
            "(the solver has no non-GPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
