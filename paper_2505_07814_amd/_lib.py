"""ctypes binding of libptyr (include/ptyr.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libptyr.so")

PTYR_OK, PTYR_E_ARG, PTYR_E_BOUNDS, PTYR_E_NOMEM, PTYR_E_DEVICE, PTYR_E_NONFINITE = range(6)
PTYR_LOSS_GAUSSIAN, PTYR_LOSS_POISSON = 0, 1
PTYR_GLOBAL_TILT = 0x1
PTYR_CHECK_FINITE = 0x2
PTYR_REUSE_FORWARD = 0x1
PTYR_ERRBIT_BOUNDS, PTYR_ERRBIT_NONFINITE, PTYR_ERRBIT_ZERO_MEAN, PTYR_ERRBIT_INDEX = 0x1, 0x2, 0x4, 0x8
PTYR_NOALLOC_SCRATCH_BYTES = (5 * 512 + 8 + 2 * 256 * 256 + 64) * 8

STATUS_NAMES = {0: "PTYR_OK", 1: "PTYR_E_ARG", 2: "PTYR_E_BOUNDS", 3: "PTYR_E_NOMEM",
                4: "PTYR_E_DEVICE", 5: "PTYR_E_NONFINITE"}


class Geom(C.Structure):
    _fields_ = [("N", C.c_int), ("M", C.c_int), ("S", C.c_int), ("H", C.c_int), ("W", C.c_int),
                ("B_max", C.c_int), ("dx", C.c_double), ("lam", C.c_double),
                ("loss_kind", C.c_int), ("loss_p", C.c_double),
                ("wave_budget_bytes", C.c_size_t), ("flags", C.c_uint), ("n_scan", C.c_int),
                ("sparse_w", C.c_double), ("pacbed_w", C.c_double), ("n_obj", C.c_int),
                ("w_gaussian", C.c_double), ("w_poisson", C.c_double),
                ("p_gaussian", C.c_double), ("p_poisson", C.c_double)]


_fp = C.c_void_p


class Params(C.Structure):
    _fields_ = [(n, _fp) for n in ("amp", "phase", "probe", "pos", "tilt", "dz",
                                   "m_amp", "v_amp", "m_phase", "v_phase", "m_probe", "v_probe",
                                   "m_pos", "v_pos", "m_tilt", "v_tilt", "m_dz", "v_dz")] + \
               [("n_pos", C.c_int), ("step", C.c_int64)]


class LR(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("amp", "phase", "probe", "pos", "tilt", "dz",
                                         "beta1", "beta2", "eps")]


class Constraints(C.Structure):
    _fields_ = [("rz_sigma", C.c_float), ("phase_positive", C.c_int), ("probe_orthogonal", C.c_int),
                ("kz_beta", C.c_float), ("kz_alpha", C.c_float), ("kz_dz", C.c_float)]


class PtyrError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}")


_lib = None


def lib():
    """Load libptyr.so (built in-tree by __graft_entry__.build()).  There is
    no fallback: a missing library is an error."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libptyr.so not built at {LIB_PATH}; run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    st = C.c_int
    vp = C.c_void_p
    sig = {
        "ptyr_status_str": (C.c_char_p, [st]),
        "ptyr_check_geom": (st, [C.POINTER(Geom)]),
        "ptyr_check_args": (st, [C.POINTER(Geom), C.c_int, vp]),
        "ptyr_workspace_bytes": (C.c_size_t, [C.POINTER(Geom)]),
        "ptyr_checkpoint_plan": (st, [C.POINTER(Geom), C.POINTER(C.c_int)]),
        "ptyr_create": (st, [C.POINTER(Geom), vp, C.c_size_t, vp, C.POINTER(vp)]),
        "ptyr_destroy": (st, [vp]),
        "ptyr_sync": (st, [vp]),
        "ptyr_forward": (st, [vp, vp, vp, vp, vp, vp, vp, vp, C.c_int, C.c_int, vp]),
        "ptyr_loss": (st, [vp, vp, vp, vp, C.c_int, C.c_int, vp, vp]),
        "ptyr_loss_noalloc": (st, [C.POINTER(Geom), vp, vp, vp, C.c_int, C.c_int, vp, vp, vp, vp]),
        "ptyr_adjoint": (st, [vp, vp, vp, vp, vp, vp, vp, vp, C.c_int, C.c_int, vp,
                              vp, vp, vp, vp, vp, vp, vp, C.c_uint]),
        "ptyr_step": (st, [vp, C.POINTER(Params), vp, C.c_int, vp, C.POINTER(LR), vp]),
        "ptyr_constrain": (st, [vp, vp, vp, vp, C.POINTER(Constraints)]),
        "ptyr_timing_enable": (st, [vp, C.c_int]),
        "ptyr_timing_read": (st, [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
        # learned initial guess (include/ptyr_cnn.h)
        "ptyr_cnn_param_count": (C.c_size_t, []),
        "ptyr_cnn_workspace_bytes": (C.c_size_t, [C.c_int]),
        "ptyr_cnn_create": (st, [C.c_int, vp, C.c_size_t, vp, C.POINTER(vp)]),
        "ptyr_cnn_destroy": (None, [vp]),
        "ptyr_cnn_sync": (st, [vp]),
        "ptyr_cnn_forward": (st, [vp, vp, vp, C.c_int, vp, C.c_int, vp]),
        "ptyr_cnn_gradient": (st, [vp, vp, vp, C.c_int, vp, vp, C.c_int, vp, vp]),
        "ptyr_cnn_adam": (st, [vp, vp, vp, vp, vp, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float]),
        "ptyr_cnn_stitch": (st, [vp, vp, vp, C.c_int, C.c_int, C.c_int, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(status, what):
    if status != PTYR_OK:
        raise PtyrError(status, what)


HEADER_SYMBOLS = ["ptyr_status_str", "ptyr_check_geom", "ptyr_check_args", "ptyr_workspace_bytes",
                  "ptyr_checkpoint_plan", "ptyr_create", "ptyr_destroy", "ptyr_sync", "ptyr_forward",
                  "ptyr_loss", "ptyr_loss_noalloc", "ptyr_adjoint", "ptyr_step", "ptyr_constrain", "ptyr_timing_enable",
                  "ptyr_timing_read"]

CNN_HEADER_SYMBOLS = ["ptyr_cnn_param_count", "ptyr_cnn_workspace_bytes", "ptyr_cnn_create", "ptyr_cnn_destroy",
                      "ptyr_cnn_sync", "ptyr_cnn_forward", "ptyr_cnn_gradient", "ptyr_cnn_adam", "ptyr_cnn_stitch"]

PTYR_K_FORWARD, PTYR_K_GRADIENT, PTYR_K_RZ = 0, 1, 2
