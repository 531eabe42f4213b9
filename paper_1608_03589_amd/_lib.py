"""ctypes binding of ``libtvpd.so`` (the C ABI declared in ``include/tvpd.h``).

Argument marshalling only: every step of the solver runs in the HIP library.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtvpd.so")

OK = 0
STATUS = {
    0: "TVPD_OK", -1: "TVPD_ERR_INVALID_ARG", -2: "TVPD_ERR_SHAPE",
    -3: "TVPD_ERR_ALIGNMENT", -4: "TVPD_ERR_WORKSPACE", -5: "TVPD_ERR_HIP",
    -6: "TVPD_ERR_UNSUPPORTED", -7: "TVPD_ERR_STEP", -8: "TVPD_ERR_DEVICE",
    -9: "TVPD_ERR_SCRATCH",
}


class Shape(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("nz", C.c_int32), ("ny", C.c_int32),
                ("nx", C.c_int32)]


class Coeffs(C.Structure):
    _fields_ = [("lam", C.c_float), ("tau", C.c_float), ("sigma", C.c_float),
                ("theta", C.c_float)]


class Params(C.Structure):
    _fields_ = [("c", Coeffs), ("max_iter", C.c_int32),
                ("check_every", C.c_int32), ("gap_tol", C.c_double),
                ("use_graph", C.c_int32), ("reserved", C.c_int32)]


class BatchOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("th", C.c_int32), ("wpb", C.c_int32),
                ("th_short", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32),
                ("primal", C.c_double), ("dual", C.c_double),
                ("gap", C.c_double)]


class TomoGeom(C.Structure):
    _fields_ = [("ny", C.c_int32), ("nx", C.c_int32), ("n_angles", C.c_int32),
                ("n_det", C.c_int32)]


class TomoParams(C.Structure):
    _fields_ = [("lam", C.c_float), ("tau", C.c_float), ("sigma_r", C.c_float),
                ("sigma_p", C.c_float), ("theta", C.c_float), ("reg", C.c_int32)]


REG_TV = 0
REG_TIKHONOV = 1


class TVPDError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed: {STATUS.get(status, status)} ({msg})")
        self.status = status


_P = C.c_void_p
_SZ = C.c_size_t
_I32 = C.c_int32
_F = C.c_float

# name -> (restype, argtypes); mirrors include/tvpd.h
SIGNATURES = {
    "tvpd_status_string": (C.c_char_p, [C.c_int]),
    "tvpd_version": (C.c_int, []),
    "tvpd_release_thread_resources": (C.c_int, []),
    "tvpd_workspace_size": (C.c_int, [C.POINTER(Shape), C.POINTER(_SZ)]),
    "tvpd_init": (C.c_int, [C.POINTER(Shape), _P, _P, _SZ, _P]),
    "tvpd_step": (C.c_int, [C.POINTER(Shape), C.POINTER(Coeffs), _I32, _P, _SZ, _P]),
    "tvpd_read_state": (C.c_int, [C.POINTER(Shape), _P, _SZ, _P, _P, _P]),
    "tvpd_iteration": (C.c_int, [C.POINTER(Shape), _P, _SZ, C.POINTER(_I32), _P]),
    "tvpd_energy_gap": (C.c_int, [C.POINTER(Shape), _F, _P, _SZ,
                                  C.POINTER(C.c_double), _P]),
    "tvpd_solve": (C.c_int, [C.POINTER(Shape), _P, _P, C.POINTER(Params), _P, _SZ,
                             C.POINTER(Result), _P]),
    "tvpd_set_tile": (C.c_int, [C.POINTER(Shape), _I32, _I32, _I32]),
    "tvpd_get_tile": (C.c_int, [C.POINTER(Shape), C.POINTER(_I32), C.POINTER(_I32),
                                C.POINTER(_I32)]),
    "tvpd_set_fused_adjoint": (C.c_int, [_I32]),
    "tvpd_set_pass_depth": (C.c_int, [_I32]),
    "tvpd_get_pass_depth": (C.c_int, [C.POINTER(_I32)]),
    "tvpd_pass_length": (C.c_int, [C.POINTER(Shape), C.POINTER(_I32)]),
    "tvpd_set_wait_limit": (C.c_int, [C.c_int64]),
    "tvpd_stream_copy": (C.c_int, [_P, _P, C.c_int64, _P]),
    "tvpd_set_tile3d": (C.c_int, [C.POINTER(Shape), _I32, _I32, _I32]),
    "tvpd_get_tile3d": (C.c_int, [C.POINTER(Shape), C.POINTER(_I32),
                                  C.POINTER(_I32), C.POINTER(_I32)]),
    "tvpd_autotune": (C.c_int, [C.POINTER(Shape), _P, _SZ, C.c_char_p,
                                C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32),
                                C.POINTER(C.c_float), _P]),
    "tvpd_tune_load": (C.c_int, [C.c_char_p, C.POINTER(_I32)]),
    "tvpd_set_blocking": (C.c_int, [_I32]),
    "tvpd_unrolled_workspace_size": (C.c_int, [C.POINTER(Shape), _I32, _I32, _I32,
                                               C.POINTER(_SZ)]),
    "tvpd_unrolled_forward": (C.c_int, [C.POINTER(Shape), _I32, _P, _P, _I32, _I32, _F,
                                        _P, _P, _SZ, _P]),
    "tvpd_unrolled_backward": (C.c_int, [C.POINTER(Shape), _I32, _P, _I32, _I32, _F,
                                         _P, _P, _P, _P, _SZ, _P]),
    "tvpd_batch_workspace_size": (C.c_int, [_I32, C.POINTER(Shape), C.POINTER(_SZ)]),
    "tvpd_solve_batched": (C.c_int, [_I32, C.POINTER(Shape), C.POINTER(C.c_int64),
                                     _P, _P, C.POINTER(Params), C.POINTER(BatchOpts),
                                     _P, _SZ, C.POINTER(Result), _P]),
    "tvpd_batch_autotune": (C.c_int, [_I32, C.POINTER(Shape), C.POINTER(C.c_int64),
                                      _P, _P, C.POINTER(Params), _P, _SZ,
                                      C.POINTER(_I32), C.POINTER(_I32),
                                      C.POINTER(C.c_float), _P]),
    "tvpd_tomo_workspace_size": (C.c_int, [C.POINTER(TomoGeom), C.POINTER(_SZ)]),
    "tvpd_radon_forward": (C.c_int, [C.POINTER(TomoGeom), _P, _P, _P, _SZ, _P]),
    "tvpd_set_projection_staging": (C.c_int, [_I32]),
    "tvpd_radon_backward": (C.c_int, [C.POINTER(TomoGeom), _P, _P, _P, _SZ, _P]),
    "tvpd_tomo_init": (C.c_int, [C.POINTER(TomoGeom), _P, _P, _SZ, _P]),
    "tvpd_tomo_step": (C.c_int, [C.POINTER(TomoGeom), _P, C.POINTER(TomoParams), _I32,
                                 _P, _SZ, _P]),
    "tvpd_tomo_read": (C.c_int, [C.POINTER(TomoGeom), _P, _SZ, _P, _P, _P,
                                 C.POINTER(_I32), _P]),
    "tvpd_tomo_energy": (C.c_int, [C.POINTER(TomoGeom), _P, _F, _I32, _P, _SZ,
                                   C.POINTER(C.c_double), _P]),
    "tvpd_tomo_opnorm": (C.c_int, [C.POINTER(TomoGeom), _I32, _P, _SZ,
                                   C.POINTER(C.c_double), _P]),
    "tvpd_fbp": (C.c_int, [C.POINTER(TomoGeom), _P, _F, _P, _P, _SZ, _P]),
    "tvpd_fbp_noalloc": (C.c_int, [C.POINTER(TomoGeom), _P, _F, _P, _P]),
    "tvpd_bst_lengths": (C.c_int, [C.POINTER(TomoGeom), C.POINTER(_I32), C.POINTER(_I32)]),
    "tvpd_bst_workspace_size": (C.c_int, [C.POINTER(TomoGeom), C.POINTER(_SZ)]),
    "tvpd_bst_backproject": (C.c_int, [C.POINTER(TomoGeom), _P, _P, _P, _SZ, _P]),
    "tvpd_bst_spectra": (C.c_int, [C.POINTER(TomoGeom), _P, _P, _P, _SZ, _P]),
    "tvpd_fbp_bst": (C.c_int, [C.POINTER(TomoGeom), _P, _F, _P, _P, _SZ, _P]),
    "tvpd_lp_mesh": (C.c_int, [C.POINTER(TomoGeom), C.POINTER(_I32), C.POINTER(_I32),
                               C.POINTER(_I32), C.POINTER(C.c_double),
                               C.POINTER(C.c_double)]),
    "tvpd_lp_workspace_size": (C.c_int, [C.POINTER(TomoGeom), C.POINTER(_SZ)]),
    "tvpd_lp_plan": (C.c_int, [C.POINTER(TomoGeom), _P, _SZ, _P]),
    "tvpd_lp_backproject": (C.c_int, [C.POINTER(TomoGeom), _P, _P, _P, _P, _SZ, _P]),
    "tvpd_tomo_solve": (C.c_int, [C.POINTER(TomoGeom), _P, C.POINTER(TomoParams), _I32,
                                  _P, _P, _SZ, _P]),
}

_lib = None


def lib():
    """Load libtvpd.so once; raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1608_03589_amd.build` (there is no fallback)")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
        # pinned buffers, events and the capture stream of the solve drivers
        # are released while the HIP runtime is still up
        atexit.register(h.tvpd_release_thread_resources)
    return _lib


def check(fn: str, status: int):
    if status != OK:
        msg = lib().tvpd_status_string(status).decode()
        raise TVPDError(fn, status, msg)
    return status


def call(name: str, *args):
    return check(name, getattr(lib(), name)(*args))
