"""ctypes binding of libisci (argument marshalling only).

Every computation runs in the HIP library; this module only converts
Python / torch arguments to pointers, sizes and streams and maps status
codes to exceptions.  If libisci.so is missing the import fails loudly --
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libisci.so")

NBUCKET = 42
MAX_ROOTS = 32

ISCI_OK = 0
ISCI_E_INVALID = -1
ISCI_E_OOM = -2
ISCI_E_HIP = -3
ISCI_E_NOT_CONVERGED = -4
ISCI_E_UNSUPPORTED = -5

# Exported symbols declared in include/isci.h.
ABI_SYMBOLS = (
    "isci_create", "isci_create_ex", "isci_dim", "isci_sigma", "isci_diag", "isci_davidson",
    "isci_davidson_defaults", "isci_strings", "isci_rowstart", "isci_get_stats",
    "isci_destroy", "isci_status_string", "isci_last_error",
    "isci_engine_create", "isci_engine_config", "isci_engine_add", "isci_engine_step",
    "isci_engine_result", "isci_engine_release", "isci_engine_sigma", "isci_engine_destroy",
    "isci_davidson_footprint", "isci_set_option", "isci_profile", "isci_profile_read",
    "isci_sigma_graph_create", "isci_graph_launch", "isci_graph_destroy", "isci_probe_fp64", "isci_density1",
    "isci_density1_noalloc", "isci_create_factored", "isci_density2",
    "isci_propagate_defaults", "isci_propagate",
)


class IsciPropagateOpts(ctypes.Structure):
    _fields_ = [("krylov", ctypes.c_int), ("imaginary", ctypes.c_int), ("tol", ctypes.c_double),
                ("coef_tau", ctypes.c_double)]


class IsciPropagateInfo(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_double), ("norm", ctypes.c_double), ("sigma_calls", ctypes.c_int),
                ("krylov_last", ctypes.c_int), ("screened_last", ctypes.c_int64)]


class IsciStats(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int64), ("nstr_alpha", ctypes.c_int64), ("nstr_beta", ctypes.c_int64),
                ("kept", ctypes.c_int64 * NBUCKET), ("terms", ctypes.c_int64 * NBUCKET),
                ("kept_total", ctypes.c_int64), ("terms_total", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class IsciAllocator(ctypes.Structure):
    """isci_allocator."""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class IsciCreateOpts(ctypes.Structure):
    """isci_create_opts."""
    _fields_ = [("onebody", ctypes.c_int), ("allocator", ctypes.POINTER(IsciAllocator)),
                ("orb_dist", ctypes.POINTER(ctypes.c_double)), ("max_dist", ctypes.c_double),
                ("gas_boundary", ctypes.c_int)]


class IsciDavidsonOpts(ctypes.Structure):
    _fields_ = [("tol_residual", ctypes.c_double), ("tol_energy", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("max_subspace", ctypes.c_int), ("block", ctypes.c_int)]


class IsciDavidsonInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("sigma_calls", ctypes.c_int),
                ("residual", ctypes.c_double * MAX_ROOTS)]


class IsciError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_LIB = None


def load(path: str = LIBPATH):
    """Load libisci.so and declare its signatures."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"libisci.so not built ({path}); run __graft_entry__.build()")
    L = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.isci_create.argtypes = [ctypes.POINTER(vp), vp, vp, i32, i32, i32, i32, dbl, vp]
    L.isci_create.restype = i32
    L.isci_create_ex.argtypes = [ctypes.POINTER(vp), vp, vp, i32, i32, i32, i32, dbl,
                                 ctypes.POINTER(IsciCreateOpts), vp]
    L.isci_create_factored.argtypes = [ctypes.POINTER(vp), vp, vp, i32, i32, i32, i32, i32, dbl,
                                       ctypes.POINTER(IsciCreateOpts), vp]
    L.isci_create_factored.restype = i32
    L.isci_create_ex.restype = i32
    L.isci_dim.argtypes = [vp, ctypes.POINTER(i64)]
    L.isci_dim.restype = i32
    L.isci_sigma.argtypes = [vp, i32, vp, i64, vp, i64, vp]
    L.isci_sigma.restype = i32
    L.isci_sigma_graph_create.argtypes = [vp, i32, vp, i64, vp, i64, ctypes.POINTER(vp)]
    L.isci_sigma_graph_create.restype = i32
    L.isci_graph_launch.argtypes = [vp, vp]
    L.isci_graph_launch.restype = i32
    L.isci_probe_fp64.argtypes = [i32, i64, i32, vp, ctypes.POINTER(dbl), vp]
    L.isci_probe_fp64.restype = i32
    L.isci_graph_destroy.argtypes = [vp]
    L.isci_graph_destroy.restype = None
    L.isci_density1.argtypes = [vp, i32, vp, i64, vp, vp]
    L.isci_density1.restype = i32
    L.isci_propagate_defaults.argtypes = [ctypes.POINTER(IsciPropagateOpts)]
    L.isci_propagate_defaults.restype = None
    L.isci_propagate.argtypes = [vp, vp, vp, dbl, i32, ctypes.POINTER(IsciPropagateOpts),
                                 ctypes.POINTER(IsciPropagateInfo), vp]
    L.isci_propagate.restype = i32
    L.isci_density2.argtypes = [vp, i32, vp, i64, vp, vp]
    L.isci_density2.restype = i32
    L.isci_density1_noalloc.argtypes = [vp, i32, vp, i64, vp, vp]
    L.isci_density1_noalloc.restype = i32
    L.isci_diag.argtypes = [vp, vp, vp]
    L.isci_diag.restype = i32
    L.isci_davidson.argtypes = [vp, i32, ctypes.POINTER(IsciDavidsonOpts), vp, i32,
                                ctypes.POINTER(dbl), vp, ctypes.POINTER(IsciDavidsonInfo), vp]
    L.isci_davidson.restype = i32
    L.isci_davidson_defaults.argtypes = [ctypes.POINTER(IsciDavidsonOpts)]
    L.isci_davidson_defaults.restype = None
    L.isci_strings.argtypes = [vp, i32, vp, vp, ctypes.POINTER(i64)]
    L.isci_strings.restype = i32
    L.isci_rowstart.argtypes = [vp, vp]
    L.isci_rowstart.restype = i32
    L.isci_get_stats.argtypes = [vp, ctypes.POINTER(IsciStats)]
    L.isci_get_stats.restype = i32
    L.isci_destroy.argtypes = [vp]
    L.isci_destroy.restype = None
    L.isci_status_string.argtypes = [i32]
    L.isci_status_string.restype = ctypes.c_char_p
    L.isci_last_error.argtypes = []
    L.isci_last_error.restype = ctypes.c_char_p
    L.isci_engine_create.argtypes = [ctypes.POINTER(vp), vp]
    L.isci_engine_create.restype = i32
    L.isci_engine_config.argtypes = [vp, i32, i32]
    L.isci_engine_config.restype = i32
    L.isci_engine_add.argtypes = [vp, vp, i32, ctypes.POINTER(IsciDavidsonOpts), vp, i32,
                                  ctypes.POINTER(ctypes.c_int)]
    L.isci_engine_add.restype = i32
    L.isci_engine_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    L.isci_engine_step.restype = i32
    L.isci_engine_result.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(dbl), vp,
                                     ctypes.POINTER(IsciDavidsonInfo)]
    L.isci_engine_result.restype = i32
    L.isci_engine_release.argtypes = [vp, i32]
    L.isci_engine_release.restype = i32
    L.isci_engine_sigma.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(vp),
                                    ctypes.POINTER(i64)]
    L.isci_engine_sigma.restype = i32
    L.isci_engine_destroy.argtypes = [vp]
    L.isci_engine_destroy.restype = None
    L.isci_davidson_footprint.argtypes = [vp, i32, ctypes.POINTER(IsciDavidsonOpts)]
    L.isci_davidson_footprint.restype = i64
    L.isci_set_option.argtypes = [vp, i32, i32]
    L.isci_set_option.restype = i32
    L.isci_profile.argtypes = [vp, i32]
    L.isci_profile.restype = i32
    L.isci_profile_read.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    L.isci_profile_read.restype = i32
    _LIB = L
    return L


def check(status: int, what: str = "isci"):
    if status != ISCI_OK:
        L = load()
        msg = L.isci_last_error().decode(errors="replace")
        raise IsciError(status, f"{what}: {L.isci_status_string(status).decode()}: {msg}")
