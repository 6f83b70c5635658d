"""ctypes declarations of the C ABI in include/msfv.h.

Argument marshalling only: every step of the MSFV path runs in the HIP
kernels of libmsfv.so.  If the shared library has not been built this module
raises at import; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsfv.so")

MSFV_OK = 0
MSFV_EINVAL = -1
MSFV_ENOMEM = -2
MSFV_ENOCONV = -3
MSFV_ENONFINITE = -4
MSFV_EDEVICE = -5
MSFV_ESTATE = -6
MSFV_BC_REDUCED = 0
MSFV_BC_LAGRANGE = 1
MSFV_COARSE_TWOLEVEL = 0
MSFV_COARSE_JACOBI = 1
MSFV_COARSE_MULTI = 2

STATUS_NAMES = {
    MSFV_OK: "MSFV_OK", MSFV_EINVAL: "MSFV_EINVAL", MSFV_ENOMEM: "MSFV_ENOMEM",
    MSFV_ENOCONV: "MSFV_ENOCONV", MSFV_ENONFINITE: "MSFV_ENONFINITE",
    MSFV_EDEVICE: "MSFV_EDEVICE", MSFV_ESTATE: "MSFV_ESTATE",
}


class MsfvConfig(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("r", ctypes.c_int * 3),
                ("bc_mode", ctypes.c_int), ("local_rtol", ctypes.c_double),
                ("local_maxit", ctypes.c_int), ("coarse_rtol", ctypes.c_double),
                ("coarse_maxit", ctypes.c_int), ("coarse_precond", ctypes.c_int)]


class MsfvSizes(ctypes.Structure):
    _fields_ = [("ncell", ctypes.c_longlong), ("ncoarse", ctypes.c_longlong),
                ("nnz_p", ctypes.c_longlong), ("nnz_k", ctypes.c_longlong),
                ("nsrc", ctypes.c_int), ("nrec", ctypes.c_int), ("nblock", ctypes.c_int),
                ("nface", ctypes.c_int), ("nedge", ctypes.c_int),
                ("workspace_bytes", ctypes.c_longlong), ("pairs_block", ctypes.c_longlong),
                ("pairs_face", ctypes.c_longlong)]


class MsfvServeStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_longlong), ("failed", ctypes.c_longlong),
                ("p50_ms", ctypes.c_double), ("p90_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("span_s", ctypes.c_double),
                ("throughput", ctypes.c_double), ("rejected", ctypes.c_longlong),
                ("budget_bytes", ctypes.c_double), ("resident_bytes", ctypes.c_double),
                ("peak_committed_bytes", ctypes.c_double)]


class MsfvStats(ctypes.Structure):
    _fields_ = [("local_max_it", ctypes.c_int), ("local_noconv", ctypes.c_int),
                ("coarse_max_it", ctypes.c_int), ("coarse_noconv", ctypes.c_int),
                ("nonfinite", ctypes.c_int), ("local_max_res", ctypes.c_double),
                ("coarse_max_res", ctypes.c_double)]


NSTAGE = 19


class MsfvProfile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * NSTAGE), ("count", ctypes.c_int * NSTAGE),
                ("work", ctypes.c_ulonglong * 8)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_IP = ctypes.POINTER(ctypes.c_int)
_DP = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes); the exported surface of include/msfv.h
SIGNATURES = {
    "msfv_create": (_I, [ctypes.POINTER(MsfvConfig), _P, ctypes.POINTER(_P)]),
    "msfv_destroy": (None, [_P]),
    "msfv_set_sources": (_I, [_P, _I, _IP, _IP, _DP]),
    "msfv_set_receivers": (_I, [_P, _I, _IP, _IP, _DP]),
    "msfv_forward": (_I, [_P, _P, _P, _P]),
    "msfv_jtv": (_I, [_P, _P, _P]),
    "msfv_forward_jtv": (_I, [_P, _P, _P, _P, _P]),
    "msfv_misfit_grad": (_I, [_P, _P, _P, _P, _P]),
    "msfv_misfit_grad_noalloc": (_I, [_P, _P, _P, _P, _P]),
    "msfv_jvp": (_I, [_P, _P, _P]),
    "msfv_jvp_fixed": (_I, [_P, _P, _P]),
    "msfv_jtv_fixed": (_I, [_P, _P, _P]),
    "msfv_set_basis": (_I, [_P, _I]),
    "msfv_sync": (_I, [_P]),
    "msfv_get_sizes": (_I, [_P, ctypes.POINTER(MsfvSizes)]),
    "msfv_get_prolongation": (_I, [_P, _IP, _IP, _DP]),
    "msfv_get_coarse": (_I, [_P, _IP, _IP, _DP, _DP]),
    "msfv_get_stats": (_I, [_P, ctypes.POINTER(MsfvStats)]),
    "msfv_profile_enable": (_I, [_P, _I]),
    "msfv_profile_read": (_I, [_P, ctypes.POINTER(MsfvProfile)]),
    "msfv_stage_name": (ctypes.c_char_p, [_I]),
    "msfv_batch_create": (_I, [_I, ctypes.POINTER(_P), _P, ctypes.POINTER(_P)]),
    "msfv_batch_destroy": (None, [_P]),
    "msfv_batch_forward_jtv": (_I, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                    ctypes.POINTER(_P)]),
    "msfv_batch_sync": (_I, [_P]),
    "msfv_batch_set_options": (_I, [_P, _I, _I, _I]),
    "msfv_batch_get_options": (_I, [_P, _IP, _IP, _IP]),
    "msfv_batch_autotune": (_I, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                 ctypes.POINTER(_P), _IP, _IP, _IP]),
    "msfv_server_create": (_I, [_I, ctypes.c_double, ctypes.POINTER(_P)]),
    "msfv_server_destroy": (None, [_P]),
    "msfv_server_add_job": (_I, [_P, _P, _I, _IP]),
    "msfv_server_request_bytes": (_I, [_P, _I, _I, ctypes.POINTER(ctypes.c_longlong),
                                       ctypes.POINTER(ctypes.c_longlong)]),
    "msfv_server_submit": (_I, [_P, _I, _I, _IP, _IP, _DP, _P, _P, _P, _P, _P,
                                ctypes.POINTER(ctypes.c_longlong)]),
    "msfv_server_wait": (_I, [_P, ctypes.c_longlong, _DP, _DP, _DP]),
    "msfv_server_drain": (_I, [_P]),
    "msfv_server_stats": (_I, [_P, ctypes.POINTER(MsfvServeStats), _I]),
    "msfv_status_string": (ctypes.c_char_p, [_I]),
    "msfv_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmsfv.so once; raise if it is missing (no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_1707_07598_amd.build` "
            "(the MSFV path has no fallback without its HIP library)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MsfvError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {detail}")


def check(status: int, where: str) -> None:
    if status != MSFV_OK:
        detail = load().msfv_last_error()
        raise MsfvError(status, where, detail.decode() if detail else "")
