"""ctypes declarations of the C interface in include/arna.h.

Argument marshalling only: every step of the filter runs in the HIP library.
Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libarna.so")

PF_OK, PF_EINVAL, PF_ENOMEM, PF_EHIP, PF_ENUMERIC, PF_ESTATE, PF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
PF_ETIMEOUT = -7
PF_MODE_RNA, PF_MODE_ARNA = 0, 1
PF_INIT_TRACKING, PF_INIT_INFOSHARE = 0, 1
PF_LIK_PATCH, PF_LIK_POINT, PF_LIK_POISSON = 0, 1, 2
PF_LAUNCH_AUTO, PF_LAUNCH_STEPWISE, PF_LAUNCH_PERSISTENT = 0, 1, 2
PF_DEBUG_TRACE, PF_DEBUG_LINEAGE = 1, 2
PF_MAX_PE, PF_MAX_PER_PE, PF_MAX_PATCH = 8192, 65536, 15
PF_MAX_PER_PE_LDS = 4096
PF_MAX_PARTICLES = 1 << 29
PF_BATCH_NOALLOC_MAX_ARGS = 4096

DBG = dict(state=0, logmass=1, pe_records=2, ring=3, nex=4, src=5, prop=6, ell=7, q=8,
           ancestors=9, v=10, lam=11, lineage=12)


class PFError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class pf_config(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("n_filters", ctypes.c_uint32), ("n_pe", ctypes.c_uint32), ("n_per_pe", ctypes.c_uint32),
        ("width", ctypes.c_uint32), ("height", ctypes.c_uint32), ("patch", ctypes.c_uint32),
        ("mode", ctypes.c_uint32), ("init_mode", ctypes.c_uint32), ("lik_mode", ctypes.c_uint32),
        ("fixed_ratio", ctypes.c_float), ("initial_ratio", ctypes.c_float),
        ("eff_cutoff", ctypes.c_float),
        ("psf_sigma", ctypes.c_float), ("background", ctypes.c_float),
        ("noise_sigma", ctypes.c_float), ("q", ctypes.c_float), ("sigma_I", ctypes.c_float),
        ("debug", ctypes.c_uint32),
        ("ring_groups", ctypes.c_uint32),
        ("block_size", ctypes.c_uint32),
        ("launch", ctypes.c_uint32),
        ("pes_per_wg", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("stream", ctypes.c_void_p),
    ]


class pf_estimate_t(ctypes.Structure):
    _fields_ = [
        ("x_global", ctypes.POINTER(ctypes.c_double)),
        ("x_pe", ctypes.POINTER(ctypes.c_double)),
        ("log_mass_pe", ctypes.POINTER(ctypes.c_double)),
        ("log_mass_glob", ctypes.POINTER(ctypes.c_double)),
        ("pe_eff", ctypes.POINTER(ctypes.c_double)),
        ("n_ex", ctypes.POINTER(ctypes.c_uint32)),
        ("n_ex_next", ctypes.POINTER(ctypes.c_uint32)),
        ("log_z_inc", ctypes.POINTER(ctypes.c_double)),
        ("step", ctypes.c_uint64),
    ]


class pf_master_t(ctypes.Structure):
    _fields_ = [
        ("xhat", ctypes.c_double * 5),
        ("log_mass_glob", ctypes.c_double),
        ("pe_eff", ctypes.c_double),
        ("log_z_inc", ctypes.c_double),
        ("n_ex", ctypes.c_uint32),
        ("n_ex_next", ctypes.c_uint32),
        ("step", ctypes.c_uint64),
    ]


class pf_pe_record(ctypes.Structure):
    _fields_ = [
        ("log_mass", ctypes.c_double),
        ("xhat", ctypes.c_double * 5),
        ("lstar", ctypes.c_float),
        ("total_q", ctypes.c_uint32),
    ]


# name -> (restype, argtypes); the list of exports declared in include/arna.h
_P = ctypes.c_void_p
_U32P = ctypes.POINTER(ctypes.c_uint32)
SIGNATURES = {
    "pf_init": (ctypes.c_int, [ctypes.POINTER(pf_config), ctypes.POINTER(ctypes.c_float),
                               ctypes.POINTER(ctypes.c_void_p)]),
    "pf_step": (ctypes.c_int, [_P, _P]),
    "pf_run": (ctypes.c_int, [_P, _P, ctypes.c_uint32, ctypes.c_uint64]),
    "pf_run_traj": (ctypes.c_int, [_P, _P, ctypes.c_uint32, ctypes.c_uint64, _P]),
    "pf_run_timed": (ctypes.c_int, [_P, _P, ctypes.c_uint32, ctypes.c_uint64,
                                    ctypes.POINTER(ctypes.c_float)]),
    "pf_run_info": (ctypes.c_int, [_P, _U32P]),
    "pf_exchange": (ctypes.c_int, [_P, _P]),
    "pf_estimate": (ctypes.c_int, [_P, ctypes.POINTER(pf_estimate_t)]),
    "pf_destroy": (None, [_P]),
    "pf_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "pf_batch_create": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)]),
    "pf_batch_run": (ctypes.c_int, [_P, _P, _P, ctypes.c_uint32, ctypes.c_int]),
    "pf_batch_run_noalloc": (ctypes.c_int, [_P, _P, _P, ctypes.c_uint32]),
    "pf_batch_destroy": (None, [_P]),
    "pf_grad_begin": (ctypes.c_int, [_P, ctypes.c_uint32]),
    "pf_grad_end": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]),
    "pf_grad_value": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "pf_debug_size": (ctypes.c_size_t, [_P, ctypes.c_int]),
    "pf_debug_get": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_size_t]),
    "pf_debug_set_state": (ctypes.c_int, [_P, _P, _P, ctypes.c_uint64]),
    "pf_debug_set_lineage": (ctypes.c_int, [_P, _P]),
    "pf_debug_force_next": (ctypes.c_int, [_P, _P, _P]),
    "pf_debug_resample_q": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.c_uint32, _P, _P]),
    "pf_debug_nex": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int,
                                    _U32P]),
    "pf_debug_ring": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _P]),
    "pf_debug_philox": (ctypes.c_int, [_P, _P, ctypes.c_uint32, _P]),
}

_lib = None


def lib():
    """Load libarna.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing; build it with "
                               "`python -m paper_1310_4624_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().pf_strerror(code).decode()
    except Exception:   # library missing: still give a readable message
        return f"error {code}"


def check(rc: int, where: str) -> None:
    if rc != PF_OK:
        raise PFError(rc, where)
