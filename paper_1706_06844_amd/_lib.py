"""ctypes binding of libfde (the C ABI of include/fde.h): argument marshalling only.

Every computation runs in the HIP kernels of libfde.so.  Importing this module does not touch the
GPU; loading the library raises if it has not been built (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfde.so")

FDE_OK = 0
FDE_EINVAL = -1
FDE_ENEGCOEF = -2
FDE_ENOMEM = -3
FDE_ENONFINITE = -4
FDE_EDEVICE = -5
FDE_EAGAIN = -6
FDE_ENOCONV = 1

FDE_FP64 = 0
FDE_MIXED_FP32 = 1
FDE_MIXED_BF16GEMM = 2
FDE_MIXED_FP32_CYCLE = 3
FDE_MIXED_CYCLE_BF16 = 4
FDE_MG_GEOMETRIC = 0
FDE_MG_GALERKIN = 1
FDE_MG_BAND = 2

KFAM = ["outer_y", "outer_x", "mg0_y", "mg0_x", "mgc_y", "mgc_x", "cgs", "transfer", "coarse", "update",
        "cgs_finalize"]


class fde_problem(ctypes.Structure):
    _fields_ = [
        ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
        ("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
        ("a1", ctypes.c_double), ("b1", ctypes.c_double),
        ("a2", ctypes.c_double), ("b2", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("precision", ctypes.c_int32), ("mg_variant", ctypes.c_int32),
        ("omega", ctypes.c_double),
        ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32), ("coarsest_n", ctypes.c_int32),
        ("restart", ctypes.c_int32), ("maxit", ctypes.c_int32),
        ("rtol", ctypes.c_double),
    ]


class fde_stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
        ("converged", ctypes.c_int32), ("reorth_steps", ctypes.c_int32),
        ("relres_true", ctypes.c_double), ("relres_est", ctypes.c_double),
    ]

    def as_dict(self):
        return {"iters": self.iters, "restarts": self.restarts, "converged": bool(self.converged), "reorth_steps": self.reorth_steps,
                "relres_true": self.relres_true, "relres_est": self.relres_est}


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_I32 = ctypes.c_int32

# name -> (restype, argtypes)
FDE_NOALLOC_MAX_N = 1023  # largest n1, n2 of fde_apply_noalloc

SIGNATURES = {
    "fde_problem_default": (None, [ctypes.POINTER(fde_problem), _D, _D, _I32, _I32, _D]),
    "fde_setup": (_I, [ctypes.POINTER(fde_problem), _P, _P, _P, _P, _P, ctypes.POINTER(_P)]),
    "fde_update_coeffs": (_I, [_P, _P, _P, _P, _P]),
    "fde_step": (_I, [_P, _P, _P, _P, ctypes.POINTER(fde_stats)]),
    "fde_step_sources": (_I, [_P, _P, _I32, ctypes.POINTER(_D), ctypes.POINTER(_P), _P,
                              ctypes.POINTER(fde_stats)]),
    "fde_solve": (_I, [_P, _P, _P, ctypes.POINTER(fde_stats)]),
    "fde_solve_mg": (_I, [_P, _P, _P, _I32, ctypes.POINTER(fde_stats)]),
    "fde_destroy": (None, [_P]),
    "fde_last_error": (ctypes.c_char_p, [_P]),
    "fde_num_levels": (_I, [_P]),
    "fde_level_size": (_I, [_P, _I, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "fde_apply": (_I, [_P, _I, _I, _P, _P]),
    "fde_residual": (_I, [_P, _I, _I, _P, _P, _P]),
    "fde_smooth": (_I, [_P, _I, _I, _P, _P, _I]),
    "fde_restrict": (_I, [_P, _I, _I, _P, _P]),
    "fde_prolong": (_I, [_P, _I, _I, _P, _P]),
    "fde_coarse_solve": (_I, [_P, _P, _P]),
    "fde_vcycle": (_I, [_P, _P, _P]),
    "fde_level_diag": (_I, [_P, _I, _P]),
    "fde_sync": (_I, [_P]),
    "fde_profile_enable": (_I, [_P, ctypes.c_uint32]),
    "fde_profile_stride": (_I, [_P, _I]),
    "fde_profile_read": (_I, [_P, _I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "fde_profile_reset": (_I, [_P]),
    "fde_footprint": (ctypes.c_size_t, [ctypes.POINTER(fde_problem)]),
    "fde_batch_create": (_I, [ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "fde_batch_destroy": (None, [_P]),
    "fde_batch_set_grouping": (_I, [_P, _I32, _I32]),
    "fde_batch_set_policy": (_I, [_P, _I32, _I32, _I32]),
    "fde_batch_set_lanes": (_I, [_P, _I32]),
    "fde_batch_admit": (_I, [_P, ctypes.POINTER(fde_problem), _P, _P, _P, _P, _P, _I32, _D, _I32,
                             ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_P)]),
    "fde_batch_step": (_I, [_P]),
    "fde_batch_poll": (_I, [_P, _I, _P, ctypes.POINTER(ctypes.c_int64)]),
    "fde_batch_cancel": (_I, [_P, _I]),
    "fde_batch_info": (_I, [_P, ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_size_t)]),
    "fde_apply_noalloc": (_I, [ctypes.POINTER(fde_problem), _P, _P, _P, _P, _P, _P, _P]),
}

_lib: Optional[ctypes.CDLL] = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libfde.so and declare its signatures.  Raises if the library is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libfde.so not found at {path}; build it with "
                           "`python -m paper_1706_06844_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
