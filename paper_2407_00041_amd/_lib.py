"""ctypes binding of libwdirac.so (argument marshalling only).

The library must have been built (``python -m paper_2407_00041_amd.build``);
there is no fallback: loading fails loudly when the shared object is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libwdirac.so")

F64, F32, F16S = 0, 1, 2
ANTIPERIODIC_T, WITH_F32, WITH_F16, COMPRESS_LINKS, COMPRESS_CLOVER, EVEN_ODD = 1, 2, 4, 8, 16, 32
OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, ENOTCONV, ENONFINITE = 0, -1, -2, -3, -4, 1, 2
FGMRES_F64, FGMRES_MIXED_F32, FGMRES_MIXED_F16S, FGMRES_SAP, FGMRES_AMG = 0, 1, 2, 3, 4
AMG_TEST_VECTORS, AMG_INTERPOLATION, AMG_COARSE_OPERATOR = 0, 1, 2
FGMRES_HIST_MAX = 4096

_P = ctypes.c_void_p
_I = ctypes.c_int


class DiracBatch(ctypes.Structure):
    _fields_ = [("out", _P), ("inp", _P), ("nrhs", _I)]


class SapParams(ctypes.Structure):
    _fields_ = [("block", _I * 4), ("cycles", _I), ("mr_iters", _I), ("additive", _I), ("prec", _I)]


class AmgParams(ctypes.Structure):
    _fields_ = [("agg", _I * 4), ("ntv", _I), ("init_iters", _I), ("setup_iters", _I), ("smoother", SapParams),
                ("coarse_restart", _I), ("coarse_maxit", ctypes.c_longlong), ("coarse_tol", ctypes.c_double),
                ("prec", _I)]


class FgmresParams(ctypes.Structure):
    _fields_ = [("restart", _I), ("tol", ctypes.c_double), ("maxit", ctypes.c_longlong),
                ("mode", _I), ("inner_restart", _I), ("inner_tol", ctypes.c_double),
                ("inner_maxit", _I), ("graph", _I), ("wave", _I), ("schur", _I), ("sap", SapParams),
                ("amg", _P)]


class FgmresStats(ctypes.Structure):
    _fields_ = [("applies", ctypes.c_longlong), ("inner_applies", ctypes.c_longlong),
                ("restarts", ctypes.c_longlong), ("converged", _I), ("breakdown", _I),
                ("nonfinite", _I), ("wave", _I), ("true_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("seconds_apply", ctypes.c_double), ("seconds_precond", ctypes.c_double),
                ("seconds_ortho", ctypes.c_double),
                ("nhist", _I), ("hist", ctypes.c_double * FGMRES_HIST_MAX)]


# symbol -> (restype, argtypes); every entry point declared in include/wdirac.h
SIGNATURES = {
    "dirac_last_error": (ctypes.c_char_p, []),
    "dirac_version": (ctypes.c_char_p, []),
    "dirac_create": (_I, [ctypes.POINTER(_P), _P, _P, _P, ctypes.c_double, ctypes.c_double,
                          ctypes.c_uint]),
    "dirac_destroy": (_I, [_P]),
    "dirac_volume": (ctypes.c_longlong, [_P]),
    "dirac_field_bytes": (ctypes.c_size_t, [_P, _I, _I]),
    "dirac_apply": (_I, [_P, _P, _P, _I, _I, _P]),
    "dirac_apply_adjoint": (_I, [_P, _P, _P, _I, _I, _P]),
    "dirac_apply_batched": (_I, [_P, ctypes.POINTER(DiracBatch), _I, _I, _I, _P]),
    "dirac_tune_set": (_I, [ctypes.c_char_p, _I]),
    "dirac_tune_get": (_I, [ctypes.c_char_p, ctypes.POINTER(_I)]),
    "dirac_autotune": (_I, [_P, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_double), _P]),
    "dirac_tune_clear": (_I, []),
    "dirac_pack": (_I, [_P, _P, _P, _I, _I, _P]),
    "dirac_unpack": (_I, [_P, _P, _P, _I, _I, _P]),
    "dirac_clover_term": (_I, [_P, _P, _P, _P]),
    "fgmres_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.POINTER(FgmresParams), _I]),
    "fgmres_solve": (_I, [_P, _P, _P, _I, ctypes.POINTER(FgmresParams),
                          ctypes.POINTER(FgmresStats), _P, ctypes.c_size_t, _P]),
    "dirac_force_workspace_bytes": (ctypes.c_size_t, [_P]),
    "dirac_sap_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.POINTER(SapParams), _I]),
    "dirac_sap": (_I, [_P, _P, _P, _I, ctypes.POINTER(SapParams), _P, ctypes.c_size_t, _P]),
    "dirac_parity_field_bytes": (ctypes.c_size_t, [_P, _I, _I]),
    "dirac_parity_split": (_I, [_P, _P, _P, _P, _I, _I, _P]),
    "dirac_parity_merge": (_I, [_P, _P, _P, _P, _I, _I, _P]),
    "dirac_apply_schur": (_I, [_P, _P, _P, _P, _I, _I, _I, _P]),
    "dirac_apply_schur_noalloc": (_I, [_P, _P, _P, _I, _I, _I, _P]),
    "dirac_schur_prepare": (_I, [_P, _P, _P, _P, _P, _I, _I, _P]),
    "dirac_schur_reconstruct": (_I, [_P, _P, _P, _P, _I, _I, _P]),
    "dirac_force": (_I, [_P, _P, _P, _P, _I, _I, _P, ctypes.c_size_t, _P]),
    "dirac_amg_create": (_I, [ctypes.POINTER(_P), _P, ctypes.POINTER(AmgParams), _P, _P]),
    "dirac_amg_destroy": (_I, [_P]),
    "dirac_amg_sizes": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_longlong)]),
    "dirac_amg_restrict": (_I, [_P, _P, _P, _I, _P]),
    "dirac_amg_prolong": (_I, [_P, _P, _P, _I, _P]),
    "dirac_amg_coarse_apply": (_I, [_P, _P, _P, _I, _P]),
    "dirac_amg_coarse_solve": (_I, [_P, _P, _P, ctypes.POINTER(ctypes.c_longlong), _P]),
    "dirac_amg_precond": (_I, [_P, _P, _P, _I, _P]),
    "dirac_amg_export": (_I, [_P, _I, _P, _P]),
}

_lib = None


def load():
    """Load libwdirac.so and declare every signature (raises if not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(f"{SO_PATH} is missing: build it with "
                               "`python -m paper_2407_00041_amd.build` (no CPU fallback exists)")
        lib = ctypes.CDLL(SO_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class WdiracError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load().dirac_last_error().decode()
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


def check(code: int, where: str) -> int:
    if code < 0:
        raise WdiracError(code, where)
    return code
