"""ctypes view of libmag.so (the C ABI declared in include/mag.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly when the shared library is missing; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmag.so")

MAG_OK = 0
MAG_EINVAL = -1
MAG_ENOTPD = -2
MAG_ENOCONV = -3
MAG_ENOMEM = -4
MAG_EHIP = -5
MAG_EINTERNAL = -6

MAG_AUTO = 0
MAG_FP64_DENSE = 1
MAG_FP32_IR = 2
MAG_HODLR = 3
MAG_HSS = 4
MAG_FP64_CHOL = 5


class MagOpts(ctypes.Structure):
    _fields_ = [
        ("solver", ctypes.c_int32),
        ("max_outer", ctypes.c_int32),
        ("gmres_restart", ctypes.c_int32),
        ("max_gmres", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("inner_tol", ctypes.c_double),
        ("leaf", ctypes.c_int32),
        ("max_rank", ctypes.c_int32),
        ("oversample", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("inner_prec", ctypes.c_int32),
        ("diag", ctypes.c_int32),
        ("power_iters", ctypes.c_int32),
        ("reserved_", ctypes.c_int32),
    ]


class MagInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("outer_iters", ctypes.c_int32),
        ("gmres_iters", ctypes.c_int32),
        ("shifted", ctypes.c_int32),
        ("shift", ctypes.c_double),
        ("resid_inf", ctypes.c_double),
        ("magnitude", ctypes.c_double),
        ("min_w", ctypes.c_double),
        ("argmin_w", ctypes.c_int64),
        ("ms_tilegen", ctypes.c_double),
        ("ms_factor", ctypes.c_double),
        ("ms_refine", ctypes.c_double),
        ("ms_total", ctypes.c_double),
        ("ms_update", ctypes.c_double),
        ("flop_update", ctypes.c_double),
        ("n_update", ctypes.c_int32),
        ("solver", ctypes.c_int32),
        ("backward_err", ctypes.c_double),
        ("cond_est", ctypes.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MagTplusOpts(ctypes.Structure):
    _fields_ = [
        ("grid", ctypes.c_int32),
        ("max_extend", ctypes.c_int32),
        ("newton", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("lo_factor", ctypes.c_double),
        ("rtol", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("t_lo", ctypes.c_double),
        ("t_hi", ctypes.c_double),
    ]


class MagTplusInfo(ctypes.Structure):
    _fields_ = [
        ("t_plus", ctypes.c_double),
        ("t_bound", ctypes.c_double),
        ("d_min", ctypes.c_double),
        ("min_w", ctypes.c_double),
        ("t_bracket_lo", ctypes.c_double),
        ("t_bracket_hi", ctypes.c_double),
        ("solves", ctypes.c_int32),
        ("newton_steps", ctypes.c_int32),
        ("no_sign_change", ctypes.c_int32),
        ("status", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MagEigOpts(ctypes.Structure):
    _fields_ = [
        ("max_iter", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("rtol", ctypes.c_double),
    ]


class MagEigInfo(ctypes.Structure):
    _fields_ = [
        ("lambda_max", ctypes.c_double),
        ("lambda_min", ctypes.c_double),
        ("cond", ctypes.c_double),
        ("resid_max", ctypes.c_double),
        ("resid_min", ctypes.c_double),
        ("iters_max", ctypes.c_int32),
        ("iters_min", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("solve_steps", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_d = ctypes.c_double

# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "mag_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "mag_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int]),
    "mag_destroy": (None, [_vp]),
    "mag_set_stream": (ctypes.c_int, [_vp, _vp]),
    "mag_set_workspace_limit": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "mag_set_spin_limit": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "mag_workspace_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_uint64)]),
    "mag_opts_default": (None, [ctypes.POINTER(MagOpts)]),
    "mag_weighting": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, _vp, ctypes.POINTER(MagOpts),
                                     ctypes.POINTER(MagInfo)]),
    "mag_magnitude": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, ctypes.POINTER(_d), _vp,
                                     ctypes.POINTER(MagOpts), ctypes.POINTER(MagInfo)]),
    "mag_dmin": (ctypes.c_int, [_vp, _vp, _i64, _i32, ctypes.POINTER(_d)]),
    "mag_padded_size": (_i64, [_i64]),
    "mag_tune_panel": (ctypes.c_int, [_vp, _i64, _i32]),
    "mag_autotune": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, _i32, ctypes.POINTER(_i32),
                                    ctypes.POINTER(_d)]),
    "mag_tune_batch_group": (ctypes.c_int, [_vp, _i64, _i32]),
    "mag_autotune_batch": (ctypes.c_int, [_vp, _i32, _vp, ctypes.POINTER(_i64), _i32, ctypes.POINTER(_d), _i32,
                                          ctypes.POINTER(_i32), ctypes.POINTER(_d)]),
    "mag_tune_save": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "mag_tune_load": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "mag_zmatvec": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, _vp, _vp]),
    "mag_residual": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, _vp, _vp, ctypes.POINTER(_d)]),
    "mag_tile32": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, _vp]),
    "mag_factor32": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, _d, _vp, _vp, ctypes.POINTER(_i32)]),
    "mag_prec_apply": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "mag_factor64": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, _vp, _vp, ctypes.POINTER(_i32)]),
    "mag_chol64_solve": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "mag_dzmatvec": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, _vp, _vp]),
    "mag_residual_noalloc": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, _vp, _vp, ctypes.POINTER(_d)]),
    "mag_residual_noalloc_max_doubles": (ctypes.c_size_t, []),
    "mag_tplus_opts_default": (None, [ctypes.POINTER(MagTplusOpts)]),
    "mag_tplus": (ctypes.c_int, [_vp, _vp, _i64, _i32, ctypes.POINTER(MagTplusOpts), ctypes.POINTER(MagOpts),
                                 ctypes.POINTER(_d), _vp, ctypes.POINTER(MagTplusInfo)]),
    "mag_dwdt": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, _vp, _vp, ctypes.POINTER(MagOpts)]),
    "mag_eig_opts_default": (None, [ctypes.POINTER(MagEigOpts)]),
    "mag_weighting_zero": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp, ctypes.POINTER(MagOpts),
                                          ctypes.POINTER(MagInfo), ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "mag_eig_extremes": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, _vp, ctypes.POINTER(MagEigOpts),
                                        ctypes.POINTER(MagOpts), ctypes.POINTER(MagEigInfo)]),
    "mag_weighting_fwd": (ctypes.c_int, [_vp, _vp, _i64, _i32, _d, _vp, ctypes.POINTER(_vp),
                                         ctypes.POINTER(MagOpts), ctypes.POINTER(MagInfo)]),
    "mag_weighting_vjp": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _d, _vp, _d, _vp, _vp,
                                         ctypes.POINTER(_d), ctypes.POINTER(MagOpts)]),
    "mag_factor_free": (None, [_vp]),
    "mag_weighting_batch": (ctypes.c_int, [_vp, _i32, _vp, ctypes.POINTER(_i64), _i32, ctypes.POINTER(_d),
                                           _vp, ctypes.POINTER(_d), ctypes.POINTER(MagOpts),
                                           ctypes.POINTER(MagInfo)]),
    "mag_tplus_batch": (ctypes.c_int, [_vp, _i32, _vp, ctypes.POINTER(_i64), _i32, ctypes.POINTER(MagTplusOpts),
                                       ctypes.POINTER(MagOpts), ctypes.POINTER(_d), _vp,
                                       ctypes.POINTER(MagTplusInfo)]),
}

_lib = None


class MagError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = code
        msg = load().mag_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} (code {code})")


def load(path: str = LIB_PATH):
    """Load libmag.so and bind every declared symbol; raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"libmag.so not found at {path}; build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int, where: str) -> int:
    if code != MAG_OK:
        raise MagError(code, where)
    return code
