"""ctypes declarations of the C ABI in include/wqfd.h (libwqfd.so, built in-tree).

Loading fails loudly if the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwqfd.so")

WQ_OK, WQ_EINVAL, WQ_EGEOM, WQ_ESINGULAR, WQ_ENOMEM, WQ_EHIP, WQ_ENOCONV, WQ_EBREAKDOWN, WQ_ENONFINITE = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
WQ_F64, WQ_F32, WQ_BF16 = 1, 2, 4
WQ_K_IDENTITY, WQ_K_SCALAR, WQ_K_SYM6 = 0, 1, 6
WQ_FD_NOALLOC_BYTES = 32 << 20

ERROR_NAMES = {WQ_EINVAL: "WQ_EINVAL", WQ_EGEOM: "WQ_EGEOM", WQ_ESINGULAR: "WQ_ESINGULAR",
               WQ_ENOMEM: "WQ_ENOMEM", WQ_EHIP: "WQ_EHIP", WQ_ENOCONV: "WQ_ENOCONV",
               WQ_EBREAKDOWN: "WQ_EBREAKDOWN", WQ_ENONFINITE: "WQ_ENONFINITE"}

# every symbol include/wqfd.h declares: (name, restype, argtypes)
_vp, _i32p, _dp, _szp, _ip = C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_size_t), \
    C.POINTER(C.c_int)
SIGNATURES = [
    ("wq_setup", C.c_int, [C.c_int, _i32p, C.POINTER(C.c_void_p), _vp, C.c_int, _vp, C.c_int, _vp, C.c_size_t,
                           _szp, _vp, C.POINTER(C.c_void_p)]),
    ("wq_setup_nurbs", C.c_int, [C.c_int, _i32p, C.POINTER(C.c_void_p), _vp, _vp, C.c_int, _vp, C.c_int, _vp,
                                 C.c_size_t, _szp, _vp, C.POINTER(C.c_void_p)]),
    ("wq_setup_gauss", C.c_int, [C.c_int, _i32p, C.POINTER(C.c_void_p), _vp, C.c_int, _vp, C.c_int, _vp,
                                 C.c_size_t, _szp, _vp, C.POINTER(C.c_void_p)]),
    ("wq_dims", C.c_int, [_vp, _i32p, _i32p]),
    ("wq_quad_points", C.c_int, [_vp, _vp, _vp, _vp]),
    ("wq_detj", C.c_int, [_vp, _vp, _vp]),
    ("wq_set_coef", C.c_int, [_vp, C.c_int, _vp, _vp]),
    ("wq_apply", C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    ("wq_apply_T", C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    ("wq_apply_acc", C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    ("wq_set_alpha", C.c_int, [_vp, _vp, _vp]),
    ("wq_alpha_mean", C.c_int, [_vp, _dp, _vp]),
    ("wq_apply_mass", C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    ("wq_rhs", C.c_int, [_vp, _vp, _vp, _vp]),
    ("wq_grad_K", C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    ("wq_grad_f", C.c_int, [_vp, _vp, _vp, _vp]),
    ("wq_grad_Kf", C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    ("wq_grad_alpha", C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    ("wq_destroy", None, [_vp]),
    ("fd_setup", C.c_int, [C.c_int, _i32p, C.POINTER(C.c_void_p), C.c_int, _vp, C.c_size_t, _szp, _vp,
                           C.POINTER(C.c_void_p)]),
    ("fd_apply", C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    ("fd_apply_noalloc", C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    ("fd_set_shift", C.c_int, [_vp, C.c_double, _vp]),
    ("fd_factors", C.c_int, [_vp, C.c_int, _vp, _vp]),
    ("fd_destroy", None, [_vp]),
    ("wq_eval_setup", C.c_int, [C.c_int, _i32p, C.POINTER(C.c_void_p), _vp, _vp, C.c_int, _vp, C.c_size_t, _szp,
                                _vp, C.POINTER(C.c_void_p)]),
    ("wq_eval_dims", C.c_int, [_vp, _i32p, _i32p]),
    ("wq_eval_slab", C.c_int, [_vp, _vp, C.c_int, C.c_int, _vp, _vp, _vp, _vp, _vp]),
    ("wq_eval_destroy", None, [_vp]),
    ("krylov_ws_bytes", C.c_size_t, [_vp]),
    ("krylov_solve", C.c_int, [_vp, _vp, C.c_int, _vp, _vp, C.c_double, C.c_int, _vp, C.c_size_t, _ip, _dp,
                               _vp]),
    ("ir_ws_bytes", C.c_size_t, [_vp]),
    ("ir_solve", C.c_int, [_vp, _vp, C.c_int, _vp, _vp, C.c_double, C.c_double, C.c_int, C.c_int, _vp,
                           C.c_size_t, _ip, _ip, _dp, _vp]),
    ("ir_fallback_count", C.c_int, []),
    ("krylov_restart_count", C.c_int, []),
    ("wq_space_1d", C.c_int, [C.c_int, C.c_int, _vp, _i32p, _i32p, _vp, _vp, _vp]),
    ("fd_eig_1d", C.c_int, [C.c_int, C.c_int, _vp, _vp, _vp]),
    ("wq_geometry_host", C.c_int, [C.c_int, _i32p, C.POINTER(C.c_void_p), _vp, _vp, _vp, _vp, _vp]),
    ("wq_last_error", C.c_char_p, []),
    ("wq_version", C.c_char_p, []),
]

_lib = None


def lib():
    """The loaded library (raises if libwqfd.so is missing: build it first)."""
    global _lib
    if _lib is None:
        # torch's HIP runtime has the same soname as the one libwqfd.so needs;
        # importing torch first makes both share that single runtime (device
        # pointers and streams are then interchangeable).
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build the HIP library first "
                               "(python -m paper_1712_08565_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class WQError(RuntimeError):
    def __init__(self, code: int, func: str):
        msg = lib().wq_last_error().decode(errors="replace")
        super().__init__(f"{func} failed with {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code: int, func: str):
    if code != WQ_OK:
        raise WQError(code, func)
