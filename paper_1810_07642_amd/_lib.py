"""ctypes loader of libtflbm.so and declarations of its C ABI (include/tflbm.h).

The library is the only compute path: if it is missing or fails to load this
module raises, there is no fallback.
"""
import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtflbm.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "tflbm.h")

TFLBM_OK = 0
TFLBM_EINVAL = -1
TFLBM_EUNSTABLE = -2
TFLBM_EHIP = -3
TFLBM_ENONFINITE = -4
TFLBM_ESTATE = -5

PREC = {"fp64": 0, "fp32": 1, "fp16s": 2}


class Params(ctypes.Structure):
    """Mirror of ``tflbm_params``."""
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("prec", ctypes.c_int32),
        ("n_exp", ctypes.c_int32), ("m_exp", ctypes.c_int32), ("fp16_scale_log2", ctypes.c_int32),
        ("gamma_field", ctypes.c_int32),
        ("tau", ctypes.c_double), ("gamma", ctypes.c_double), ("g", ctypes.c_double),
        ("hstar", ctypes.c_double), ("delta", ctypes.c_double), ("ax", ctypes.c_double),
        ("ay", ctypes.c_double), ("theta0", ctypes.c_double), ("href", ctypes.c_double),
    ]


_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dp = ctypes.c_void_p  # device double* passed as an address

SIGNATURES = {
    "tflbm_version": (ctypes.c_char_p, []),
    "tflbm_strerror": (ctypes.c_char_p, [_int]),
    "tflbm_last_error": (ctypes.c_char_p, [_vp]),
    "tflbm_default_params": (None, [ctypes.POINTER(Params)]),
    "tflbm_check_params": (_int, [ctypes.POINTER(Params)]),
    "tflbm_create": (_int, [ctypes.POINTER(Params), ctypes.POINTER(_vp)]),
    "tflbm_destroy": (None, [_vp]),
    "tflbm_workspace_bytes": (_sz, [_vp]),
    "tflbm_bind": (_int, [_vp, _vp, _sz]),
    "tflbm_init": (_int, [_vp, _dp, _dp, _vp]),
    "tflbm_init_fields": (_int, [_vp, _dp, _dp, _dp, _vp]),
    "tflbm_step": (_int, [_vp, _i64, _vp]),
    "tflbm_step_count": (_i64, [_vp]),
    "tflbm_step_graphs": (_int, [_vp]),
    "tflbm_steps_per_pass": (_int, [_vp]),
    "tflbm_read": (_int, [_vp, _dp, _dp, _dp, _vp]),
    "tflbm_mass": (_int, [_vp, ctypes.POINTER(ctypes.c_double), _vp]),
    "tflbm_mass_noalloc": (_int, [_vp, _dp, _vp]),
    "tflbm_check": (_int, [_vp, _vp]),
    "tflbm_term_norms": (_int, [_vp, ctypes.POINTER(ctypes.c_double), _vp]),
    "tflbm_state_bytes": (_sz, [_vp]),
    "tflbm_state_save": (_int, [_vp, _vp, _vp]),
    "tflbm_state_load": (_int, [_vp, _vp, _i64, _vp]),
    "tflbm_capture_bytes": (_sz, [_vp]),
    "tflbm_step_capture": (_int, [_vp, _i64, _vp, _vp]),
    "tflbm_adj_bytes": (_sz, [_vp]),
    "tflbm_adj_seed": (_int, [_vp, _vp, _dp, _vp]),
    "tflbm_adj_step": (_int, [_vp, _vp, _vp, _vp]),
    "tflbm_adj_steps": (_int, [_vp, _vp, _vp, ctypes.c_int64, _vp]),
    "tflbm_adj_finish": (_int, [_vp, _vp, _dp, _dp, _dp, _dp, _vp]),
}

_lib = None


def header_functions():
    """Names of the functions declared in include/tflbm.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tflbm_[a-z0-9_]+)\s*\(", text)))


def load():
    """Load libtflbm.so (once) and declare its functions; raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1810_07642_amd.build` "
            "(the HIP library is the only compute path)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class TFLBMError(RuntimeError):
    def __init__(self, code, where, detail=""):
        lib = load()
        msg = f"{where}: {lib.tflbm_strerror(code).decode()} ({code})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)
        self.code = code


def check(code, where, handle=None):
    if code != TFLBM_OK:
        detail = ""
        if handle is not None and code == TFLBM_EHIP:
            detail = load().tflbm_last_error(handle).decode()
        raise TFLBMError(code, where, detail)
    return code
