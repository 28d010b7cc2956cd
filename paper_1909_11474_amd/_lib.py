"""ctypes loader for libmt_tersoff.so: argument marshalling only.

The shared library must have been built (``paper_1909_11474_amd.build``);
loading fails loudly otherwise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmt_tersoff.so")

MT_OK = 0
MT_EINVAL = -1
MT_ENOMEM = -2
MT_EHIP = -3
MT_ENBR_OVERFLOW = -4
MT_ENOREF = -5
MT_ESTATE = -6
MT_ECOINCIDENT = -7

MT_FP64 = 0
MT_FP32_ACC64 = 1
MT_BATCHED = 0
MT_PLAIN = 1

MT_MAX_NBR = 16
MT_MAX_BATCHED_ATOMS = 512
MT_NOALLOC_SCRATCH_BYTES = 32 << 20

_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double

# name -> (restype, argtypes); the same names as include/mt_tersoff.h
SIGNATURES = {
    "mt_set_create": (_i, [ctypes.POINTER(_vp), _i, ctypes.POINTER(ctypes.c_int64), _vp, _vp,
                           _d, _d, _i, _vp]),
    "mt_set_attach_reference": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "mt_set_destroy": (_i, [_vp]),
    "mt_set_stats": (_i, [_vp, ctypes.POINTER(ctypes.c_int64)]),
    "mt_set_neighbors": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "mt_set_update_positions": (_i, [_vp, _vp, _vp]),
    "mt_set_list_skin": (_i, [_vp, _d, _vp]),
    "mt_set_update_geometry": (_i, [_vp, _vp, _vp]),
    "mt_md_max_disp": (_i, [_i, _vp, _vp, _vp, _vp]),
    "mt_md_kick": (_i, [_i, _vp, _vp, _vp, _vp, ctypes.POINTER(_d), _vp, _d, _vp]),
    "mt_md_drift": (_i, [_i, _vp, _vp, _d, _vp]),
    "mt_md_scale": (_i, [_i, _vp, _d, _vp]),
    "mt_md_kinetic": (_i, [_i, _vp, _vp, _vp, _vp]),
    "tersoff_eval": (_i, [_vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tersoff_eval_tf": (_i, [_vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fitness_eval": (_i, [_vp, _vp, _i, ctypes.POINTER(_d), _i, _i, _vp, _vp]),
    "fitness_eval_tf": (_i, [_vp, _vp, _i, ctypes.POINTER(_d), _i, _i, _vp, _vp]),
    "fitness_grad": (_i, [_vp, _vp, _i, ctypes.POINTER(_d), _i, _vp, _vp, _vp]),
    "fitness_grad_tf": (_i, [_vp, _vp, _i, ctypes.POINTER(_d), _i, _vp, _vp, _vp]),
    "fitness_terms": (_i, [_vp, _vp, _i, _vp, _vp, _vp, _vp]),
    "fitness_eval_noalloc": (_i, [_vp, _vp, _i, ctypes.POINTER(_d), _i, _vp, _vp]),
    "mt_autotune": (_i, [_vp, _i, _i, ctypes.c_char_p]),
    "mt_profile_enable": (_i, [_vp, _i]),
    "mt_profile_read": (_i, [_vp, ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_int64)]),
    "mt_profile_fitness_kernels": (_i, [_vp, _vp, _i, _i, _i, _i, ctypes.POINTER(_d),
                                        ctypes.POINTER(ctypes.c_int64), _vp]),
    "mt_profile_fitness_launches": (_i, [_vp, _vp, _i, _i, _i, _i, _i, ctypes.POINTER(_d),
                                         ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i), _vp]),
    "mt_last_error": (ctypes.c_char_p, []),
    "mt_version": (ctypes.c_char_p, []),
}

_lib = None


class MTError(RuntimeError):
    def __init__(self, code: int, where: str, message: str):
        super().__init__(f"{where} failed with status {code}: {message}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load the library (once) and declare every exported signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_1909_11474_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int, where: str):
    if code != MT_OK:
        msg = load().mt_last_error().decode(errors="replace")
        raise MTError(code, where, msg)
