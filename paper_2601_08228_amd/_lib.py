"""ctypes loader for libwprod.so (the HIP library); no computation happens here.

torch is imported first so that the HIP runtime it ships is the one the
library binds to (both carry the soname libamdhip64.so.7): device pointers and
streams from torch are then valid inside the library.
"""

import ctypes
import os

import torch  # noqa: F401  (must be loaded before the library, see above)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwprod.so")

# Status codes and enums of include/wprod.h.
WP_OK = 0
WP_ENOCONV = -7
WP_ESCRATCH = -8
WP_F64 = 0
WP_F32 = 1
GEMM_MODES = {"native": 0, "bf16": 1, "bf16x3": 2}

_c_i64 = ctypes.c_int64
_c_int = ctypes.c_int
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t

# Exported functions: name -> (restype, argtypes).
SIGNATURES = {
    "w_status_string": (ctypes.c_char_p, [_c_int]),
    "w_version": (_c_int, []),
    "w_transform": (_c_int, [_vp, _vp, _c_i64, _c_i64, _c_i64, _c_int, _c_int, _vp]),
    "w_itransform": (_c_int, [_vp, _vp, _c_i64, _c_i64, _c_i64, _c_int, _c_int, _vp]),
    "w_transform_adj": (_c_int, [_vp, _vp, _c_i64, _c_i64, _c_i64, _c_int, _c_int, _vp]),
    "w_itransform_adj": (_c_int, [_vp, _vp, _c_i64, _c_i64, _c_i64, _c_int, _c_int, _vp]),
    "w_transform_split": (_c_int, [_vp, _vp, _vp, _c_i64, _c_i64, _c_i64, _c_int, _vp]),
    "w_itransform_adj_split": (_c_int, [_vp, _vp, _vp, _c_i64, _c_i64, _c_i64, _c_int, _vp]),
    "w_face_product": (_c_int, [_vp, _vp, _vp, _c_i64, _c_i64, _c_i64, _c_i64, _c_int, _c_int,
                                _c_int, _vp]),
    "w_face_product_split": (_c_int, [_vp, _vp, _vp, _vp, _vp, _c_i64, _c_i64, _c_i64, _c_i64,
                                      _c_int, _c_int, _c_int, _vp]),
    "w_face_product_gemm": (_c_int, [_vp, _vp, _vp, _c_i64, _c_i64, _c_i64, _c_i64, _c_int,
                                     _c_int, _c_int, _c_int, _vp, _sz, _vp]),
    "w_face_product_workspace": (_sz, [_c_i64, _c_i64, _c_i64, _c_i64, _c_int, _c_int]),
    "w_product": (_c_int, [_vp, _vp, _vp, _c_i64, _c_i64, _c_i64, _c_i64, _c_int, _c_int, _c_int,
                           _c_int, _c_int, _vp, _sz, _vp]),
    "w_product_workspace": (_sz, [_c_i64, _c_i64, _c_i64, _c_i64, _c_int, _c_int, _c_int]),
    "w_product_noalloc": (_c_int, [_vp, _vp, _vp, _c_i64, _c_i64, _c_i64, _c_i64, _c_int, _c_int,
                                   _c_int, _c_int, _c_int, _vp]),
    "w_product_noalloc_scratch_bytes": (_sz, []),
    "w_svd": (_c_int, [_vp, _c_i64, _c_i64, _c_i64, _c_int, _c_int, _vp, _vp, _vp, _vp, _c_int,
                       _vp, _vp, _c_int, _vp, _sz, _vp]),
    "w_svd_workspace": (_sz, [_c_i64, _c_i64, _c_i64, _c_int, _c_int, _c_int]),
    "w_svd_timed": (_c_int, [_vp, _c_i64, _c_i64, _c_i64, _c_int, _c_int, _vp, _vp, _vp, _vp,
                             _c_int, _vp, _vp, _c_int, _vp, _sz, _vp, _vp, _vp]),
    "w_svd_sparse": (_c_int, [_vp, _c_i64, _c_i64, _c_i64, _c_int, _c_int, _vp, _vp, _vp, _vp,
                              _c_int, _vp, _vp, _c_int, _vp, _sz, _vp]),
    "w_svd_sparse_workspace": (_sz, [_c_i64, _c_i64, _c_i64, _c_int, _c_int, _c_int]),
    "w_pinv": (_c_int, [_vp, _vp, _c_i64, _c_i64, _c_i64, _c_int, _c_int, ctypes.c_double, _vp,
                        _c_int, _vp, _sz, _vp]),
    "w_pinv_workspace": (_sz, [_c_i64, _c_i64, _c_i64, _c_int, _c_int, _c_int]),
    "w_transform_scheme": (_c_int, [_vp, _vp, _c_i64, _c_i64, _c_i64, _c_int, _vp, _c_int, _c_int,
                                    _vp]),
    "w_transform_scheme_split": (_c_int, [_vp, _vp, _vp, _c_i64, _c_i64, _c_i64, _c_int, _vp,
                                          _c_int, _vp]),
    "w_product_scheme": (_c_int, [_vp, _vp, _vp, _c_i64, _c_i64, _c_i64, _c_i64, _c_int, _vp,
                                  _c_int, _c_int, _c_int, _c_int, _vp, _sz, _vp]),
    "w_product_scheme_workspace": (_sz, [_c_i64, _c_i64, _c_i64, _c_i64, _c_int, _c_int, _c_int]),
}

_lib = None


def load():
    """Load libwprod.so once; raise ImportError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                "libwprod.so is not built (expected at %s); run "
                "`python -m paper_2601_08228_amd.build`" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class WprodError(RuntimeError):
    def __init__(self, fn, status):
        msg = load().w_status_string(status).decode()
        super().__init__("%s failed: %s (status %d)" % (fn, msg, status))
        self.status = status


def check(fn, status):
    if status != WP_OK:
        raise WprodError(fn, status)
