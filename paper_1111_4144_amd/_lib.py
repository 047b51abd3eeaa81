"""ctypes binding of libcholinv.so (the C-ABI declared in include/cholinv.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C-ABI.  There is no fallback: if the library has not been
built, loading it raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcholinv.so")

CI_F32, CI_F64, CI_C64, CI_C128 = 0, 1, 2, 3
CI_METHOD_CHOL, CI_METHOD_LDL = 0, 1
CI_III_A, CI_III_B, CI_IV_SAME = 0, 1, 2
CI_PLAIN, CI_MIXED = 0, 1
CI_FN_FACTOR, CI_FN_INVERSE, CI_FN_BATCHED, CI_FN_NONHERM = 0, 1, 2, 3
CI_ERR_UNSUPPORTED = -2000
CI_ERR_WORKSPACE = -2001
CI_ERR_NOALLOC_LIMIT = -2002
CI_NOALLOC_MAX_BATCH = 2097152
CI_ERR_LAUNCH = -1000
CI_SMALL_NMAX = 64

# Every symbol include/cholinv.h declares.
EXPORTS = ("chol_factor", "ldl_factor", "chol_solve", "chol_inverse", "chol_inverse_batched",
           "chol_inverse_batched_noalloc", "chol_inverse_nonherm", "chol_inverse_q15", "chol_inverse_compare",
           "chol_inverse_q15_compare", "chol_inverse_backward", "chol_workspace_size",
           "chol_status_string", "chol_version",
           "chol_autotune", "chol_tuned_engine", "chol_tune_set", "chol_autotune_varlen",
           "chol_autotune_clear")


class ci_opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("ns_steps", ctypes.c_int32), ("fill_lower", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t
_lib = None


class CholinvError(RuntimeError):
    def __init__(self, fn, code):
        self.code = code
        super().__init__("%s failed: %s (code %d)" % (fn, status_string(code), code))


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcholinv.so is not built; run `python -m paper_1111_4144_amd.build` "
                           "(or __graft_entry__.build()) first")
    L = ctypes.CDLL(LIB_PATH)
    L.chol_factor.argtypes = [_i32, _i64, _i64, _vp, _i64, _i64, _vp, _vp, _sz, _vp]
    L.ldl_factor.argtypes = [_i32, _i64, _i64, _vp, _i64, _i64, _vp, _vp, _vp]
    L.chol_solve.argtypes = [_i32, _i32, _i64, _i64, _i64, _vp, _i64, _i64, _vp, _vp, _i64, _i64,
                             _vp, _i64, _i64, _vp]
    L.chol_inverse.argtypes = [_i32, _i64, _vp, _i64, _vp, _i64, ctypes.POINTER(ci_opts), _vp,
                               _sz, _vp, _vp]
    L.chol_inverse_batched.argtypes = [_i32, _i64, _i64, _vp, _vp, _i64, _vp, _i64, _vp, _i64,
                                       ctypes.POINTER(ci_opts), _vp, _sz, _vp, _vp]
    L.chol_inverse_batched_noalloc.argtypes = [_i32, _i64, _i64, _vp, _vp, _i64, _vp, _i64, _vp,
                                               _i64, ctypes.POINTER(ci_opts), _vp, _vp]
    L.chol_inverse_nonherm.argtypes = [_i32, _i64, _i64, _vp, _i64, _vp, ctypes.POINTER(ci_opts),
                                       _vp, _sz, _vp, _vp]
    L.chol_inverse_q15.argtypes = [_i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp]
    L.chol_inverse_compare.argtypes = [_i32, _i32, _i32, _i64, _i64, _vp, _i64, _vp, _vp, _vp]
    L.chol_inverse_q15_compare.argtypes = [_i32, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp]
    L.chol_inverse_backward.argtypes = [_i32, _i64, _i64, _vp, _vp, _vp, _i64, _vp]
    L.chol_workspace_size.argtypes = [_i32, _i32, _i64, _i64, ctypes.POINTER(ci_opts)]
    L.chol_workspace_size.restype = _sz
    L.chol_status_string.argtypes = [_i32]
    L.chol_status_string.restype = ctypes.c_char_p
    L.chol_version.restype = ctypes.c_char_p
    L.chol_autotune.argtypes = [_i32, ctypes.POINTER(ci_opts), _i32, _i32, _i64, ctypes.c_char_p, _vp]
    L.chol_tuned_engine.argtypes = [_i32, ctypes.POINTER(ci_opts), _i32]
    L.chol_tune_set.argtypes = [_i32, ctypes.POINTER(ci_opts), _i32, _i32]
    L.chol_autotune_varlen.argtypes = [_i32, ctypes.POINTER(ci_opts), _i64, _vp, _vp, _i64, _vp,
                                       _vp, _vp, _sz, _vp]
    L.chol_autotune_varlen.restype = _i32
    L.chol_tune_set.restype = _i32
    L.chol_autotune_clear.argtypes = []
    L.chol_autotune_clear.restype = None
    for fn in ("chol_factor", "ldl_factor", "chol_solve", "chol_inverse", "chol_inverse_batched",
               "chol_inverse_batched_noalloc", "chol_inverse_nonherm", "chol_inverse_q15", "chol_inverse_compare",
               "chol_inverse_q15_compare", "chol_inverse_backward"):
        getattr(L, fn).restype = _i32
    _lib = L
    return L


def status_string(code: int) -> str:
    return lib().chol_status_string(int(code)).decode()


def check(fn: str, code: int) -> None:
    if code != 0:
        raise CholinvError(fn, code)


def make_opts(method="chol", precision="plain", ns_steps=0, fill_lower=True) -> ci_opts:
    m = {"chol": CI_METHOD_CHOL, "ldl": CI_METHOD_LDL}[method] if isinstance(method, str) else int(method)
    p = {"plain": CI_PLAIN, "mixed": CI_MIXED}[precision] if isinstance(precision, str) else int(precision)
    return ci_opts(m, p, int(ns_steps), int(bool(fill_lower)))
