"""FP64 CPU oracle for Cholesky/LDL-based inversion of Hermitian positive-definite
matrices (Krishnamoorthy & Menon, arXiv:1111.4144).

TEST INFRASTRUCTURE ONLY.  This package is imported by the tests, by the smoke
check and by the CPU-baseline leg of the benchmark; nothing in the GPU library
or its Python binding imports it.  It shares no code with the GPU path.

The arithmetic lives in ``cholinv_oracle.c`` (plain single-threaded C, FP64,
``-ffp-contract=off``); this module only marshals numpy arrays through ctypes.
Real inputs (float32/float64) run the real instantiation, complex inputs
(complex64/complex128) the complex one; everything is upcast to FP64 exactly
before the call, so the oracle inverts the stored values.

Functions and the passages they follow:

* ``chol``          Section II, eqs. (3)-(4)
* ``ldl``           Section II.A, eqs. (10)-(11)
* ``chol_solve``    Section II, eqs. (5)-(7)
* ``ldl_solve``     Section II.A, eqs. (12)-(14)
* ``inv_prop``      Section IV.A (method "chol", eq. 24) / IV.B ("ldl", eq. 29)
* ``inv_prop_all_cores``  the same routine over a stack, matrices shared among threads
* ``inv_eqsolve``   Section III.A, eq. (15)
* ``inv_tri``       Section III.B, eqs. (16)-(19)
* ``inv_nonherm``   Section III.C
* ``grad``          gA = -X Gh X, the gradient of Re<G, A^{-1}> on Hermitian A
* ``ns_step``       one Newton-Schulz refinement step X + X(I - AX)
* ``gauss_jordan``  brute-force inverse, an independent route
* ``herm_eig`` / ``kappa2``  cyclic Jacobi eigenvalues / 2-norm condition
* ``count_mults``   the multiply counter behind Table 1's operation counts
"""
from __future__ import annotations

import contextlib
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcholinv_oracle.so")
_lib = None

_i32 = ctypes.c_int
_i64 = ctypes.c_long
_vp = ctypes.c_void_p
METHODS = {"chol": 0, "ldl": 1}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    for sfx in ("d", "z"):
        getattr(lib, "or_chol_" + sfx).argtypes = [_i32, _vp, _i64, _vp, _i64]
        getattr(lib, "or_ldl_" + sfx).argtypes = [_i32, _vp, _i64, _vp, _i64, _vp, _i32]
        getattr(lib, "or_chol_solve_" + sfx).argtypes = [_i32, _vp, _i64, _vp, _vp]
        getattr(lib, "or_ldl_solve_" + sfx).argtypes = [_i32, _vp, _i64, _vp, _vp, _vp]
        getattr(lib, "or_inv_prop_" + sfx).argtypes = [_i32, _i32, _vp, _i64, _vp, _i64, _i32]
        getattr(lib, "or_inv_eqsolve_" + sfx).argtypes = [_i32, _i32, _vp, _i64, _vp, _i64]
        getattr(lib, "or_inv_tri_" + sfx).argtypes = [_i32, _vp, _i64, _vp, _i64]
        getattr(lib, "or_grad_" + sfx).argtypes = [_i32, _vp, _vp, _vp]
        getattr(lib, "or_ns_step_" + sfx).argtypes = [_i32, _vp, _i64, _vp, _vp]
        getattr(lib, "or_gauss_jordan_" + sfx).argtypes = [_i32, _vp, _i64, _vp, _i64]
        getattr(lib, "or_inv_prop_batched_" + sfx).argtypes = [_i32, _i64, _i32, _vp, _vp, _vp]
        getattr(lib, "or_inv_prop_varlen_" + sfx).argtypes = [_i32, _i64, _vp, _vp, _vp, _vp, _vp]
        getattr(lib, "or_inv_prop_batched_omp_" + sfx).argtypes = [_i32, _i64, _i32, _vp, _vp,
                                                                   _vp]
        getattr(lib, "or_grad_batched_" + sfx).argtypes = [_i64, _i32, _vp, _vp, _vp]
        for name in ("chol", "ldl", "inv_prop", "inv_eqsolve", "inv_tri", "gauss_jordan"):
            getattr(lib, "or_%s_%s" % (name, sfx)).restype = _i32
    lib.or_inv_q15.argtypes = [_i32, _vp, _vp, _vp, _vp]
    lib.or_inv_q15.restype = _i32
    lib.or_inv_q15_batched.argtypes = [_i64, _i32, _vp, _vp, _vp, _vp, _vp]
    lib.or_inv_q15_cmp_batched.argtypes = [_i32, _i64, _i32, _vp, _vp, _vp, _vp, _vp]
    lib.or_inv_nonherm_z.argtypes = [_i32, _vp, _vp]
    lib.or_inv_nonherm_z.restype = _i32
    lib.or_herm_eig_z.argtypes = [_i32, _vp, _i64, _vp]
    lib.or_herm_eig_z.restype = _i32
    lib.or_count_get.restype = ctypes.c_ulonglong
    lib.or_set_threads.argtypes = [_i32]
    lib.or_max_threads.restype = _i32
    _lib = lib
    return lib


def _prep(a):
    """Exact FP64 copy (C-contiguous) and the type suffix."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return np.ascontiguousarray(a, dtype=np.complex128), "z"
    return np.ascontiguousarray(a, dtype=np.float64), "d"


def _p(arr):
    return arr.ctypes.data_as(_vp)


def _method(method):
    return METHODS[method] if isinstance(method, str) else int(method)


# --------------------------------------------------------------------------
# Section II: factorisations and solves
# --------------------------------------------------------------------------
def chol(a):
    """R with A = R^* R (eqs. 3-4). Returns (R, info); info = 1-based failing row."""
    a, s = _prep(a)
    n = a.shape[-1]
    r = np.zeros_like(a)
    info = getattr(_load(), "or_chol_" + s)(n, _p(a), n, _p(r), n)
    return r, int(info)


def ldl(a, require_pos=False):
    """(R unit upper, d, info) with A = R^* D R (eqs. 10-11)."""
    a, s = _prep(a)
    n = a.shape[-1]
    r = np.zeros_like(a)
    d = np.zeros(n, np.float64)
    info = getattr(_load(), "or_ldl_" + s)(n, _p(a), n, _p(r), n, _p(d), int(require_pos))
    return r, d, int(info)


def chol_solve(r, y):
    """x with R^* R x = y (eqs. 5-7)."""
    r, s = _prep(r)
    y = np.ascontiguousarray(y, dtype=r.dtype)
    x = np.zeros_like(y)
    getattr(_load(), "or_chol_solve_" + s)(r.shape[-1], _p(r), r.shape[-1], _p(y), _p(x))
    return x


def ldl_solve(r, d, y):
    """x with R^* D R x = y (eqs. 12-14)."""
    r, s = _prep(r)
    d = np.ascontiguousarray(d, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=r.dtype)
    x = np.zeros_like(y)
    getattr(_load(), "or_ldl_solve_" + s)(r.shape[-1], _p(r), r.shape[-1], _p(d), _p(y), _p(x))
    return x


# --------------------------------------------------------------------------
# Sections III and IV: inversions
# --------------------------------------------------------------------------
def inv_prop(a, method="chol", fill_lower=True):
    """Proposed inversion (Section IV). a: (n, n) or (B, n, n). Returns (X, info)."""
    a, s = _prep(a)
    lib = _load()
    n = a.shape[-1]
    if a.ndim == 2:
        x = np.zeros_like(a)
        info = getattr(lib, "or_inv_prop_" + s)(_method(method), n, _p(a), n, _p(x), n,
                                                int(fill_lower))
        return x, int(info)
    flat = a.reshape(-1, n, n)
    x = np.zeros_like(flat)
    info = np.zeros(flat.shape[0], np.int32)
    getattr(lib, "or_inv_prop_batched_" + s)(_method(method), flat.shape[0], n, _p(flat),
                                             _p(x), _p(info))
    return x.reshape(a.shape), info.reshape(a.shape[:-2])


def inv_prop_all_cores(a, threads, method="chol"):
    """inv_prop over a stack (B, n, n) with the matrices shared out among
    `threads` OpenMP threads (each matrix by the same single-threaded routine;
    the results are those of inv_prop). Returns (X, info)."""
    a, s = _prep(a)
    lib = _load()
    n = a.shape[-1]
    flat = a.reshape(-1, n, n)
    x = np.zeros_like(flat)
    info = np.zeros(flat.shape[0], np.int32)
    lib.or_set_threads(int(threads))
    getattr(lib, "or_inv_prop_batched_omp_" + s)(_method(method), flat.shape[0], n, _p(flat),
                                                 _p(x), _p(info))
    return x.reshape(a.shape), info.reshape(a.shape[:-2])


def build_flags():
    """The compiler and flags the oracle library is built with."""
    from . import build as _build
    return "gcc " + " ".join(_build.CFLAGS)


def inv_prop_varlen(packed, sizes, offsets, method="chol"):
    """Proposed inversion of a packed batch of dense matrices of order sizes[b]
    starting at element offsets[b]. Returns (packed X, info)."""
    a, s = _prep(packed)
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    x = np.zeros_like(a)
    info = np.zeros(sizes.shape[0], np.int32)
    getattr(_load(), "or_inv_prop_varlen_" + s)(_method(method), sizes.shape[0], _p(sizes),
                                                _p(offsets), _p(a), _p(x), _p(info))
    return x, info


def inv_eqsolve(a, method="chol"):
    """Section III.A equation-solving inversion. Returns (X, info)."""
    a, s = _prep(a)
    n = a.shape[-1]
    x = np.zeros_like(a)
    info = getattr(_load(), "or_inv_eqsolve_" + s)(_method(method), n, _p(a), n, _p(x), n)
    return x, int(info)


def inv_tri(a):
    """Section III.B triangular-operations inversion (Cholesky). Returns (X, info)."""
    a, s = _prep(a)
    n = a.shape[-1]
    x = np.zeros_like(a)
    info = getattr(_load(), "or_inv_tri_" + s)(n, _p(a), n, _p(x), n)
    return x, int(info)


def inv_nonherm(d):
    """Section III.C: D^{-1} = D^* (D D^*)^{-1} for a square D. Returns (D^{-1}, info)."""
    d = np.ascontiguousarray(d, dtype=np.complex128)
    out = np.zeros_like(d)
    info = _load().or_inv_nonherm_z(d.shape[-1], _p(d), _p(out))
    return out, int(info)


def inv_q15(q, variant="IV.A"):
    """Fixed-point form of the proposed inversion (eqs. 3-4 and Section IV.A in
    Q15 with Q30 sums, integer square root and rounded integer division; the
    format is this implementation's reading), or with variant "III.A" / "III.B"
    the Section III comparison methods in the same format (same factor, same
    output stage).  q: int16 [batch, n, n, 2] (re, im) standing for q / 2^15.
    Returns (x int16 [batch, n, n, 2], xexp, sat, info int32 [batch]) with
    A^{-1} ~ x 2^xexp."""
    q = np.ascontiguousarray(q, dtype=np.int16)
    if q.ndim == 3:
        q = q[None]
    batch, n = q.shape[0], q.shape[1]
    x = np.zeros_like(q)
    xexp = np.zeros(batch, np.int32)
    sat = np.zeros(batch, np.int32)
    info = np.zeros(batch, np.int32)
    if variant == "IV.A":
        _load().or_inv_q15_batched(batch, n, _p(q), _p(x), _p(xexp), _p(sat), _p(info))
    else:
        v = {"III.A": 0, "III.B": 1}[variant]
        _load().or_inv_q15_cmp_batched(v, batch, n, _p(q), _p(x), _p(xexp), _p(sat), _p(info))
    return x, xexp, sat, info


def dequant_q15(x, xexp):
    """complex128 values x 2^xexp of int16 (re, im) mantissas [batch, n, n, 2]."""
    x = np.asarray(x, np.float64)
    return (x[..., 0] + 1j * x[..., 1]) * np.ldexp(1.0, np.asarray(xexp))[:, None, None]


# --------------------------------------------------------------------------
# Gradient, refinement, independent routes
# --------------------------------------------------------------------------
def grad(x, g):
    """gA = -X Gh X with Gh = (G + G^H)/2 for full Hermitian X; (n,n) or (B,n,n)."""
    x, s = _prep(x)
    g = np.ascontiguousarray(g, dtype=x.dtype)
    n = x.shape[-1]
    ga = np.zeros_like(x)
    flat = x.reshape(-1, n, n)
    getattr(_load(), "or_grad_batched_" + s)(flat.shape[0], n, _p(x), _p(g), _p(ga))
    return ga


def ns_step(a, x):
    """One Newton-Schulz step X + X(I - A X), A rebuilt from its upper triangle."""
    a, s = _prep(a)
    x = np.ascontiguousarray(x, dtype=a.dtype)
    x1 = np.zeros_like(x)
    n = a.shape[-1]
    getattr(_load(), "or_ns_step_" + s)(n, _p(a), n, _p(x), _p(x1))
    return x1


def gauss_jordan(a):
    """Brute-force inverse of the Hermitian matrix given by a's upper triangle."""
    a, s = _prep(a)
    n = a.shape[-1]
    x = np.zeros_like(a)
    info = getattr(_load(), "or_gauss_jordan_" + s)(n, _p(a), n, _p(x), n)
    return x, int(info)


def herm_eig(a):
    """Increasing eigenvalues of the Hermitian matrix given by a's upper triangle."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    n = a.shape[-1]
    w = np.zeros(n, np.float64)
    rc = _load().or_herm_eig_z(n, _p(a), n, _p(w))
    if rc:
        raise RuntimeError("Jacobi eigenvalue iteration did not converge")
    return w


def kappa2(a):
    """2-norm condition number of a positive-definite Hermitian matrix."""
    w = herm_eig(a)
    return float(w[-1] / w[0])


@contextlib.contextmanager
def count_mults():
    """Count the multiplies inside the equations' sums: ``with count_mults() as c:``
    then ``c()`` returns the count so far."""
    lib = _load()
    lib.or_count_reset()
    yield lambda: int(lib.or_count_get())
