"""Host-side checks of the C-ABI (no GPU work is launched).

The library must load, export every symbol include/cholinv.h declares, and
reject invalid arguments with the documented codes before touching the GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1111_4144_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libcholinv.so not built")
    return L, L.lib()


def test_header_declares_exactly_the_exported_names():
    from paper_1111_4144_amd import _lib as L
    with open(os.path.join(ROOT, "include", "cholinv.h")) as f:
        hdr = f.read()
    declared = set(re.findall(r"^(?:int|size_t|void|const char\*)\s+(\w+)\(", hdr, re.M))
    assert declared == set(L.EXPORTS)


def test_library_exports_every_symbol():
    L, lib = _lib()
    for name in L.EXPORTS:
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.chol_version()


def test_argument_validation_codes():
    L, lib = _lib()
    o = L.make_opts()
    p = ctypes.c_void_p(0x1000)          # never dereferenced: validation fails first
    # bad dtype
    assert lib.chol_inverse_batched(9, 1, 4, None, None, 0, p, 16, p, 16, ctypes.byref(o), None,
                                    0, None, None) == -1
    # negative batch
    assert lib.chol_inverse_batched(2, -1, 4, None, None, 0, p, 16, p, 16, ctypes.byref(o), None,
                                    0, None, None) == -2
    # order beyond the batched limit
    assert lib.chol_inverse_batched(2, 1, 65, None, None, 0, p, 65 * 65, p, 65 * 65,
                                    ctypes.byref(o), None, 0, None, None) == -3
    # varlen without sizes
    assert lib.chol_inverse_batched(2, 3, 0, None, p, 8, p, 0, p, 0, ctypes.byref(o), None, 0,
                                    None, None) == -4
    # stride too small
    assert lib.chol_inverse_batched(2, 2, 4, None, None, 0, p, 15, p, 16, ctypes.byref(o), None,
                                    0, None, None) == -8
    # mixed precision on an FP64 type
    m = L.make_opts("chol", "mixed", 1)
    assert lib.chol_inverse_batched(3, 2, 4, None, None, 0, p, 16, p, 16, ctypes.byref(m), None,
                                    0, None, None) == -11
    # too many refinement steps / refinement without mixed precision
    bad = L.ci_opts(0, 1, 4, 1)
    assert lib.chol_inverse(0, 4, p, 4, p, 4, ctypes.byref(bad), None, 0, None, None) == -7
    bad = L.ci_opts(0, 0, 1, 1)
    assert lib.chol_inverse(0, 4, p, 4, p, 4, ctypes.byref(bad), None, 0, None, None) == -7
    # lda < n
    assert lib.chol_inverse(0, 4, p, 3, p, 4, None, None, 0, None, None) == -4
    # factor: stride < lda*n for a batch
    assert lib.chol_factor(0, 2, 4, p, 4, 15, None, None, 0, None) == -6
    # ldl without d
    assert lib.ldl_factor(0, 2, 4, p, 4, 16, None, None, None) == -7
    # backward: order too large
    assert lib.chol_inverse_backward(2, 1, 65, p, p, p, 65 * 65, None) == -3
    # solve: bad method, order beyond the batched limit, LDL without d,
    # ldb < nrhs, stride_b too small, in place with a different layout
    assert lib.chol_solve(0, 2, 1, 4, 1, p, 4, 16, None, p, 1, 4, p, 1, 4, None) == -2
    assert lib.chol_solve(0, 0, 1, 65, 1, p, 65, 0, None, p, 1, 65, p, 1, 65, None) == -4
    assert lib.chol_solve(0, 1, 2, 4, 1, p, 4, 16, None, p, 1, 4, p, 1, 4, None) == -9
    assert lib.chol_solve(0, 0, 2, 4, 3, p, 4, 16, None, p, 2, 12, p, 3, 12, None) == -11
    assert lib.chol_solve(0, 0, 2, 4, 2, p, 4, 16, None, p, 2, 7, p, 2, 8, None) == -12
    assert lib.chol_solve(0, 0, 2, 4, 2, p, 4, 16, None, p, 2, 8, p, 2, 9, None) == -13
    assert lib.chol_solve(0, 0, 0, 4, 1, None, 4, 16, None, None, 1, 4, None, 1, 4, None) == 0
    # non-Hermitian inverse: order beyond the batched limit, output = input,
    # workspace too small (two dense batches are needed)
    assert lib.chol_inverse_nonherm(0, 2, 65, p, 65 * 65, p, None, None, 0, None, None) == -3
    assert lib.chol_inverse_nonherm(0, 2, 4, p, 16, p, None, None, 0, None, None) == -6
    q = ctypes.c_void_p(0x2000)
    assert lib.chol_inverse_nonherm(0, 2, 4, p, 16, q, None, p, 255, None, None) == \
        L.CI_ERR_WORKSPACE
    assert lib.chol_workspace_size(L.CI_FN_NONHERM, 0, 2, 4, None) == 512
    # fixed point: order beyond 16, output = input, exponent array missing
    assert lib.chol_inverse_q15(2, 17, p, 17 * 17, q, q, None, None, None) == -2
    assert lib.chol_inverse_q15(2, 4, p, 16, p, q, None, None, None) == -5
    assert lib.chol_inverse_q15(2, 4, p, 16, q, None, None, None, None) == -6
    # comparison methods: unknown variant, LDL with III.B, order beyond 16
    assert lib.chol_inverse_compare(2, 3, 0, 2, 4, p, 16, q, None, None) == -2
    assert lib.chol_inverse_compare(2, L.CI_IV_SAME, 2, 2, 4, p, 16, q, None, None) == -3
    # the fixed-point comparison: unknown variant, order beyond 16
    assert lib.chol_inverse_q15_compare(L.CI_IV_SAME, 2, 4, p, 16, q, q, None, None, None) == -1
    assert lib.chol_inverse_q15_compare(L.CI_III_B, 2, 17, p, 17 * 17, q, q, None, None, None) == -3
    assert lib.chol_inverse_compare(2, L.CI_III_B, 1, 2, 4, p, 16, q, None, None) == -3
    assert lib.chol_inverse_compare(2, L.CI_III_A, 0, 2, 17, p, 17 * 17, q, None, None) == -5
    # empty work is a no-op
    assert lib.chol_inverse_batched(2, 0, 4, None, None, 0, None, 16, None, 16, None, None, 0,
                                    None, None) == 0
    assert L.status_string(-3) == "argument 3 is invalid"
    assert L.status_string(L.CI_ERR_WORKSPACE) == "workspace too small"


def test_workspace_sizes_are_host_only():
    L, lib = _lib()
    assert lib.chol_workspace_size(L.CI_FN_BATCHED, 2, 1000, 8, None) == 0


def test_tune_set_validates_engines():
    """chol_tune_set records only engines that can invert the combination (no
    GPU work: the table is host-side)."""
    L, lib = _lib()
    mixed = L.make_opts("chol", "mixed", 1)
    plain = L.make_opts()
    try:
        assert lib.chol_tune_set(L.CI_C64, ctypes.byref(mixed), 16, 6) == 0
        assert lib.chol_tuned_engine(L.CI_C64, ctypes.byref(mixed), 16) == 6
        assert lib.chol_tune_set(L.CI_C64, ctypes.byref(mixed), 16, 0) == 0
        assert lib.chol_tune_set(L.CI_C128, ctypes.byref(plain), 16, 6) == -4   # complex128
        assert lib.chol_tune_set(L.CI_C64, ctypes.byref(mixed), 8, 6) == -4     # order < 9
        assert lib.chol_tune_set(L.CI_C64, ctypes.byref(plain), 16, 5) == -4    # MFMA needs mixed
        assert lib.chol_tune_set(L.CI_C64, ctypes.byref(mixed), 16, 9) == -4    # no such engine
        assert lib.chol_tune_set(L.CI_C128, ctypes.byref(plain), 16, 7) == 0    # eight lanes
        assert lib.chol_tune_set(L.CI_F64, ctypes.byref(plain), 5, 7) == 0
        assert lib.chol_tune_set(L.CI_C64, ctypes.byref(plain), 16, 7) == -4    # FP64 types only
        assert lib.chol_tune_set(L.CI_F32, ctypes.byref(mixed), 16, 7) == -4
        assert lib.chol_tune_set(L.CI_C64, ctypes.byref(mixed), 17, 4) == -3
        assert lib.chol_tune_set(7, ctypes.byref(mixed), 16, 4) == -1
    finally:
        lib.chol_autotune_clear()
