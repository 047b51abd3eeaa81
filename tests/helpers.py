"""Shared helpers for the parity tests (comparison metrics and GPU plumbing)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O

# Tolerances on the per-matrix relative Frobenius error against the FP64 oracle,
# in units of the 2-norm condition number kappa(A).
TOL_FP64 = 1e-12       # plain FP64 path
TOL_FP32 = 2e-6        # FP32 path (mixed precision, after refinement, or plain FP32)


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


def rel_err(x, ref):
    """Per-matrix ||x - ref||_F / ||ref||_F over the last two axes."""
    x = np.asarray(x, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    num = np.sqrt(np.sum(np.abs(x - ref) ** 2, axis=(-1, -2)))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=(-1, -2)))
    return num / den


def kappas(a):
    """2-norm condition numbers of a stack of Hermitian PD matrices (oracle Jacobi)."""
    a = np.asarray(a)
    flat = a.reshape(-1, a.shape[-2], a.shape[-1])
    return np.array([O.kappa2(m.astype(np.complex128)) for m in flat]).reshape(a.shape[:-2])


def assert_within(x, ref, a, tol, what=""):
    """Every matrix must satisfy err <= tol * kappa; returns (max err, max err/kappa)."""
    err = rel_err(x, ref)
    k = kappas(a)
    ratio = err / k
    worst = int(np.argmax(ratio))
    assert np.all(np.isfinite(err)), "%s: non-finite result" % what
    assert ratio.max() <= tol, "%s: matrix %d err %.3e kappa %.3e (err/kappa %.3e > %.1e)" % (
        what, worst, err.flat[worst], k.flat[worst], ratio.max(), tol)
    return float(err.max()), float(ratio.max())


def hermitian_full(x):
    """Mirror the upper triangle (for comparing upper-only outputs)."""
    x = np.array(x)
    n = x.shape[-1]
    il = np.tril_indices(n, -1)
    xt = np.swapaxes(x, -1, -2)
    x[..., il[0], il[1]] = np.conj(xt[..., il[0], il[1]])
    return x
