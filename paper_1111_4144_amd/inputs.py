"""Seeded synthetic inputs for the Hermitian positive-definite inversion workloads.

This module only draws random matrices; it holds none of the inversion's
arithmetic, and both the GPU path's tests and the CPU oracle consume what it
returns.  Everything is built in FP64 (or complex128), made exactly Hermitian
(lower triangle = conjugate of the upper, imaginary diagonal = 0) and only then
rounded to the storage type, so the stored matrix is exactly Hermitian.

Large batches are drawn in chunks of ``CHUNK`` matrices, chunk ``c`` from the
generator ``default_rng([seed, stream, c])``; any prefix of a batch can
therefore be regenerated on its own (the benchmark's CPU baseline uses that).

Workloads (each one a synthetic stand-in; no dataset is involved):

* ``plain_fp64_4x4``   4096 complex128 4x4, A = B B^H + 4I
* ``mimo``             complex64 n x n, A = B B^H + sigma I, sigma = 10^U(-2, 0)
* ``varlen_spd``       real float32 SPD, n ~ U{2..64}, A = Q diag(lambda) Q^T,
                       Q Haar, lambda log-spaced over [1, 1e3]; packed storage
* ``large_spd``        real SPD n x n, lambda log-spaced over [1, 1e6]
* ``grad_16``          65,536 complex64 16x16, A = B B^H + I, G iid CN(0, 1)
* ``kms``              Kac-Murdock-Szego matrices a_ij = rho^(j-i) (closed-form inverse)

B has iid standard complex normal entries (real and imaginary parts N(0, 1/2)).
"""
from __future__ import annotations

import numpy as np

CHUNK = 4096

SEED_PLAIN = 1000
SEED_MIMO = 1001
SEED_VARLEN = 1002
SEED_LARGE = 1003
SEED_GRAD = 1004


def _rng(seed, stream, chunk):
    return np.random.default_rng([int(seed), int(stream), int(chunk)])


def complex_normal(rng, shape):
    """iid CN(0, 1): real and imaginary parts independent N(0, 1/2)."""
    s = np.sqrt(0.5)
    return (rng.standard_normal(shape) * s) + 1j * (rng.standard_normal(shape) * s)


def hermitize(a):
    """Return a copy whose strict lower triangle is the conjugate of the upper
    triangle and whose diagonal is real (exact, no arithmetic on the upper part)."""
    a = np.array(a, copy=True)
    n = a.shape[-1]
    il = np.tril_indices(n, -1)
    at = np.swapaxes(a, -1, -2)
    a[..., il[0], il[1]] = np.conj(at[..., il[0], il[1]])
    idx = np.arange(n)
    if np.iscomplexobj(a):
        a[..., idx, idx] = a[..., idx, idx].real
    return a


def haar_orthogonal(rng, count, n):
    """count Haar-distributed real orthogonal n x n matrices: QR of a Gaussian
    matrix with the column signs fixed by sign(diag R) (Mezzadri 2007)."""
    z = rng.standard_normal((count, n, n))
    q, r = np.linalg.qr(z)
    d = np.sign(np.diagonal(r, axis1=-2, axis2=-1))
    d[d == 0] = 1.0
    return q * d[..., None, :]


def log_spaced(n, top):
    """lambda_k = top^(k/(n-1)), k = 0..n-1 (lambda = [1] for n = 1)."""
    if n == 1:
        return np.ones(1)
    return top ** (np.arange(n) / (n - 1))


def _bbh_plus(rng, count, n, shift):
    b = complex_normal(rng, (count, n, n))
    a = b @ np.conj(np.swapaxes(b, -1, -2))
    idx = np.arange(n)
    a[:, idx, idx] += shift[:, None]
    return hermitize(a)


# ---------------------------------------------------------------------------
def plain_fp64_4x4(seed=SEED_PLAIN, count=4096):
    """count complex128 4x4 Hermitian PD matrices A = B B^H + 4I."""
    rng = _rng(seed, 4, 0)
    return _bbh_plus(rng, count, 4, np.full(count, 4.0)).astype(np.complex128)


def mimo(n, count, seed=SEED_MIMO, dtype=np.complex64, first_chunk=0):
    """count complex Hermitian PD n x n matrices A = B B^H + sigma I with
    sigma = 10^U(-2, 0) per matrix (condition numbers up to ~1e4 at n = 16).
    Chunk c of the full batch is drawn from default_rng([seed, n, c]);
    first_chunk skips the leading chunks."""
    out = np.empty((count, n, n), dtype=dtype)
    done = 0
    c = first_chunk
    while done < count:
        m = min(CHUNK, count - done)
        rng = _rng(seed, n, c)
        sigma = 10.0 ** rng.uniform(-2.0, 0.0, size=CHUNK)
        a = _bbh_plus(rng, CHUNK, n, sigma)
        out[done:done + m] = a[:m].astype(dtype)
        done += m
        c += 1
    return out


def varlen_sizes(count, seed=SEED_VARLEN, nmin=2, nmax=64):
    rng = _rng(seed, 0, 0)
    return rng.integers(nmin, nmax + 1, size=count).astype(np.int32)


def varlen_spd(count, seed=SEED_VARLEN, dtype=np.float32, top=1e3, sizes=None):
    """Packed batch of real SPD matrices A = Q diag(lambda) Q^T, n ~ U{2..64},
    Q Haar, lambda log-spaced over [1, top].  Returns (packed, sizes, offsets):
    matrix b is dense row major, order sizes[b], starting at element offsets[b]."""
    if sizes is None:
        sizes = varlen_sizes(count, seed)
    sizes = np.asarray(sizes, dtype=np.int32)
    count = sizes.shape[0]
    offsets = np.zeros(count, np.int64)
    if count:
        offsets[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    total = int(offsets[-1] + int(sizes[-1]) ** 2) if count else 0
    packed = np.empty(total, dtype=dtype)
    for c0 in range(0, count, CHUNK):
        rng = _rng(seed, 1, c0 // CHUNK)
        sz = sizes[c0:c0 + CHUNK]
        for n in np.unique(sz):
            sel = np.nonzero(sz == n)[0]
            q = haar_orthogonal(rng, sel.shape[0], int(n))
            lam = log_spaced(int(n), top)
            a = hermitize((q * lam[None, None, :]) @ np.swapaxes(q, -1, -2)).astype(dtype)
            for k, b in enumerate(sel):
                o = offsets[c0 + b]
                packed[o:o + n * n] = a[k].reshape(-1)
    return packed, sizes, offsets


def large_spd(n, seed=SEED_LARGE, top=1e6, dtype=np.float64, return_factors=False):
    """Real SPD n x n A = Q diag(lambda) Q^T, lambda log-spaced over [1, top]."""
    rng = _rng(seed, n, 0)
    q = haar_orthogonal(rng, 1, n)[0]
    lam = log_spaced(n, top)
    a = hermitize((q * lam[None, :]) @ q.T).astype(dtype)
    if return_factors:
        return a, q, lam
    return a


def grad_16(count=65536, seed=SEED_GRAD, n=16, dtype=np.complex64):
    """(A, G): A = B B^H + I complex Hermitian PD, G iid CN(0, 1) upstream gradient."""
    a = np.empty((count, n, n), dtype=dtype)
    g = np.empty((count, n, n), dtype=dtype)
    done = 0
    c = 0
    while done < count:
        m = min(CHUNK, count - done)
        rng = _rng(seed, n, c)
        a[done:done + m] = _bbh_plus(rng, CHUNK, n, np.ones(CHUNK))[:m].astype(dtype)
        g[done:done + m] = complex_normal(rng, (CHUNK, n, n))[:m].astype(dtype)
        done += m
        c += 1
    return a, g


def kms(n, rho, dtype=np.complex128):
    """Kac-Murdock-Szego matrix a_ij = rho^(j-i) for j >= i, a_ji = conj(a_ij)."""
    i = np.arange(n)
    p = np.maximum(i[None, :] - i[:, None], 0)
    if np.isrealobj(rho) and not np.issubdtype(np.dtype(dtype), np.complexfloating):
        # real rho, real storage: the symmetric matrix rho^|j-i| directly (no
        # complex temporaries, which matter at orders in the thousands)
        a = float(rho) ** np.abs(i[None, :] - i[:, None]).astype(np.float64)
        return a.astype(dtype)
    a = np.asarray(rho, dtype=np.complex128) ** p
    a = hermitize(np.triu(a))
    if not np.issubdtype(np.dtype(dtype), np.complexfloating):
        a = a.real
    return a.astype(dtype)


def random_hpd(rng, count, n, shift=1.0, complex_=True, dtype=None):
    """Small generic test inputs: B B^H + shift*I (complex) or B B^T + shift*I (real)."""
    if complex_:
        a = _bbh_plus(rng, count, n, np.full(count, float(shift)))
        return a.astype(dtype or np.complex128)
    b = rng.standard_normal((count, n, n))
    a = b @ np.swapaxes(b, -1, -2)
    idx = np.arange(n)
    a[:, idx, idx] += shift
    return hermitize(a).astype(dtype or np.float64)


def quantize_q15(a):
    """Complex (or real) matrices [batch, n, n] to Q15 mantissas int16
    [batch, n, n, 2] (re, im) with one power-of-two scale per matrix: a =
    q 2^(e - 15), e the smallest integer with max |re|, |im| < 2^e, values
    rounded to nearest and clipped to +-32767.  Returns (q, e)."""
    a = np.asarray(a)
    a = a.astype(np.complex128)
    if a.ndim == 2:
        a = a[None]
    peak = np.maximum(np.abs(a.real), np.abs(a.imag)).max(axis=(-1, -2))
    e = np.floor(np.log2(np.maximum(peak, np.finfo(np.float64).tiny))).astype(np.int32) + 1
    scale = np.ldexp(1.0, 15 - e)[:, None, None]
    q = np.empty(a.shape + (2,), np.int16)
    q[..., 0] = np.clip(np.rint(a.real * scale), -32767, 32767)
    q[..., 1] = np.clip(np.rint(a.imag * scale), -32767, 32767)
    return q, e
