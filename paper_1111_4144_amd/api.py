"""PyTorch-facing functions over libcholinv.

PyTorch provides device memory and the current HIP stream; every computation
runs in the library's gfx950 kernels (see include/cholinv.h).  Tensors must be
on the GPU.  Calls are asynchronous on torch's current stream unless
``check_errors=True`` (which synchronises to read the per-matrix ``info``).

* ``inverse(A, method, precision, ns_steps)``   X = A^{-1} (Section IV)
* ``inverse_varlen(packed, sizes, offsets)``    packed batch of uneven orders
  (``varlen_workspace_bytes`` sizes its reusable workspace)
* ``factor(A)`` / ``ldl(A)``                    Section II / II.A factorisations
* ``inverse_backward(X, G)``                    gA = -X Gh X
* ``CholInverse``                               autograd.Function saving X
* ``autotune`` / ``autotune_varlen`` / ``tuned_engine`` / ``tune_set`` / ``autotune_clear``
  engine choice per order, large-order configuration, uneven-batch bucket edge
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L

_DT = {torch.float32: L.CI_F32, torch.float64: L.CI_F64, torch.complex64: L.CI_C64,
       torch.complex128: L.CI_C128}


def _dtype_code(t: torch.Tensor) -> int:
    try:
        return _DT[t.dtype]
    except KeyError:
        raise TypeError("unsupported dtype %s" % t.dtype) from None


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_device(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("libcholinv operates on GPU tensors only")


def _workspace(nbytes: int, device) -> torch.Tensor | None:
    if nbytes == 0:
        return None
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def _finish(fn, info, check_errors):
    if check_errors and info is not None:
        bad = torch.nonzero(info).flatten()
        if bad.numel():
            b = int(bad[0])
            raise torch.linalg.LinAlgError(
                "%s: matrix %d is not positive definite (pivot %d failed)" % (fn, b, int(info[b])))


def inverse(A: torch.Tensor, *, method="chol", precision="plain", ns_steps=None,
            fill_lower=True, check_errors=False, return_info=False, out=None):
    """X = A^{-1} for Hermitian positive-definite A[..., n, n] (upper triangle read).

    precision "plain": all arithmetic in A's dtype.  "mixed" (float32 /
    complex64 only): FP32 bulk, FP64 pivots, then ``ns_steps`` (default 1)
    Newton-Schulz steps with an FP64 residual.
    """
    _check_device(A)
    if A.dim() < 2 or A.shape[-1] != A.shape[-2]:
        raise ValueError("A must be [..., n, n]")
    if ns_steps is None:
        ns_steps = 1 if precision == "mixed" else 0
    n = A.shape[-1]
    batch_shape = A.shape[:-2]
    A3 = A.reshape(-1, n, n)
    if not A3.is_contiguous():
        A3 = A3.contiguous()
    B = A3.shape[0]
    if out is not None:
        _check_device(out)
        if out.shape != A.shape or not out.is_contiguous() or out.dtype != A.dtype:
            raise ValueError("out must be a contiguous tensor shaped like A")
        X = out.view(-1, n, n)
    else:
        X = torch.empty_like(A3)
    info = torch.empty(B, dtype=torch.int32, device=A.device)   # every entry is written
    opts = L.make_opts(method, precision, ns_steps, fill_lower)
    dt = _dtype_code(A)
    lib = L.lib()
    s = _stream(A.device)
    if n <= L.CI_SMALL_NMAX:
        rc = lib.chol_inverse_batched(dt, B, n, None, None, 0, _ptr(A3), n * n, _ptr(X), n * n,
                                      ctypes.byref(opts), None, 0, _ptr(info), s)
        L.check("chol_inverse_batched", rc)
    else:
        ws = lib.chol_workspace_size(L.CI_FN_INVERSE, dt, 1, n, ctypes.byref(opts))
        work = _workspace(ws, A.device)
        for b in range(B):
            rc = lib.chol_inverse(dt, n, _ptr(A3[b]), n, _ptr(X[b]), n, ctypes.byref(opts),
                                  _ptr(work), ws, _ptr(info[b:b + 1]), s)
            L.check("chol_inverse", rc)
    _finish("inverse", info, check_errors)
    X = X.reshape(*batch_shape, n, n)
    info = info.reshape(batch_shape)
    return (X, info) if return_info else X


def varlen_workspace_bytes(packed: torch.Tensor, batch: int) -> int:
    """Workspace size (bytes) of ``inverse_varlen`` for ``batch`` matrices."""
    opts = L.make_opts("chol", "plain", 0, True)
    return int(L.lib().chol_workspace_size(L.CI_FN_BATCHED, _dtype_code(packed), batch, 0,
                                           ctypes.byref(opts)))


def inverse_varlen(packed: torch.Tensor, sizes: torch.Tensor, offsets: torch.Tensor, *,
                   n_max: int | None = None, method="chol", precision="plain", ns_steps=None,
                   fill_lower=True, out=None, check_errors=False, return_info=False,
                   workspace: torch.Tensor | None = None):
    """Inverse of every matrix of a packed batch: matrix b has order sizes[b] and
    starts at element offsets[b] (dense, leading dimension sizes[b])."""
    _check_device(packed, sizes, offsets)
    if ns_steps is None:
        ns_steps = 1 if precision == "mixed" else 0
    sizes = sizes.to(torch.int32).contiguous()
    offsets = offsets.to(torch.int64).contiguous()
    B = sizes.shape[0]
    if n_max is None:
        n_max = int(sizes.max()) if B else 1
    X = out if out is not None else torch.empty_like(packed)
    info = torch.empty(B, dtype=torch.int32, device=packed.device)   # every entry is written
    opts = L.make_opts(method, precision, ns_steps, fill_lower)
    lib = L.lib()
    dt = _dtype_code(packed)
    ws = lib.chol_workspace_size(L.CI_FN_BATCHED, dt, B, 0, ctypes.byref(opts))
    if workspace is None or workspace.numel() < ws:
        workspace = _workspace(ws, packed.device)
    rc = lib.chol_inverse_batched(dt, B, 0, _ptr(sizes), _ptr(offsets), int(n_max), _ptr(packed),
                                  0, _ptr(X), 0, ctypes.byref(opts), _ptr(workspace), ws,
                                  _ptr(info), _stream(packed.device))
    L.check("chol_inverse_batched", rc)
    _finish("inverse_varlen", info, check_errors)
    return (X, info) if return_info else X


def factor(A: torch.Tensor, *, inplace=False, return_info=False):
    """Cholesky factor R (upper, A = R^* R, eqs. 3-4) of A[..., n, n]; the strict
    lower triangle is copied from A unchanged."""
    _check_device(A)
    n = A.shape[-1]
    R = A if inplace else A.clone()
    R3 = R.reshape(-1, n, n)
    B = R3.shape[0]
    info = torch.zeros(B, dtype=torch.int32, device=A.device)
    lib = L.lib()
    dt = _dtype_code(A)
    if n <= L.CI_SMALL_NMAX:
        rc = lib.chol_factor(dt, B, n, _ptr(R3), n, n * n, _ptr(info), None, 0, _stream(A.device))
        L.check("chol_factor", rc)
    else:
        ws = lib.chol_workspace_size(L.CI_FN_FACTOR, dt, 1, n, None)
        work = _workspace(ws, A.device)
        for b in range(B):
            rc = lib.chol_factor(dt, 1, n, _ptr(R3[b]), n, n * n, _ptr(info[b:b + 1]),
                                 _ptr(work), ws, _stream(A.device))
            L.check("chol_factor", rc)
    return (R, info.reshape(A.shape[:-2])) if return_info else R


def ldl(A: torch.Tensor, *, return_info=False):
    """LDL factors (R unit upper in the strict upper triangle, d) of A[..., n, n]
    (eqs. 10-11).  Returns (R_with_A's_diagonal_and_lower, d)."""
    _check_device(A)
    n = A.shape[-1]
    R = A.clone()
    R3 = R.reshape(-1, n, n)
    B = R3.shape[0]
    rdt = torch.float32 if A.dtype in (torch.float32, torch.complex64) else torch.float64
    d = torch.empty(B, n, dtype=rdt, device=A.device)
    info = torch.zeros(B, dtype=torch.int32, device=A.device)
    rc = L.lib().ldl_factor(_dtype_code(A), B, n, _ptr(R3), n, n * n, _ptr(d), _ptr(info),
                            _stream(A.device))
    L.check("ldl_factor", rc)
    d = d.reshape(*A.shape[:-2], n)
    return (R, d, info.reshape(A.shape[:-2])) if return_info else (R, d)


def _rhs_block(Y, n, lead):
    """(Y as [B, n, k], vector?) for right-hand sides [..., n] or [..., n, k]."""
    if Y.dim() == lead + 1 and Y.shape[-1] == n:
        return Y.reshape(-1, n, 1), True
    if Y.dim() == lead + 2 and Y.shape[-2] == n:
        return Y.reshape(-1, n, Y.shape[-1]), False
    raise ValueError("right-hand sides must be [..., n] or [..., n, k] with the factor's batch")


def solve_factored(R: torch.Tensor, Y: torch.Tensor, *, d: torch.Tensor | None = None,
                   out: torch.Tensor | None = None) -> torch.Tensor:
    """x = A^{-1} y from the factor of A: R from :func:`factor` (eqs. 5-7) or,
    with d, (R, d) from :func:`ldl` (eqs. 12-14).  Y is [..., n] (one
    right-hand side per matrix) or [..., n, k]; out may be Y (in place)."""
    _check_device(R, Y)
    if Y.dtype != R.dtype:
        raise TypeError("Y must have the factor's dtype")
    n = R.shape[-1]
    lead = R.dim() - 2
    R3 = R.reshape(-1, n, n).contiguous()
    B = R3.shape[0]
    Y3, vec = _rhs_block(Y.contiguous(), n, lead)
    if Y3.shape[0] != B:
        raise ValueError("batch of Y does not match the factor's")
    k = Y3.shape[-1]
    if out is None:
        X = torch.empty(Y.shape, dtype=Y.dtype, device=Y.device)
    elif out.shape != Y.shape or out.dtype != Y.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous tensor shaped like Y")
    else:
        X = out
    X3 = X.view(Y3.shape)
    method = L.CI_METHOD_CHOL
    if d is not None:
        method = L.CI_METHOD_LDL
        d = d.reshape(B, n).contiguous()
        _check_device(d)
    rc = L.lib().chol_solve(_dtype_code(R), method, B, n, k, _ptr(R3), n, n * n,
                            None if d is None else _ptr(d), _ptr(Y3), k, n * k, _ptr(X3), k,
                            n * k, _stream(R.device))
    L.check("chol_solve", rc)
    return X


def solve(A: torch.Tensor, Y: torch.Tensor, *, method="chol", return_info=False):
    """x = A^{-1} y for Hermitian positive-definite A[..., n, n] (n <= 64):
    the factorisation (eqs. 3-4 or 10-11), then the two substitutions."""
    if method == "chol":
        Rf, info = factor(A, return_info=True)
        X = solve_factored(Rf, Y)
    elif method == "ldl":
        Rf, d, info = ldl(A, return_info=True)
        X = solve_factored(Rf, Y, d=d)
    else:
        raise ValueError("method must be 'chol' or 'ldl'")
    return (X, info) if return_info else X


def inverse_nonherm(D: torch.Tensor, *, method="chol", precision="plain", ns_steps=None,
                    return_info=False, check_errors=False):
    """D^{-1} for general nonsingular D[..., n, n] (n <= 64) by Section III.C:
    A = D D^* is Hermitian positive definite and D^{-1} = D^* A^{-1}.  The
    options apply to the inversion of A (whose condition number is kappa(D)^2)."""
    _check_device(D)
    n = D.shape[-1]
    D3 = D.reshape(-1, n, n).contiguous()
    B = D3.shape[0]
    X = torch.empty_like(D3)
    info = torch.zeros(B, dtype=torch.int32, device=D.device)
    lib = L.lib()
    dt = _dtype_code(D)
    if ns_steps is None:
        ns_steps = 1 if precision == "mixed" else 0
    opts = L.make_opts(method, precision, ns_steps)
    ws = lib.chol_workspace_size(L.CI_FN_NONHERM, dt, B, n, ctypes.byref(opts))
    work = _workspace(ws, D.device)
    rc = lib.chol_inverse_nonherm(dt, B, n, _ptr(D3), n * n, _ptr(X), ctypes.byref(opts),
                                  _ptr(work), ws, _ptr(info), _stream(D.device))
    L.check("chol_inverse_nonherm", rc)
    _finish("inverse_nonherm", info, check_errors)
    X = X.reshape(D.shape)
    return (X, info.reshape(D.shape[:-2])) if return_info else X


def inverse_q15(Q: torch.Tensor, *, variant="IV.A", return_info=False):
    """Fixed-point inversion of complex Hermitian matrices given as int16
    mantissas Q[..., n, n, 2] (re, im; value Q / 2^15), n <= 16: Cholesky and
    the Section IV.A back-substitution in Q15 storage with int64 Q30 sums
    (variant "IV.A"), or the Section III methods "III.A" / "III.B" in the same
    format.  Returns (X int16 [..., n, n, 2], xexp int32 [...]) with
    A^{-1} = X 2^xexp, plus (sat, info) with return_info."""
    _check_device(Q)
    if Q.dtype != torch.int16 or Q.shape[-1] != 2 or Q.shape[-2] != Q.shape[-3]:
        raise TypeError("Q must be int16 [..., n, n, 2]")
    n = Q.shape[-2]
    Q4 = Q.reshape(-1, n, n, 2).contiguous()
    B = Q4.shape[0]
    X = torch.empty_like(Q4)
    xexp = torch.zeros(B, dtype=torch.int32, device=Q.device)
    sat = torch.zeros(B, dtype=torch.int32, device=Q.device)
    info = torch.zeros(B, dtype=torch.int32, device=Q.device)
    if variant == "IV.A":
        rc = L.lib().chol_inverse_q15(B, n, _ptr(Q4), n * n, _ptr(X), _ptr(xexp), _ptr(sat),
                                      _ptr(info), _stream(Q.device))
        L.check("chol_inverse_q15", rc)
    else:
        var = {"III.A": L.CI_III_A, "III.B": L.CI_III_B}[variant]
        rc = L.lib().chol_inverse_q15_compare(var, B, n, _ptr(Q4), n * n, _ptr(X), _ptr(xexp),
                                              _ptr(sat), _ptr(info), _stream(Q.device))
        L.check("chol_inverse_q15_compare", rc)
    X = X.reshape(Q.shape)
    lead = Q.shape[:-3]
    if return_info:
        return X, xexp.reshape(lead), sat.reshape(lead), info.reshape(lead)
    return X, xexp.reshape(lead)


def inverse_compare(A: torch.Tensor, *, variant="III.A", method="chol", return_info=False):
    """The comparison methods of Section III on the GPU (orders <= 16, element
    type arithmetic): "III.A" equation solving (eq. 15; Cholesky or LDL) or
    "III.B" triangular operations (eqs. 17-19; Cholesky); "IV" is the
    proposed Section IV route in the same framework (same factor code and
    arithmetic), the like-for-like reference.  X in full."""
    _check_device(A)
    var = {"III.A": L.CI_III_A, "III.B": L.CI_III_B, "IV": L.CI_IV_SAME}[variant]
    meth = {"chol": L.CI_METHOD_CHOL, "ldl": L.CI_METHOD_LDL}[method]
    n = A.shape[-1]
    A3 = A.reshape(-1, n, n).contiguous()
    B = A3.shape[0]
    X = torch.empty_like(A3)
    info = torch.zeros(B, dtype=torch.int32, device=A.device)
    rc = L.lib().chol_inverse_compare(_dtype_code(A), var, meth, B, n, _ptr(A3), n * n, _ptr(X),
                                      _ptr(info), _stream(A.device))
    L.check("chol_inverse_compare", rc)
    X = X.reshape(A.shape)
    return (X, info.reshape(A.shape[:-2])) if return_info else X


_DT_CODE = {"f32": L.CI_F32, "f64": L.CI_F64, "c64": L.CI_C64, "c128": L.CI_C128}


def _code_of(dtype) -> int:
    if isinstance(dtype, str):
        return _DT_CODE[dtype]
    return _DT[dtype]


def autotune(dtype, *, method="chol", precision="plain", ns_steps=None, orders=(1, 16),
             batch=65536, cache=None, device=None) -> int:
    """Time the candidate engines for each order in ``orders`` (inclusive range
    within 1..16) on the current device and stream and record the fastest for
    later calls with the same dtype, method and precision; ``orders = (n, n)``
    with n > 64 times the large-order configurations at order n instead.
    ``cache``: a text file whose entries for this device are loaded instead of
    measured (new ones are appended).  Returns the number of orders measured."""
    if ns_steps is None:
        ns_steps = 1 if precision == "mixed" else 0
    opts = L.make_opts(method, precision, ns_steps, True)
    path = None if cache is None else str(cache).encode()
    rc = L.lib().chol_autotune(_code_of(dtype), ctypes.byref(opts), int(orders[0]), int(orders[1]),
                               int(batch), path, _stream(device))
    if rc < 0:
        L.check("chol_autotune", rc)
    return int(rc)


def tuned_engine(dtype, n, *, method="chol", precision="plain") -> int:
    """The recorded engine for order n (0 = built-in choice)."""
    opts = L.make_opts(method, precision, 0, True)
    rc = L.lib().chol_tuned_engine(_code_of(dtype), ctypes.byref(opts), int(n))
    if rc < 0:
        L.check("chol_tuned_engine", rc)
    return int(rc)


def autotune_varlen(packed: torch.Tensor, sizes: torch.Tensor, offsets: torch.Tensor, *,
                    n_max: int | None = None, method="chol", precision="plain", ns_steps=None,
                    workspace: torch.Tensor | None = None) -> int:
    """Time the uneven-batch path on this batch for each edge of its last size
    bucket (33, 25, 17) and record the fastest for later ``inverse_varlen``
    calls with the same dtype, method and precision.  Returns the edge."""
    _check_device(packed, sizes, offsets)
    if ns_steps is None:
        ns_steps = 1 if precision == "mixed" else 0
    sizes = sizes.to(torch.int32).contiguous()
    offsets = offsets.to(torch.int64).contiguous()
    B = sizes.shape[0]
    if n_max is None:
        n_max = int(sizes.max()) if B else 1
    X = torch.empty_like(packed)
    opts = L.make_opts(method, precision, ns_steps, True)
    lib = L.lib()
    dt = _dtype_code(packed)
    ws = lib.chol_workspace_size(L.CI_FN_BATCHED, dt, B, 0, ctypes.byref(opts))
    if workspace is None or workspace.numel() < ws:
        workspace = _workspace(ws, packed.device)
    rc = lib.chol_autotune_varlen(dt, ctypes.byref(opts), B, _ptr(sizes), _ptr(offsets),
                                  int(n_max), _ptr(packed), _ptr(X), _ptr(workspace), ws,
                                  _stream(packed.device))
    if rc < 0:
        L.check("chol_autotune_varlen", rc)
    return int(rc)


def tune_set(dtype, n, engine, *, method="chol", precision="plain") -> None:
    """Record ``engine`` for order n without measuring (0 = built-in choice);
    n > 64: a large-order configuration for n's bucket; n = 0: the
    uneven-batch bucket edge."""
    opts = L.make_opts(method, precision, 0, True)
    L.check("chol_tune_set", L.lib().chol_tune_set(_code_of(dtype), ctypes.byref(opts), int(n),
                                                   int(engine)))


def autotune_clear() -> None:
    """Forget every recorded engine choice."""
    L.lib().chol_autotune_clear()


def inverse_backward(X: torch.Tensor, G: torch.Tensor) -> torch.Tensor:
    """gA = -X Gh X, Gh = (G + G^H)/2, from the forward's full Hermitian X."""
    _check_device(X, G)
    n = X.shape[-1]
    X3 = X.reshape(-1, n, n).contiguous()
    G3 = G.reshape(-1, n, n).to(X.dtype).contiguous()
    gA = torch.empty_like(X3)
    rc = L.lib().chol_inverse_backward(_dtype_code(X), X3.shape[0], n, _ptr(X3), _ptr(G3),
                                       _ptr(gA), n * n, _stream(X.device))
    L.check("chol_inverse_backward", rc)
    return gA.reshape(X.shape)


class CholInverse(torch.autograd.Function):
    """X = A^{-1} with the hand-written adjoint; the backward reuses the saved X.

    The gradient is the Hermitian one, gA = -X Gh X, i.e. the gradient of the
    real loss along Hermitian perturbations of A (the domain of the method)."""

    @staticmethod
    def forward(ctx, A, method="chol", precision="plain", ns_steps=None):
        if A.requires_grad and A.dtype == torch.complex128 and A.shape[-1] > 32:
            # the adjoint of complex128 orders 33..64 would need three 64 x 64
            # complex128 matrices (200 KB) in one workgroup's LDS
            raise RuntimeError("CholInverse: no backward for complex128 orders above 32")
        X = inverse(A, method=method, precision=precision, ns_steps=ns_steps, fill_lower=True)
        ctx.save_for_backward(X)
        return X

    @staticmethod
    def backward(ctx, G):
        (X,) = ctx.saved_tensors
        return inverse_backward(X, G), None, None, None
