"""GPU parity of the batched solves A x = y (Section II eqs. 5-7, Section II.A
eqs. 12-14) against the FP64 oracle.

* factor + solve on the GPU against the oracle's factor + solve of the same
  (rounded) input, per system: relative Frobenius error of the n x k block
  <= 1e-12 * kappa (FP64 types) or 2e-6 * kappa (FP32 types);
* the solve kernel alone, fed the oracle's factor rounded to the working type;
* in place (x = b), strided right-hand-side blocks, empty batches;
* the MIMO detection batch (1,048,576 complex 8 x 8 systems) with sampled
  systems checked one by one.
The oracle's solves are pinned to numpy.linalg.solve by the CPU tests.
"""
import ctypes

import numpy as np
import pytest

import oracle as O
from paper_1111_4144_amd import inputs as G
from tests.helpers import TOL_FP32, TOL_FP64, assert_within, torch_cuda

pytestmark = pytest.mark.gpu

_NP = {"f32": np.float32, "f64": np.float64, "c64": np.complex64, "c128": np.complex128}
_TOL = {"f32": TOL_FP32, "c64": TOL_FP32, "f64": TOL_FP64, "c128": TOL_FP64}


def _inputs(dt, batch, n, k, seed):
    rng = np.random.default_rng([seed, n, k])
    cplx = dt.startswith("c")
    a = G.random_hpd(rng, batch, n, shift=0.5, complex_=cplx).astype(_NP[dt])
    y = rng.standard_normal((batch, n, k))
    if cplx:
        y = y + 1j * rng.standard_normal((batch, n, k))
    return a, y.astype(_NP[dt])


def _oracle_solve(a, y, method):
    """Per system: the oracle's factor of A, then its solve of every column."""
    a = a.astype(np.complex128 if np.iscomplexobj(a) else np.float64)
    y = y.astype(a.dtype)
    x = np.zeros_like(y)
    for b in range(a.shape[0]):
        if method == "chol":
            r, info = O.chol(a[b])
            assert info == 0
            for c in range(y.shape[-1]):
                x[b, :, c] = O.chol_solve(r, y[b, :, c])
        else:
            r, d, info = O.ldl(a[b])
            assert info == 0
            for c in range(y.shape[-1]):
                x[b, :, c] = O.ldl_solve(r, d, y[b, :, c])
    return x


@pytest.mark.parametrize("method", ["chol", "ldl"])
@pytest.mark.parametrize("dt", ["f32", "f64", "c64", "c128"])
@pytest.mark.parametrize("n,k", [(1, 1), (2, 1), (4, 1), (7, 1), (8, 1), (16, 1), (16, 3),
                                 (24, 1), (64, 2)])
def test_solve_vs_oracle(n, k, dt, method):
    t = torch_cuda()
    from paper_1111_4144_amd import api
    batch = 261                                   # a ragged last block of lanes
    a, y = _inputs(dt, batch, n, k, 17)
    ref = _oracle_solve(a, y, method)
    x, info = api.solve(t.from_numpy(a).cuda(), t.from_numpy(y).cuda(), method=method,
                        return_info=True)
    t.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    assert_within(x.cpu().numpy(), ref, a, _TOL[dt], "solve %s %s n=%d k=%d" % (dt, method, n, k))


@pytest.mark.parametrize("method", ["chol", "ldl"])
@pytest.mark.parametrize("dt", ["f64", "c64"])
def test_solve_kernel_from_oracle_factor(dt, method):
    """The solve alone: the oracle's factor, rounded to the working type, is the
    input of both sides."""
    t = torch_cuda()
    from paper_1111_4144_amd import api
    n, k, batch = 13, 2, 70
    a, y = _inputs(dt, batch, n, k, 23)
    cplx = dt.startswith("c")
    wide = np.complex128 if cplx else np.float64
    rs = np.zeros((batch, n, n), wide)
    ds = np.zeros((batch, n))
    for b in range(batch):
        if method == "chol":
            rs[b], info = O.chol(a[b].astype(wide))
        else:
            rs[b], ds[b], info = O.ldl(a[b].astype(wide))
        assert info == 0
    r_w = rs.astype(_NP[dt])
    rdt = np.float32 if dt in ("f32", "c64") else np.float64
    d_w = ds.astype(rdt)
    ref = np.zeros((batch, n, k), wide)
    for b in range(batch):
        for c in range(k):
            yc = y[b, :, c].astype(wide)
            ref[b, :, c] = (O.chol_solve(r_w[b].astype(wide), yc) if method == "chol" else
                            O.ldl_solve(r_w[b].astype(wide), d_w[b].astype(np.float64), yc))
    R = t.from_numpy(r_w).cuda()
    Y = t.from_numpy(y).cuda()
    D = t.from_numpy(d_w).cuda() if method == "ldl" else None
    x = api.solve_factored(R, Y, d=D).cpu().numpy()
    assert_within(x, ref, a, _TOL[dt], "solve kernel %s %s" % (dt, method))


def test_solve_in_place_and_strided():
    """x = b in place through the C-ABI, and right-hand-side blocks with
    leading dimension and stride larger than the block (the padding is kept)."""
    t = torch_cuda()
    from paper_1111_4144_amd import _lib as L, api
    n, k, batch = 10, 3, 50
    a, y = _inputs("f64", batch, n, k, 31)
    ref = _oracle_solve(a, y, "chol")
    R = api.factor(t.from_numpy(a).cuda())
    # in place
    Y = t.from_numpy(y.copy()).cuda()
    rc = L.lib().chol_solve(L.CI_F64, 0, batch, n, k, R.data_ptr(), n, n * n, None,
                            Y.data_ptr(), k, n * k, Y.data_ptr(), k, n * k, None)
    assert rc == 0
    t.cuda.synchronize()
    assert_within(Y.cpu().numpy(), ref, a, TOL_FP64, "in place")
    # strided: ldb = k + 2, one padding row per system
    ldb, sb = k + 2, (n + 1) * (k + 2)
    pad = np.full((batch, n + 1, ldb), 7.25)
    pad[:, :n, :k] = y
    B = t.from_numpy(pad.reshape(batch, -1).copy()).cuda()
    X = t.full_like(B, -3.5)
    rc = L.lib().chol_solve(L.CI_F64, 0, batch, n, k, R.data_ptr(), n, n * n, None,
                            B.data_ptr(), ldb, sb, X.data_ptr(), ldb, sb, None)
    assert rc == 0
    t.cuda.synchronize()
    xs = X.cpu().numpy().reshape(batch, n + 1, ldb)
    assert_within(xs[:, :n, :k], ref, a, TOL_FP64, "strided")
    assert (xs[:, :n, k:] == -3.5).all() and (xs[:, n, :] == -3.5).all()
    # in place with one right-hand side per system (the LDS-staged kernel)
    a8, y8 = _inputs("c64", 130, 8, 1, 37)
    ref8 = _oracle_solve(a8, y8, "chol")
    R8 = api.factor(t.from_numpy(a8).cuda())
    Y8 = t.from_numpy(y8[:, :, 0].copy()).cuda()
    assert api.solve_factored(R8, Y8, out=Y8).data_ptr() == Y8.data_ptr()
    assert_within(Y8.cpu().numpy()[:, :, None], ref8, a8, TOL_FP32, "in place, staged")
    # empty batch / empty order / no right-hand sides: nothing to do
    lib = L.lib()
    assert lib.chol_solve(L.CI_F64, 0, 0, n, k, None, n, 0, None, None, k, 0, None, k, 0, None) == 0
    assert lib.chol_solve(L.CI_F64, 0, 4, 0, k, None, 1, 0, None, None, k, 0, None, k, 0, None) == 0
    assert lib.chol_solve(L.CI_F64, 0, 4, n, 0, R.data_ptr(), n, n * n, None, B.data_ptr(), 1,
                          n, X.data_ptr(), 1, n, None) == 0


@pytest.mark.parametrize("method", ["chol", "ldl"])
def test_solve_mimo_batch_sampled(method):
    """1,048,576 complex64 8 x 8 systems (B B^H + sigma I, one right-hand side
    each), factor + solve at the full size; 256 sampled systems against the
    oracle."""
    t = torch_cuda()
    from paper_1111_4144_amd import api
    n, count = 8, 1 << 20
    a = G.mimo(n, count)
    rng = np.random.default_rng(41)
    y = (rng.standard_normal((count, n)) + 1j * rng.standard_normal((count, n))).astype(np.complex64)
    x = api.solve(t.from_numpy(a).cuda(), t.from_numpy(y).cuda(), method=method).cpu().numpy()
    idx = np.sort(rng.choice(count, 256, replace=False))
    ref = _oracle_solve(a[idx], y[idx, :, None], method)
    assert_within(x[idx, :, None], ref, a[idx], TOL_FP32, "mimo solve " + method)
    assert np.isfinite(x).all()
