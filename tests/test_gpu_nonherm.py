"""GPU parity of the non-Hermitian inversion D^{-1} = D^* (D D^*)^{-1}
(Section III.C) against the oracle's route, which the CPU tests pin to
numpy.linalg.inv.  Error per matrix relative to the oracle <= tol * kappa(A),
A = D D^* (kappa(D)^2): 1e-12 for FP64 types, 2e-6 for FP32 types."""
import numpy as np
import pytest

import oracle as O
from tests.helpers import TOL_FP32, TOL_FP64, assert_within, kappas, torch_cuda

pytestmark = pytest.mark.gpu

_NP = {"f32": np.float32, "f64": np.float64, "c64": np.complex64, "c128": np.complex128}


def _general(dt, batch, n, seed):
    """Nonsingular non-Hermitian D: Gaussian plus a diagonal shift of
    sqrt(n) (condition numbers in the tens)."""
    rng = np.random.default_rng([seed, n])
    d = rng.standard_normal((batch, n, n))
    if dt.startswith("c"):
        d = d + 1j * rng.standard_normal((batch, n, n))
    d = d + np.sqrt(n) * np.eye(n)
    return d.astype(_NP[dt])


@pytest.mark.parametrize("dt,prec", [("f64", "plain"), ("c128", "plain"), ("f32", "plain"),
                                     ("c64", "plain"), ("c64", "mixed")])
@pytest.mark.parametrize("n", [1, 3, 8, 16, 29, 64])
def test_nonherm_vs_oracle(n, dt, prec):
    t = torch_cuda()
    from paper_1111_4144_amd import api
    batch = 75
    d = _general(dt, batch, n, 5)
    dw = d.astype(np.complex128)
    ref = np.stack([O.inv_nonherm(dw[b])[0] for b in range(batch)])
    x, info = api.inverse_nonherm(t.from_numpy(d).cuda(), precision=prec, return_info=True)
    assert (info.cpu().numpy() == 0).all()
    x = x.cpu().numpy()
    a = dw @ np.conj(np.swapaxes(dw, -1, -2))       # only the tolerance's kappa
    tol = TOL_FP64 if dt in ("f64", "c128") else TOL_FP32
    assert_within(x, ref, a, tol, "nonherm %s %s n=%d" % (dt, prec, n))
    # X D - I = E D for the error E of X, so its size is at most
    # ||E|| ||D|| <= tol kappa(A) ||D^{-1}|| ||D|| = tol kappa(A)^{3/2}
    resid = np.abs(x.astype(np.complex128) @ dw - np.eye(n)).max(axis=(-1, -2))
    k = kappas(a)
    assert (resid <= 4 * n * tol * k ** 1.5).all(), (resid / k ** 1.5).max()


def test_nonherm_singular_reports_info():
    t = torch_cuda()
    from paper_1111_4144_amd import api
    n = 6
    d = _general("f64", 4, n, 9)
    d[2, 3, :] = 0.0                                 # matrix 2 singular: D D^* has a zero pivot
    x, info = api.inverse_nonherm(t.from_numpy(d).cuda(), return_info=True)
    info = info.cpu().numpy()
    assert info[2] == O.chol(d[2] @ d[2].T)[1] == 4
    assert (info[[0, 1, 3]] == 0).all()
    assert np.isnan(x.cpu().numpy()[2]).all()
