"""Parity of the blocked large-order path (orders above 64, real types).

* against the FP64 oracle (Section IV inversion, eqs. 3-4 factor) at orders
  that span several panels with a ragged last panel;
* against closed forms at the full sizes: the Kac-Murdock-Szego matrix, whose
  inverse is tridiagonal, and Q diag(lambda) Q^T, whose inverse is
  Q diag(1/lambda) Q^T (sampled entries);
* failure reporting: a matrix that is not positive definite gives the
  1-based index of the first failing pivot (as the oracle's factor) and NaN.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_1111_4144_amd import inputs as I
from tests.helpers import TOL_FP32, TOL_FP64, rel_err, torch_cuda

pytestmark = pytest.mark.gpu

_NP = {"f32": np.float32, "f64": np.float64}


def _inverse(a, dt, prec, ns_steps=None):
    torch = torch_cuda()
    from paper_1111_4144_amd import api
    t = torch.from_numpy(np.ascontiguousarray(a.astype(_NP[dt]))).cuda()
    x, info = api.inverse(t, precision=prec, ns_steps=ns_steps, return_info=True)
    torch.cuda.synchronize()
    return x.cpu().numpy().astype(np.float64), int(info)


CASES = [("f64", "plain"), ("f32", "plain"), ("f32", "mixed")]


@pytest.mark.parametrize("dt,prec", CASES)
@pytest.mark.parametrize("n", [65, 130, 200, 333, 520])
def test_large_inverse_vs_oracle(n, dt, prec):
    top = 1e3
    a = I.large_spd(n, seed=I.SEED_LARGE + n, top=top)
    a_in = a.astype(_NP[dt]).astype(np.float64)      # the oracle sees the rounded input
    ref, info_ref = O.inv_prop(a_in)
    assert info_ref == 0
    x, info = _inverse(a, dt, prec)
    assert info == 0
    tol = TOL_FP64 if dt == "f64" else TOL_FP32
    err = float(rel_err(x, ref))
    assert err <= tol * top, "n=%d %s %s: err %.3e" % (n, dt, prec, err)
    # the output is exactly symmetric (upper half mirrored)
    assert np.array_equal(x, x.T)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("n", [65, 200, 333])
def test_large_factor_vs_oracle(n, dt):
    torch = torch_cuda()
    from paper_1111_4144_amd import api
    a = I.large_spd(n, seed=I.SEED_LARGE + 7 * n, top=1e2)
    a_in = a.astype(_NP[dt]).astype(np.float64)
    r_ref, info_ref = O.chol(a_in)
    assert info_ref == 0
    t = torch.from_numpy(a.astype(_NP[dt])).cuda()
    r, info = api.factor(t, return_info=True)
    r = r.cpu().numpy().astype(np.float64)
    assert int(info) == 0
    iu = np.triu_indices(n)
    tol = 1e-13 if dt == "f64" else 2e-6
    err = np.abs(r[iu] - r_ref[iu]).max() / np.abs(r_ref).max()
    assert err <= tol * 1e2, "n=%d %s: err %.3e" % (n, dt, err)
    il = np.tril_indices(n, -1)
    assert np.array_equal(r[il], a.astype(_NP[dt]).astype(np.float64)[il])   # untouched


def _kms_inverse(n, rho):
    """Closed form: (1 - rho^2)^{-1} tridiag(-rho; 1, 1 + rho^2, ..., 1; -rho)."""
    d = np.full(n, 1.0 + rho * rho)
    d[0] = d[-1] = 1.0
    x = np.diag(d) - rho * (np.eye(n, k=1) + np.eye(n, k=-1))
    return x / (1.0 - rho * rho)


@pytest.mark.parametrize("dt,prec", CASES)
def test_kms_closed_form_4096(dt, prec):
    n, rho = 4096, 0.5
    a = I.kms(n, rho, dtype=np.float64)
    kappa = ((1 + rho) / (1 - rho)) ** 2          # bound on the 2-norm condition number
    x, info = _inverse(a, dt, prec)
    assert info == 0
    ref = _kms_inverse(n, rho)
    tol = TOL_FP64 if dt == "f64" else TOL_FP32
    err = float(rel_err(x, ref))
    assert err <= tol * kappa, "%s %s: err %.3e" % (dt, prec, err)


def _closed_form_samples(q, lam, idx):
    """x_ij = sum_k q_ik q_jk / lambda_k for the sampled (i, j)."""
    i, j = idx
    return np.einsum("sk,sk->s", q[i] / lam[None, :], q[j])


@pytest.mark.parametrize("n,dt,prec,top", [(4096, "f64", "plain", 1e6),
                                           (8192, "f32", "mixed", 1e6)])
def test_full_size_sampled_closed_form(n, dt, prec, top):
    """The full-size workloads: sampled entries against Q diag(1/lambda) Q^T."""
    a, q, lam = I.large_spd(n, top=top, return_factors=True)
    x, info = _inverse(a, dt, prec)
    assert info == 0
    rng = np.random.default_rng(5)
    idx = (rng.integers(0, n, 4096), rng.integers(0, n, 4096))
    ref = _closed_form_samples(q, lam, idx)
    scale = 1.0 / lam.min()                        # ||A^{-1}||_2
    err = np.abs(x[idx] - ref).max() / scale
    # the rounding of A itself to the working type perturbs A^{-1} by up to
    # kappa * u relative; FP32 gets the FP32 bound, FP64 the FP64 one
    tol = TOL_FP64 if dt == "f64" else TOL_FP32
    assert err <= tol * top, "n=%d %s: sampled err %.3e" % (n, dt, err)
    assert np.array_equal(x[idx], x[idx[1], idx[0]])


def test_large_not_positive_definite():
    torch_cuda()
    n = 300
    a = I.large_spd(n, seed=11, top=10.0)
    a[250, 250] = -5.0                             # pivot 251 fails
    r_ref, info_ref = O.chol(a)
    assert info_ref == 251
    for dt, prec in CASES:
        x, info = _inverse(a, dt, prec)
        assert info == info_ref, (dt, prec, info)
        assert np.isnan(x).all()


def test_large_mixed_refinement_improves():
    """One Newton-Schulz step reduces the error of the FP32 factor-based inverse."""
    n, top = 520, 1e4
    a = I.large_spd(n, seed=3, top=top, dtype=np.float32).astype(np.float64)
    ref, _ = O.inv_prop(a)
    x0, _ = _inverse(a, "f32", "mixed", ns_steps=0)
    x1, _ = _inverse(a, "f32", "mixed", ns_steps=1)
    e0, e1 = float(rel_err(x0, ref)), float(rel_err(x1, ref))
    assert e1 < 0.5 * e0, (e0, e1)


def test_blocked_section_iv_variant():
    """The Section IV recurrence in block form (selected by the environment in
    a child process) against the oracle, next to the default inverse."""
    import os
    import subprocess
    import sys
    torch_cuda()
    code = r'''
import numpy as np, torch
import oracle as O
from paper_1111_4144_amd import api, inputs as I
from tests.helpers import rel_err
worst = 0.0
for n, dt, prec in [(200, np.float64, "plain"), (333, np.float32, "plain"), (333, np.float32, "mixed")]:
    a = I.large_spd(n, seed=77 + n, top=1e3)
    ref, _ = O.inv_prop(a.astype(dt).astype(np.float64))
    x = api.inverse(torch.from_numpy(a.astype(dt)).cuda(), precision=prec).cpu().numpy()
    tol = 1e-12 if dt == np.float64 else 2e-6
    err = float(rel_err(x.astype(np.float64), ref))
    assert err <= tol * 1e3, (n, prec, err)
print("blocked_iv ok")
'''
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, CHOLINV_LARGE_INVERSE="blocked_iv", PYTHONPATH=root)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "blocked_iv ok" in r.stdout
