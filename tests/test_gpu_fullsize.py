"""The batched workloads at their full sizes, launched as the benchmark
launches them, checked against the oracle on sampled matrices:

* the MIMO batch (524,288 complex64 matrices per order; engines chosen by the
  autotuner on this device, mixed precision with one Newton-Schulz step, and
  plain FP64 on the same matrices in complex128): the first, the last and
  2046 drawn at random;
* the uneven batch (262,144 real float matrices of orders 2..64, packed; the
  bucket edge chosen by the tuner on the batch, and the lowest edge, which
  sends orders 17..64 to the matrix cores): the first, the last and three of
  every order;
* the differentiation workload (65,536 complex64 16x16, forward in mixed
  precision with one Newton-Schulz step, then the hand-written backward):
  the gradient of the first, the last and 2046 drawn at random against the
  oracle's analytic gradient at the exact inverse."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_1111_4144_amd import inputs as I
from tests.helpers import TOL_FP32, TOL_FP64, assert_within, kappas, rel_err, torch_cuda

pytestmark = pytest.mark.gpu

COUNT = 524288


@pytest.mark.parametrize("n", [8, 16])
def test_mimo_full_size_sampled(n):
    torch = torch_cuda()
    from paper_1111_4144_amd import api
    api.autotune_clear()
    try:
        api.autotune(torch.complex64, precision="mixed", ns_steps=1, orders=(n, n), batch=COUNT)
        a = I.mimo(n, COUNT)
        A = torch.from_numpy(a).cuda()
        x, info = api.inverse(A, precision="mixed", ns_steps=1, return_info=True)
        rng = np.random.default_rng(31 + n)
        idx = np.unique(np.concatenate([[0, COUNT - 1], rng.choice(COUNT, 2046, replace=False)]))
        xs = x.cpu().numpy()[idx]
        assert not info.cpu().numpy().any()
        ref, io = O.inv_prop(a[idx])
        assert not io.any()
        e, r = assert_within(xs, ref, a[idx], TOL_FP32, "full-size %dx%d mixed" % (n, n))
        print("%dx%d mixed ns=1 (engine %d): max rel err %.3e, max err/kappa %.3e"
              % (n, n, api.tuned_engine(torch.complex64, n, precision="mixed"), e, r))
        del x
        y = api.inverse(A.to(torch.complex128)).cpu().numpy()[idx]
        e, r = assert_within(y, ref, a[idx], TOL_FP64, "full-size %dx%d plain c128" % (n, n))
        print("%dx%d plain FP64: max rel err %.3e, max err/kappa %.3e" % (n, n, e, r))
    finally:
        api.autotune_clear()


VARLEN_COUNT = 262144


def test_varlen_full_size_sampled():
    torch = torch_cuda()
    from paper_1111_4144_amd import api
    packed, sizes, offs = I.varlen_spd(VARLEN_COUNT)
    P = torch.from_numpy(packed).cuda()
    S = torch.from_numpy(sizes).cuda()
    OF = torch.from_numpy(offs).cuda()
    ws = torch.empty(api.varlen_workspace_bytes(P, VARLEN_COUNT), dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(47)
    pick = [0, VARLEN_COUNT - 1]
    for n in np.unique(sizes):
        pick += list(rng.choice(np.nonzero(sizes == n)[0], 3, replace=False))
    pick = np.unique(np.array(pick))
    api.autotune_clear()
    try:
        tuned = api.autotune_varlen(P, S, OF, n_max=64, workspace=ws)
        for edge in sorted({tuned, 17}):
            api.tune_set(torch.float32, 0, edge)
            X, info = api.inverse_varlen(P, S, OF, n_max=64, workspace=ws, return_info=True)
            assert not info.cpu().numpy().any()
            x = X.cpu().numpy()
            worst = 0.0
            for n in np.unique(sizes[pick]):
                bs = pick[sizes[pick] == n]
                a = np.stack([packed[offs[b]:offs[b] + n * n].reshape(n, n) for b in bs])
                xs = np.stack([x[offs[b]:offs[b] + n * n].reshape(n, n) for b in bs])
                ref, io = O.inv_prop(a.astype(np.float64))
                assert not io.any()
                e, r = assert_within(xs.astype(np.float64), ref, a.astype(np.float64), TOL_FP32,
                                     "full-size uneven batch, edge %d, order %d" % (edge, n))
                worst = max(worst, r)
            print("uneven batch, edge %d: %d sampled matrices, max err/kappa %.3e"
                  % (edge, len(pick), worst))
    finally:
        api.autotune_clear()


GRAD_COUNT = 65536


def test_differentiation_full_size_sampled():
    torch = torch_cuda()
    from paper_1111_4144_amd import api
    a, g = I.grad_16(count=GRAD_COUNT)
    A = torch.from_numpy(a).cuda().requires_grad_(True)
    X = api.CholInverse.apply(A, "chol", "mixed", 1)
    X.backward(torch.from_numpy(g).cuda())
    rng = np.random.default_rng(53)
    idx = np.unique(np.concatenate([[0, GRAD_COUNT - 1],
                                    rng.choice(GRAD_COUNT, 2046, replace=False)]))
    ga = A.grad.cpu().numpy()[idx]
    xo, io = O.inv_prop(a[idx])
    assert not io.any()
    want = O.grad(xo, g[idx])
    err = rel_err(ga, want)
    bound = 2 * TOL_FP32 * kappas(a[idx]) + 1e-5
    assert np.all(err <= bound), (err / bound).max()
    assert np.array_equal(ga, np.conj(np.swapaxes(ga, -1, -2)))      # exactly Hermitian
    print("differentiation, %d sampled of %d: max grad rel err %.3e" % (len(idx), GRAD_COUNT,
                                                                       err.max()))
