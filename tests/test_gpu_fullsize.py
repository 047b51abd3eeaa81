"""The MIMO batch at its full size (524,288 complex64 matrices per order),
launched as the benchmark launches it (engines chosen by the autotuner on
this device, mixed precision with one Newton-Schulz step, and plain FP64 on
the same matrices in complex128), checked against the oracle on sampled
matrices (the first, the last and 2046 drawn at random)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_1111_4144_amd import inputs as I
from tests.helpers import TOL_FP32, TOL_FP64, assert_within, torch_cuda

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
