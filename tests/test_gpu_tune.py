"""The autotuner: it records one valid engine per order, the recorded engines
keep parity with the oracle, and a cache file written by one run is loaded
(not re-measured) by the next."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_1111_4144_amd import inputs as I
from tests.helpers import TOL_FP32, assert_within, torch_cuda

pytestmark = pytest.mark.gpu


def test_autotune_records_and_keeps_parity(tmp_path):
    torch = torch_cuda()
    from paper_1111_4144_amd import api
    cache = tmp_path / "tune.txt"
    api.autotune_clear()
    try:
        measured = api.autotune(torch.complex64, precision="mixed", orders=(6, 16), batch=4096,
                                cache=cache)
        assert measured >= 1
        engines = {n: api.tuned_engine(torch.complex64, n, precision="mixed") for n in range(6, 17)}
        for n, e in engines.items():
            # orders with a choice record one; the rest keep the built-in path
            assert e in (0, 1, 2, 3, 4, 5, 6), (n, e)
        assert any(e != 0 for e in engines.values())
        lines = cache.read_text().splitlines()
        assert len(lines) == measured
        # parity through the recorded engines (orders 8, 12, 16)
        for n in (8, 12, 16):
            a = I.mimo(n, 512, seed=4242 + n)
            x = api.inverse(torch.from_numpy(a).cuda(), precision="mixed").cpu().numpy()
            ref, _ = O.inv_prop(a)
            assert_within(x, ref, a, TOL_FP32, "tuned engine %d, order %d" % (engines[n], n))
        # a second run loads the cache instead of measuring
        api.autotune_clear()
        assert api.tuned_engine(torch.complex64, 16, precision="mixed") == 0
        again = api.autotune(torch.complex64, precision="mixed", orders=(6, 16), batch=4096,
                             cache=cache)
        assert again == 0
        assert {n: api.tuned_engine(torch.complex64, n, precision="mixed")
                for n in range(6, 17)} == engines
    finally:
        api.autotune_clear()


def test_autotune_rejects_bad_arguments():
    torch = torch_cuda()
    from paper_1111_4144_amd import api, _lib as L
    with pytest.raises(L.CholinvError):
        api.autotune(torch.float32, orders=(0, 8))
    with pytest.raises(L.CholinvError):
        api.autotune(torch.float32, orders=(4, 17))


@pytest.mark.parametrize("dt,prec", [("c64", "mixed"), ("c64", "plain"), ("f32", "mixed")])
@pytest.mark.parametrize("n", [9, 12, 16])
def test_every_engine_keeps_parity(n, dt, prec):
    """Each candidate engine of orders 9..16 (pinned with tune_set, so the
    built-in choice does not hide the others) against the oracle, on a batch
    with a ragged last block."""
    torch = torch_cuda()
    from paper_1111_4144_amd import api
    npd = np.complex64 if dt == "c64" else np.float32
    if dt == "c64":
        a = I.mimo(n, 1000, seed=900 + n)
    else:
        a = I.random_hpd(np.random.default_rng(n), 1000, n, shift=0.5, complex_=False, dtype=npd)
    ref, _ = O.inv_prop(a)
    engines = [4, 5, 6] if prec == "mixed" else [4, 6]
    api.autotune_clear()
    try:
        for e in engines:
            api.tune_set(dt, n, e, precision=prec)
            assert api.tuned_engine(dt, n, precision=prec) == e
            x = api.inverse(torch.from_numpy(a).cuda(), precision=prec).cpu().numpy()
            assert np.array_equal(x, np.conj(np.swapaxes(x, -1, -2)))
            assert_within(x, ref, a, TOL_FP32, "engine %d, %s %s order %d" % (e, dt, prec, n))
    finally:
        api.autotune_clear()
