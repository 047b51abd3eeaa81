"""The autotuner: it records one valid engine per order, the recorded engines
keep parity with the oracle, and a cache file written by one run is loaded
(not re-measured) by the next."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from paper_1111_4144_amd import inputs as I
from tests.helpers import TOL_FP32, TOL_FP64, assert_within, torch_cuda

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


@pytest.mark.parametrize("dt", ["c128", "f64"])
@pytest.mark.parametrize("n", [1, 3, 8, 9, 13, 16])
@pytest.mark.parametrize("method", ["chol", "ldl"])
def test_eight_lane_engine_keeps_parity(n, dt, method):
    """The eight-lanes-per-matrix FP64 engine (one column per lane up to order
    8, two above), pinned with tune_set, against the oracle on a batch whose
    last wave is ragged; the sixteen-lane engine on the same batch for
    comparison."""
    torch = torch_cuda()
    from paper_1111_4144_amd import api
    cplx = dt == "c128"
    a = I.random_hpd(np.random.default_rng(300 + n), 1001, n, shift=0.5, complex_=cplx,
                     dtype=np.complex128 if cplx else np.float64)
    ref, _ = O.inv_prop(a, method=method)
    api.autotune_clear()
    try:
        for e in (7, 4):
            api.tune_set(dt, n, e, method=method)
            x = api.inverse(torch.from_numpy(a).cuda(), method=method).cpu().numpy()
            assert np.array_equal(x, np.conj(np.swapaxes(x, -1, -2)))
            assert_within(x, ref, a, TOL_FP64, "engine %d, %s %s order %d" % (e, dt, method, n))
    finally:
        api.autotune_clear()


def test_autotune_large_records_a_configuration(tmp_path):
    """Tuning a large order records one of the configurations for its bucket,
    keeps parity through it, and is loaded from the cache by a second run."""
    torch = torch_cuda()
    from paper_1111_4144_amd import api
    cache = tmp_path / "tune_large.txt"
    api.autotune_clear()
    try:
        assert api.autotune(torch.float32, precision="mixed", orders=(520, 520), cache=cache) == 1
        cfg = api.tuned_engine(torch.float32, 520, precision="mixed")
        assert 0 <= cfg <= 5
        assert api.tuned_engine(torch.float32, 600, precision="mixed") == cfg   # same bucket
        a = I.large_spd(520, seed=8, top=1e3, dtype=np.float32).astype(np.float64)
        ref, _ = O.inv_prop(a)
        x = api.inverse(torch.from_numpy(a.astype(np.float32)).cuda(), precision="mixed")
        err = float(np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref))
        assert err <= TOL_FP32 * 1e3, (cfg, err)
        api.autotune_clear()
        assert api.autotune(torch.float32, precision="mixed", orders=(520, 520), cache=cache) == 0
        assert api.tuned_engine(torch.float32, 520, precision="mixed") == cfg
    finally:
        api.autotune_clear()


@pytest.mark.parametrize("prec,ns", [("plain", 0), ("mixed", 1)])
def test_autotune_varlen_edges_keep_parity(prec, ns):
    """The uneven-batch tuner returns one of its bucket edges; every edge
    (pinned) keeps parity with the oracle on a batch that spans all sizes."""
    torch = torch_cuda()
    from paper_1111_4144_amd import api
    packed, sizes, offs = I.varlen_spd(1500, seed=31)
    P = torch.from_numpy(packed).cuda()
    S = torch.from_numpy(sizes).cuda()
    OF = torch.from_numpy(offs).cuda()
    xo, io = O.inv_prop_varlen(packed, sizes, offs)
    api.autotune_clear()
    try:
        edge = api.autotune_varlen(P, S, OF, n_max=64, precision=prec, ns_steps=ns)
        assert edge in (17, 25, 33)
        assert api.tuned_engine(torch.float32, 0, precision=prec) == edge
        for e in (17, 25, 33):
            api.tune_set(torch.float32, 0, e, precision=prec)
            x, info = api.inverse_varlen(P, S, OF, n_max=64, precision=prec, ns_steps=ns,
                                         return_info=True)
            x = x.cpu().numpy()
            assert np.array_equal(info.cpu().numpy(), io)
            for b in range(0, 1500, 5):
                n, o = int(sizes[b]), int(offs[b])
                xm = x[o:o + n * n].reshape(n, n).astype(np.float64)
                ref = xo[o:o + n * n].reshape(n, n)
                err = np.linalg.norm(xm - ref) / np.linalg.norm(ref)
                kap = O.kappa2(packed[o:o + n * n].reshape(n, n).astype(np.complex128))
                assert err <= TOL_FP32 * kap, (e, b, n, err)
    finally:
        api.autotune_clear()


def test_refinement_three_product_form_matches_four_product_form():
    """The MFMA refinement forms complex products with three real products
    ((Ar + Ai)(Xr + Xi) among them) where the lane form uses four; the extra
    FP32 rounding sits in the small correction X E and must not show in the
    refined inverse: on the same 16 x 16 MIMO matrices the three-product
    engines (5, 6) stay within twice the four-product engine's (4) error
    against the oracle, in the median and the maximum."""
    torch = torch_cuda()
    from paper_1111_4144_amd import api
    a = I.mimo(16, 2000, seed=4711)
    ref, _ = O.inv_prop(a)
    A = torch.from_numpy(a).cuda()
    errs = {}
    api.autotune_clear()
    try:
        for e in (4, 5, 6):
            api.tune_set("c64", 16, e, precision="mixed")
            x = api.inverse(A, precision="mixed", ns_steps=1).cpu().numpy()
            errs[e] = np.linalg.norm(x - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))
    finally:
        api.autotune_clear()
    for e in (5, 6):
        assert np.median(errs[e]) <= 2 * np.median(errs[4]), (e, np.median(errs[e]), np.median(errs[4]))
        assert errs[e].max() <= 2 * errs[4].max(), (e, errs[e].max(), errs[4].max())
