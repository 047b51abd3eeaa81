"""GPU parity of the uneven-order batch path (one persistent launch after a
device-side bucketing prologue) and of its HIP-graph capture."""
import numpy as np
import pytest

import oracle as O
from paper_1111_4144_amd import inputs as G
from tests.helpers import TOL_FP32, TOL_FP64, torch_cuda

pytestmark = pytest.mark.gpu


def _unpack(packed, sizes, offs, b):
    n = int(sizes[b])
    return packed[offs[b]:offs[b] + n * n].reshape(n, n)


def _check(xg, packed, sizes, offs, xo, tol, what):
    worst = 0.0
    for b in range(len(sizes)):
        n = int(sizes[b])
        if n == 0:
            continue
        x = _unpack(xg, sizes, offs, b).astype(np.float64)
        ref = _unpack(xo, sizes, offs, b)
        a = _unpack(packed, sizes, offs, b)
        err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
        k = O.kappa2(a.astype(np.complex128)) if n <= 64 else 1.0
        worst = max(worst, err / k)
        assert err <= tol * k, "%s: matrix %d (n=%d) err %.3e kappa %.3e" % (what, b, n, err, k)
    return worst


@pytest.mark.parametrize("dtype,prec,ns,method", [
    (np.float32, "plain", 0, "chol"), (np.float32, "plain", 0, "ldl"),
    (np.float32, "mixed", 0, "chol"), (np.float32, "mixed", 0, "ldl"),
    (np.float32, "mixed", 1, "chol"), (np.float32, "mixed", 2, "ldl"),
    (np.float64, "plain", 0, "chol"), (np.float64, "plain", 0, "ldl")])
def test_varlen_matches_oracle(dtype, prec, ns, method):
    t = torch_cuda()
    from paper_1111_4144_amd import api
    packed, sizes, offs = G.varlen_spd(3000, seed=21, dtype=dtype)
    X, info = api.inverse_varlen(t.from_numpy(packed).cuda(), t.from_numpy(sizes).cuda(),
                                 t.from_numpy(offs).cuda(), method=method, precision=prec,
                                 ns_steps=ns, return_info=True)
    t.cuda.synchronize()
    xo, io = O.inv_prop_varlen(packed, sizes, offs, method)
    assert np.array_equal(info.cpu().numpy(), io)
    tol = TOL_FP64 if dtype == np.float64 else TOL_FP32
    w = _check(X.cpu().numpy(), packed, sizes, offs, xo, tol, "varlen %s %s" % (prec, method))
    print("max err/kappa %.3e" % w)


def test_varlen_edge_cases():
    """Orders 0 (nothing to do), 1, beyond n_max (info -1, X untouched), a
    non-positive-definite matrix, and a bucket with a ragged tile."""
    t = torch_cuda()
    from paper_1111_4144_amd import api
    sizes = np.array([0, 1, 5, 64, 40, 17, 9, 3, 33, 16, 8, 70 % 65], dtype=np.int32)
    sizes[-1] = 50                                   # beyond n_max=48 below
    offs = np.zeros(len(sizes), np.int64)
    offs[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    rng = np.random.default_rng(4)
    packed = np.zeros(int(offs[-1] + sizes[-1] ** 2), np.float64)
    for b, n in enumerate(sizes):
        if n:
            packed[offs[b]:offs[b] + n * n] = G.random_hpd(rng, 1, int(n), complex_=False)[0].ravel()
    bad = 4                                          # n = 40: make pivot 7 fail
    m = _unpack(packed, sizes, offs, bad).copy()
    m[:] = np.eye(40)
    m[6, 6] = -1.0
    packed[offs[bad]:offs[bad] + 1600] = m.ravel()
    sizes_c = sizes.copy()
    sizes_c[3] = 64
    out = t.full((packed.size,), 5.0, dtype=t.float64, device="cuda")
    X, info = api.inverse_varlen(t.from_numpy(packed).cuda(), t.from_numpy(sizes).cuda(),
                                 t.from_numpy(offs).cuda(), n_max=64, out=out, return_info=True)
    info = info.cpu().numpy()
    x = X.cpu().numpy()
    xo, io = O.inv_prop_varlen(packed, sizes, offs)
    assert info[0] == 0 and info[bad] == 7 and np.all(np.isnan(_unpack(x, sizes, offs, bad)))
    good = [b for b in range(len(sizes)) if sizes[b] and b != bad]
    for b in good:
        assert info[b] == 0
        assert np.allclose(_unpack(x, sizes, offs, b), _unpack(xo, sizes, offs, b), rtol=1e-9, atol=1e-12)
    # n_max = 48: the orders 64 and 50 are rejected with info -1 and left untouched
    out2 = t.full((packed.size,), 5.0, dtype=t.float64, device="cuda")
    X2, info2 = api.inverse_varlen(t.from_numpy(packed).cuda(), t.from_numpy(sizes).cuda(),
                                   t.from_numpy(offs).cuda(), n_max=48, out=out2, return_info=True)
    info2 = info2.cpu().numpy()
    x2 = X2.cpu().numpy()
    for b in (3, len(sizes) - 1):
        assert info2[b] == -1
        assert np.all(_unpack(x2, sizes, offs, b) == 5.0)


@pytest.mark.parametrize("prec,method,fill", [("plain", "chol", True), ("plain", "ldl", False),
                                               ("mixed", "chol", False)])
def test_varlen_last_bucket_edge_cases(prec, method, fill):
    """The last bucket of a real float batch without refinement: every order
    33..64, a failing pivot near the end of an order-63 matrix, a failing first
    pivot, failing pivots in the orders padded to 48 (the first of the second
    sub-block, the last one), and with fill_lower off the lower triangles left
    untouched."""
    t = torch_cuda()
    from paper_1111_4144_amd import api
    sizes = np.concatenate([np.arange(33, 65), [63, 57, 2, 40, 48, 33]]).astype(np.int32)
    offs = np.zeros(len(sizes), np.int64)
    offs[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    rng = np.random.default_rng(31)
    packed = np.zeros(int(offs[-1] + sizes[-1] ** 2), np.float32)
    for b, n in enumerate(sizes):
        a = G.random_hpd(rng, 1, int(n), shift=0.5, complex_=False)[0]
        packed[offs[b]:offs[b] + n * n] = a.astype(np.float32).ravel()
    # order 63: pivot 62; order 57: pivot 1; order 48: pivot 17; order 33: pivot 33
    bad = {len(sizes) - 6: 62, len(sizes) - 5: 1, len(sizes) - 2: 17, len(sizes) - 1: 33}
    for b, piv in bad.items():
        n = int(sizes[b])
        m = np.eye(n, dtype=np.float32)
        m[piv - 1, piv - 1] = -2.0
        packed[offs[b]:offs[b] + n * n] = m.ravel()
    out = t.full((packed.size,), 7.0, dtype=t.float32, device="cuda")
    X, info = api.inverse_varlen(t.from_numpy(packed).cuda(), t.from_numpy(sizes).cuda(),
                                 t.from_numpy(offs).cuda(), n_max=64, method=method,
                                 precision=prec, ns_steps=0, fill_lower=fill, out=out,
                                 return_info=True)
    info = info.cpu().numpy()
    x = X.cpu().numpy()
    xo, io = O.inv_prop_varlen(packed.astype(np.float64), sizes, offs, method)
    assert np.array_equal(info, io)
    for b, piv in bad.items():
        assert info[b] == piv
        xb = _unpack(x, sizes, offs, b)
        up = np.triu(np.ones(xb.shape, bool))
        assert np.all(np.isnan(xb[up]))
    for b in range(len(sizes)):
        if b in bad:
            continue
        n = int(sizes[b])
        xb = _unpack(x, sizes, offs, b).astype(np.float64)
        ref = _unpack(xo, sizes, offs, b)
        a = _unpack(packed, sizes, offs, b).astype(np.complex128)
        up = np.triu(np.ones((n, n), bool))
        if not fill:
            assert np.all(xb[~up] == 7.0), "order %d: lower triangle written" % n
            xb = np.where(up, xb, xb.T)
        else:
            assert np.array_equal(xb, xb.T)
        err = np.linalg.norm(xb - ref) / np.linalg.norm(ref)
        assert err <= TOL_FP32 * O.kappa2(a), "order %d err %.3e" % (n, err)


@pytest.mark.parametrize("prec,ns", [("mixed", 1), ("plain", 0)])
def test_varlen_graph_capture_replays_match_eager(prec, ns):
    """Refined mixed precision (four-lane LDS route for the last bucket) and
    plain FP32 (one wave per matrix on the matrix cores)."""
    t = torch_cuda()
    from paper_1111_4144_amd import api
    packed, sizes, offs = G.varlen_spd(2000, seed=22)
    P = t.from_numpy(packed).cuda()
    S = t.from_numpy(sizes).cuda()
    F = t.from_numpy(offs).cuda()
    eager = api.inverse_varlen(P, S, F, n_max=64, precision=prec, ns_steps=ns)
    out = t.empty_like(P)
    from paper_1111_4144_amd import _lib as L
    import ctypes
    ws = L.lib().chol_workspace_size(L.CI_FN_BATCHED, L.CI_F32, len(sizes), 0, None)
    work = t.empty(ws, dtype=t.uint8, device="cuda")
    s = t.cuda.Stream()
    s.wait_stream(t.cuda.current_stream())
    with t.cuda.stream(s):                            # warm-up outside the capture
        api.inverse_varlen(P, S, F, n_max=64, precision=prec, ns_steps=ns, out=out, workspace=work)
    t.cuda.current_stream().wait_stream(s)
    g = t.cuda.CUDAGraph()
    with t.cuda.graph(g):
        api.inverse_varlen(P, S, F, n_max=64, precision=prec, ns_steps=ns, out=out, workspace=work)
    for r in range(3):
        out.fill_(float("nan"))
        junk = api.inverse_varlen(P, S, F, n_max=64)   # eager work between replays
        g.replay()
        t.cuda.synchronize()
        assert t.equal(out, eager), "replay %d differs from the eager result" % r
