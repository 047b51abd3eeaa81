"""The allocation-free entry point chol_inverse_batched_noalloc, called through
the C-ABI: on two uneven batches in a row (the second smaller, so the shared
library-held plan must be rebuilt, not reused), and on a uniform batch, its
results must equal those of chol_inverse_batched with a caller workspace bit
for bit (the same kernels run on the same matrices), and match the oracle."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle as O
from paper_1111_4144_amd import inputs as G
from tests.helpers import TOL_FP32, torch_cuda

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _noalloc_varlen(torch, P, S, OF, n_max, opts):
    from paper_1111_4144_amd import _lib as L
    X = torch.full_like(P, float("nan"))
    info = torch.full((S.shape[0],), 7, dtype=torch.int32, device=P.device)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.lib().chol_inverse_batched_noalloc(L.CI_F32, S.shape[0], 0, _ptr(S), _ptr(OF), n_max,
                                              _ptr(P), 0, _ptr(X), 0, ctypes.byref(opts),
                                              _ptr(info), s)
    L.check("chol_inverse_batched_noalloc", rc)
    torch.cuda.synchronize()
    return X.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("prec,ns", [("plain", 0), ("mixed", 1)])
def test_noalloc_varlen_matches_workspace_entry_point(prec, ns):
    torch = torch_cuda()
    from paper_1111_4144_amd import _lib as L, api
    opts = L.make_opts("chol", prec, ns, True)
    for count, seed in ((3000, 61), (700, 62)):           # the second call is smaller
        packed, sizes, offs = G.varlen_spd(count, seed=seed)
        P = torch.from_numpy(packed).cuda()
        S = torch.from_numpy(sizes).cuda()
        OF = torch.from_numpy(offs).cuda()
        xw, iw = api.inverse_varlen(P, S, OF, n_max=64, precision=prec, ns_steps=ns,
                                    return_info=True)
        xw, iw = xw.cpu().numpy(), iw.cpu().numpy()
        xn, inn = _noalloc_varlen(torch, P, S, OF, 64, opts)
        assert np.array_equal(inn, iw)
        assert np.array_equal(xn, xw), "count %d: outputs differ" % count
        xo, io = O.inv_prop_varlen(packed, sizes, offs)
        assert np.array_equal(inn, io)
        for b in range(0, count, 7):
            n, o = int(sizes[b]), int(offs[b])
            x = xn[o:o + n * n].reshape(n, n).astype(np.float64)
            ref = xo[o:o + n * n].reshape(n, n)
            a = packed[o:o + n * n].reshape(n, n)
            err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
            assert err <= TOL_FP32 * O.kappa2(a.astype(np.complex128)), (count, b, n, err)


def test_noalloc_uniform_batch():
    torch = torch_cuda()
    from paper_1111_4144_amd import _lib as L, api
    a = G.mimo(8, 1000, seed=63)
    A = torch.from_numpy(a).cuda()
    want = api.inverse(A, precision="mixed", ns_steps=1).cpu().numpy()
    X = torch.empty_like(A)
    opts = L.make_opts("chol", "mixed", 1, True)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.lib().chol_inverse_batched_noalloc(L.CI_C64, 1000, 8, None, None, 0, _ptr(A), 64,
                                              _ptr(X), 64, ctypes.byref(opts), None, s)
    L.check("chol_inverse_batched_noalloc", rc)
    torch.cuda.synchronize()
    assert np.array_equal(X.cpu().numpy(), want)


def test_noalloc_rejects_batches_beyond_the_scratch():
    torch_cuda()
    from paper_1111_4144_amd import _lib as L
    p = ctypes.c_void_p(0x1000)          # never dereferenced: the size check fails first
    opts = L.make_opts()
    rc = L.lib().chol_inverse_batched_noalloc(L.CI_F32, L.CI_NOALLOC_MAX_BATCH + 1, 0, p, p, 64,
                                              p, 0, p, 0, ctypes.byref(opts), None, None)
    assert rc == L.CI_ERR_NOALLOC_LIMIT
    assert "scratch" in L.status_string(rc)
