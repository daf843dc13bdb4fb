"""vrs_scan_topk_noalloc (the scan with its workspace in a static device
array, for callers that cannot allocate) against vrs_scan_topk on the same
inputs, through the C ABI: two calls in a row, the second with a smaller
input, ids and distances bit-identical; a call needing more workspace than
the array holds is refused."""

import ctypes as C

import numpy as np
import pytest
import torch

from paper_2403_15807_amd import inputs, vrs

pytestmark = pytest.mark.gpu
I32_MIN = -(2 ** 31)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _noalloc(T, q, terms, k, metric, strategy=vrs.STRATEGY_AUTO):
    B = q.shape[0]
    idx = torch.full((B, k), -7, dtype=torch.int64, device="cuda")
    dist = torch.full((B, k), -7.0, dtype=torch.float32, device="cuda")
    nv = torch.empty(B, dtype=torch.int32, device="cuda")
    cert = torch.empty(B, dtype=torch.uint8, device="cuda")
    o = vrs.vrs_opts()
    o.strategy, o.tile = strategy, -1
    o.n_valid, o.certified = nv.data_ptr(), cert.data_ptr()
    p = vrs.make_pred(terms)
    st = vrs.lib().vrs_scan_topk_noalloc(T.handle, C.c_void_p(q.data_ptr()), B, C.byref(p), k, metric,
                                         C.c_void_p(idx.data_ptr()), C.c_void_p(dist.data_ptr()), C.byref(o),
                                         None)
    torch.cuda.synchronize()
    return st, idx, dist, nv


def test_noalloc_matches_the_workspace_entry_point_twice():
    assert torch.cuda.is_available()
    n, d = 100_000, 128
    x = inputs.table(0, n, d, 100)
    a = inputs.attributes(0, n, 1, 100)
    T = vrs.Table(_dev(x), _dev(a))
    # first call, then a smaller one (fewer queries, smaller k, other predicate)
    for B, k, terms, metric, strategy in ((16, 10, [(0, I32_MIN, 10)], vrs.L2SQ, vrs.STRATEGY_MASK),
                                          (3, 4, [(0, 20, 23)], vrs.L2SQ, vrs.STRATEGY_GATHER)):
        q = _dev(inputs.queries(0, B, d, 100, stream_offset=B))
        ref = T.scan_topk(q, terms, k, metric, strategy=strategy)
        st, idx, dist, nv = _noalloc(T, q, terms, k, metric, strategy)
        assert st == vrs.VRS_OK, vrs.lib().vrs_last_error()
        assert torch.equal(idx, ref.idx)
        assert torch.equal(dist.view(torch.int32), ref.dist.view(torch.int32))
        assert torch.equal(nv, ref.n_valid)
    T.close()


def test_noalloc_refuses_a_scan_larger_than_its_scratch():
    n, d = 200_000, 128
    x = inputs.table(0, n, d, 100)
    T = vrs.Table(_dev(x), None)
    B, k = 8192, 256
    need = T.workspace_bytes(B, k)
    assert need > vrs.NOALLOC_SCRATCH_BYTES
    q = _dev(inputs.queries(0, B, d, 100))
    st, idx, dist, _ = _noalloc(T, q, [], k, vrs.L2SQ)
    assert st == vrs.VRS_E_WORKSPACE
    assert b"static scratch" in vrs.lib().vrs_last_error()
    assert (idx == -7).all()  # nothing launched, outputs untouched
    T.close()
