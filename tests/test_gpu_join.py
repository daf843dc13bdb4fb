"""GPU parity of the vector join (vrs_join_topk) against the FP64 oracle:
every row of R, as its stored vector, is a query against S (the N:N form of
Section 3.1 with a whole relation as the batch).  Ids equal, distances
bit-identical, per-row n_valid, over several batches of R."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2403_15807_amd import inputs, vrs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _ready(oracle_lib):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return oracle_lib


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _check(r, ref, what):
    torch.cuda.synchronize()
    gi, gd = r.idx.cpu().numpy(), r.dist.cpu().numpy()
    bad = np.nonzero((gi != ref[0]).any(axis=1))[0]
    assert bad.size == 0, f"{what}: ids differ in rows {bad[:8]}"
    assert np.array_equal(gd.view(np.uint32), ref[1].view(np.uint32)), f"{what}: distances"
    assert np.array_equal(r.n_valid.cpu().numpy(), ref[3]), f"{what}: n_valid"


@pytest.mark.parametrize("metric", [vrs.L2SQ, vrs.IP])
def test_self_join_f32(metric):
    n, d = 12000, 64  # two batches of R (8192 + 3808)
    x = inputs.table(6, n, d, 40)
    a = inputs.attributes(6, n, 1, 10)
    norm = metric == vrs.IP
    T = vrs.Table(_dev(x), _dev(a), normalize=norm)
    ot = O.Table.build(x, a, O.F32, normalize=norm)
    for pred in ([], [(0, 0, 4)]):
        ref = O.join_topk(ot, ot, pred, 10, metric)
        r = T.join_topk(T, pred, 10, metric, diag=True)
        _check(r, ref, f"self-join metric {metric} pred {pred}")
        assert (r.err_ratio.cpu().numpy() < 1.0).all()


@pytest.mark.parametrize("store", [vrs.BF16, vrs.FP8E4M3])
def test_join_quantised_tables(store):
    # R stored in low precision (its stored values are the queries) against
    # S stored the same way
    nr, ns, d = 3000, 30000, 256
    xr = inputs.table(7, nr, d, 30)
    xs = inputs.table(8, ns, d, 30)
    a = inputs.attributes(8, ns, 1, 10)
    R = vrs.Table(_dev(xr), None, store=store, normalize=True)
    S = vrs.Table(_dev(xs), _dev(a), store=store, normalize=True)
    dt = O.BF16 if store == vrs.BF16 else O.FP8
    orr = O.Table.build(xr, np.zeros((1, nr), np.int32), dt, normalize=True)
    ors = O.Table.build(xs, a, dt, normalize=True)
    for pred in ([], [(0, 2, 9)]):
        ref = O.join_topk(orr, ors, pred, 5, O.IP)
        _check(R.join_topk(S, pred, 5, vrs.IP), ref, f"store {store} pred {pred}")


def test_join_argument_errors():
    x = inputs.table(6, 1000, 64, 10)
    y = inputs.table(6, 1000, 32, 10)
    A, Bt = vrs.Table(_dev(x), None), vrs.Table(_dev(y), None)
    with pytest.raises(vrs.VrsError) as e:
        A.join_topk(Bt, [], 5, vrs.L2SQ)
    assert e.value.status == vrs.VRS_E_ARG
    with pytest.raises(vrs.VrsError) as e:
        A.join_topk(A, [], 0, vrs.L2SQ)
    assert e.value.status == vrs.VRS_E_ARG
