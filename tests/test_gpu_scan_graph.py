"""The single-predicate scan captured into a HIP graph: every replay, with
new query vectors written into the captured buffer and eager work and
synchronisations of the program in between, returns what the eager call
returns for the same queries (ids and distances bit for bit)."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2403_15807_amd import inputs, vrs

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("B,strategy,tile", [(1, vrs.STRATEGY_MASK, 0), (1, vrs.STRATEGY_GATHER, 0),
                                             (4, vrs.STRATEGY_AUTO, -1), (16, vrs.STRATEGY_MASK, 4),
                                             (70, vrs.STRATEGY_GATHER, 5)])
def test_graph_replays_equal_eager_calls(B, strategy, tile):
    n, d, k = 40001, 128, 50
    x = inputs.table(21, n, d, 100)
    a = inputs.attributes(21, n, 2, 1000)
    T = vrs.Table(_dev(x), _dev(a))
    pred = [(0, 0, 400), (1, 100, 900)]
    q = _dev(inputs.queries(21, B, d, 100))
    g = T.scan_graph(q, pred, k, vrs.L2SQ, strategy=strategy, tile=tile)
    torch.cuda.synchronize()
    ot = O.Table(O.F32, x, a)
    ref0 = O.scan_topk(ot, q.cpu().numpy(), pred, k, O.L2SQ)
    assert np.array_equal(g.result.idx.cpu().numpy(), ref0[0])  # the creating (eager) run
    for rep in range(5):
        qh = inputs.queries(22 + rep, B, d, 100)
        q.copy_(_dev(qh))
        g.launch()
        torch.cuda.synchronize()
        got_i, got_d = g.result.idx.clone(), g.result.dist.clone()
        # the program's own eager work between replays
        e = T.scan_topk(_dev(qh), pred, k, vrs.L2SQ, strategy=strategy, tile=tile)
        other = T.scan_topk(_dev(inputs.queries(90 + rep, 3, d, 100)), [(0, 0, 999)], 7, vrs.L2SQ)
        torch.cuda.synchronize()
        assert torch.equal(got_i, e.idx), rep
        assert torch.equal(got_d.view(torch.int32), e.dist.view(torch.int32)), rep
        assert other.idx.shape == (3, 7)
    ref = O.scan_topk(ot, qh, pred, k, O.L2SQ)
    assert np.array_equal(got_i.cpu().numpy(), ref[0])
    g.close()
