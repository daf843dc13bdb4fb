"""The access-path chooser never changes results: on workloads of the
chooser's distribution (float32, bfloat16 and FP8 tables), the learned pick,
the heuristic pick and every other available arm return the same ids and
distances.  (Its timing quality is judged on recorded held-out timings by
tests/test_chooser_regret.py, deterministically.)"""

import os

import numpy as np
import pytest
import torch

from paper_2403_15807_amd import chooser as CH
from paper_2403_15807_amd import inputs, vrs

pytestmark = pytest.mark.gpu


def test_shipped_weights_load():
    vrs.lib()
    assert os.path.exists(vrs.CHOOSER_WEIGHTS)
    assert vrs.lib().vrs_chooser_load(vrs.CHOOSER_WEIGHTS.encode()) == vrs.VRS_OK


@pytest.mark.parametrize("store,d", [(vrs.F32, 128), (vrs.BF16, 768), (vrs.FP8E4M3, 768)])
def test_every_arm_returns_the_same_result(store, d):
    vrs.lib().vrs_chooser_load(vrs.CHOOSER_WEIGHTS.encode())
    n = 400_000
    x = inputs.table(7, n, d, 1000)
    a = inputs.attributes(7, n, 2, CH.ATTR_RANGE)
    T = vrs.Table(torch.from_numpy(x).cuda(), torch.from_numpy(a).cuda(), store=store, normalize=True)
    nt = vrs.num_tiles()
    for B, sel, k in ((1, 0.3, 10), (24, 0.01, 100), (300, 0.9, 1)):
        q = torch.from_numpy(inputs.queries(7, B, d, 1000, stream_offset=B)).cuda()
        width = inputs.two_term_width(sel, CH.ATTR_RANGE)
        pred = [(0, 0, width), (1, 0, width)]
        ref = T.scan_topk(q, pred, k, vrs.IP, chooser=vrs.CHOOSER_LEARNED)
        outs = [T.scan_topk(q, pred, k, vrs.IP, chooser=vrs.CHOOSER_HEURISTIC)]
        for s in (vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER):
            for t in range(nt):
                _, su, tu = T.plan(B, pred, k, vrs.IP, strategy=s, tile=t, chooser=vrs.CHOOSER_HEURISTIC)
                if su != s or tu != t:
                    continue  # arm not available for this table and k
                if t < 4 and (B + [1, 2, 4, 8][t] - 1) // [1, 2, 4, 8][t] > 64:
                    continue  # a streaming tile that would re-read the table too often to run here
                outs.append(T.scan_topk(q, pred, k, vrs.IP, strategy=s, tile=t))
        torch.cuda.synchronize()
        for r in outs:
            assert torch.equal(r.idx, ref.idx), (store, B, sel, k)
            assert torch.equal(r.dist.view(torch.int32), ref.dist.view(torch.int32)), (store, B, sel, k)
    T.close()
