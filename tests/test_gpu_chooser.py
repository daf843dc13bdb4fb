"""The trained access-path chooser against the selectivity-threshold
heuristic on held-out workloads of the chooser's distribution (kept small so
the test runs in seconds): the learned picks must be faster in total, and
every arm must return the same result."""

import math
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


def _time(T, q, pred, k, chooser, reps=3):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    T.scan_topk(q, pred, k, vrs.IP, chooser=chooser)
    best = math.inf
    for _ in range(reps):
        e0.record()
        r = T.scan_topk(q, pred, k, vrs.IP, chooser=chooser)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best, r


def test_learned_picks_beat_the_heuristic_and_never_change_results():
    vrs.lib().vrs_chooser_load(vrs.CHOOSER_WEIGHTS.encode())
    ws = [w for w in inputs.chooser_workloads(CH.CFG_HELDOUT + 7, 200)
          if w.d <= 128 and w.n <= 3_000_000][:16]
    assert len(ws) >= 8
    src = {}
    tl = th = 0.0
    for w in ws:
        if (w.d, w.dtype) not in src:
            x = inputs.table(7, 3_000_000, w.d, 1000)
            a = inputs.attributes(7, 3_000_000, 2, CH.ATTR_RANGE)
            src[(w.d, w.dtype)] = vrs.Table(torch.from_numpy(x).cuda(), torch.from_numpy(a).cuda(),
                                            store=w.dtype, normalize=True)
        T = src[(w.d, w.dtype)].view(w.n)
        q = torch.from_numpy(inputs.queries(7, w.b, w.d, 1000, stream_offset=w.seed % 1000)).cuda()
        width = inputs.two_term_width(w.sel, CH.ATTR_RANGE)
        pred = [(0, 0, width), (1, 0, width)]
        t_l, r_l = _time(T, q, pred, w.k, vrs.CHOOSER_LEARNED)
        t_h, r_h = _time(T, q, pred, w.k, vrs.CHOOSER_HEURISTIC)
        assert torch.equal(r_l.idx, r_h.idx) and torch.equal(r_l.dist, r_h.dist)
        tl += t_l
        th += t_h
    assert tl <= 1.05 * th, (tl, th)
