"""Pins of the oracle's vector join: every row of R (its stored vector, as a
float32 query) against the rows of S, exact filtered top-k (the N:N strategy
of Section 3.1 with a whole relation as the query batch; the paper names
joins as the large-batch use of the tensor form, Section 5.2).  Checked
against exact rational distances with a full sort, the self-join's closed
forms (every row is its own nearest neighbour, ties by lower id) and the
exact symmetry of the squared-L2 chain."""

from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def _exact_l2(a, b):
    return sum((Fraction(float(u)) - Fraction(float(v))) ** 2 for u, v in zip(a, b))


def _exact_ip(a, b):
    return -sum(Fraction(float(u)) * Fraction(float(v)) for u, v in zip(a, b))


def test_join_matches_a_full_exact_sort():
    rng = np.random.default_rng(11)
    nr, ns, d, k = 25, 80, 5, 7
    r = rng.standard_normal((nr, d)).astype(np.float32)
    s = rng.standard_normal((ns, d)).astype(np.float32)
    a = rng.integers(0, 3, (1, ns)).astype(np.int32)
    tr, ts = O.Table(O.F32, r, np.zeros((1, nr), np.int32)), O.Table(O.F32, s, a)
    for metric, fn in ((O.L2SQ, _exact_l2), (O.IP, _exact_ip)):
        for pred in ([], [(0, 1, 3)]):
            idx, dist, _, nv = O.join_topk(tr, ts, pred, k, metric)
            for i in range(nr):
                qual = [j for j in range(ns) if not pred or 1 <= a[0, j] < 3]
                want = sorted(qual, key=lambda j: (fn(r[i], s[j]), j))[:k]
                assert list(idx[i][:len(want)]) == want
                assert nv[i] == min(k, len(qual))


def test_self_join_closed_forms_and_symmetry():
    rng = np.random.default_rng(12)
    n, d = 300, 16
    x = rng.standard_normal((n, d)).astype(np.float32)
    x[200] = x[17]  # a duplicate: row 17 and row 200 both have 17 first
    t = O.Table(O.F32, x, np.zeros((1, n), np.int32))
    idx, dist, d64, _ = O.join_topk(t, t, [], 5, O.L2SQ)
    for i in range(n):
        if i in (17, 200):
            assert list(idx[i][:2]) == [17, 200] and dist[i][0] == 0.0 and dist[i][1] == 0.0
        else:
            assert idx[i][0] == i and dist[i][0] == 0.0
    # the squared-L2 chain is symmetric bit for bit: (a - b)^2 == (b - a)^2
    for i in range(0, n, 7):
        for c in range(1, 5):
            j = idx[i][c]
            back = O.distances(t, x[j], np.array([i]), O.L2SQ)[0]
            assert back == d64[i][c]


@pytest.mark.parametrize("dtype", [O.BF16, O.FP8])
def test_join_queries_are_the_stored_values(dtype):
    rng = np.random.default_rng(13)
    x = rng.standard_normal((200, 32)).astype(np.float32)
    t = O.Table.build(x, np.zeros((1, 200), np.int32), dtype, normalize=True)
    q = O.stored_as_f32(t)
    if dtype == O.BF16:
        assert np.array_equal(q.view(np.uint32) & 0xffff, np.zeros_like(q.view(np.uint32)))
    else:
        vals = O.e4m3_values(t.rows).reshape(t.n, t.d)
        assert np.array_equal(q, (vals * t.scale[:, None].astype(np.float64)).astype(np.float32))
    idx, _, d64, _ = O.join_topk(t, t, [], 3, O.IP)
    # a normalised stored row is at least as similar to itself as the rows
    # around it: its own distance is within rounding of the best one
    for i in range(200):
        own = O.distances(t, q[i], np.array([i]), O.IP)[0]
        assert own <= d64[i][0] + 1e-2
