"""Pins of the oracle's threshold selection (Section 3, the selection with a
query vector and a similarity predicate, eq. 1 and eq. 3; the evaluation's
similarity predicate is a cosine-similarity threshold, Section 5 "Dataset").

The selection of query b is the set of qualifying rows whose FP64 distance is
below thr[b], ascending by row id.  It is checked against exact rational
arithmetic (thresholds placed in wide gaps of the exact distances, where the
FP64 rounding cannot move a row across), closed forms, and the top-k of the
same oracle."""

from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def _exact_dist(q, xs, scale, metric):
    """Exact rational distance of the stored values (no rounding)."""
    if metric == O.L2SQ:
        return sum((Fraction(float(a)) - Fraction(scale) * Fraction(b)) ** 2 for a, b in zip(q, xs))
    return -Fraction(scale) * sum(Fraction(float(a)) * Fraction(b) for a, b in zip(q, xs))


def _stored(ot, i):
    if ot.dtype == O.F32:
        return [float(v) for v in ot.rows[i]], 1.0
    if ot.dtype == O.BF16:
        return [float(v) for v in O.bf16_values(ot.rows[i])], 1.0
    return [float(v) for v in O.e4m3_values(ot.rows[i])], float(ot.scale[i])


def _gap_thresholds(exact, m=4):
    """Thresholds at midpoints of the widest gaps between distinct exact
    distances (far wider than any FP64 rounding)."""
    u = sorted(set(exact))
    gaps = sorted(((u[i + 1] - u[i], i) for i in range(len(u) - 1)), reverse=True)[:m]
    return [float((u[i] + u[i + 1]) / 2) for _, i in gaps]


@pytest.mark.parametrize("dtype,metric", [(O.F32, O.L2SQ), (O.F32, O.IP), (O.BF16, O.IP), (O.FP8, O.IP)])
def test_range_is_the_exact_set_below_the_threshold(dtype, metric):
    rng = np.random.default_rng(5)
    n, d = 300, 6
    x = rng.standard_normal((n, d)).astype(np.float32)
    a = rng.integers(0, 4, (1, n)).astype(np.int32)
    ot = O.Table.build(x, a, dtype)
    q = rng.standard_normal((1, d)).astype(np.float32)
    exact = [_exact_dist(q[0], *_stored(ot, i), metric) for i in range(n)]
    for pred in ([], [(0, 1, 3)]):
        qual = [i for i in range(n) if not pred or 1 <= a[0, i] < 3]
        for thr in _gap_thresholds([exact[i] for i in qual]):
            want = [i for i in qual if exact[i] < Fraction(thr)]
            idx, dist, d64, cnt = O.scan_range(ot, q, pred, thr, n, metric)
            assert cnt[0] == len(want)
            assert list(idx[0][:cnt[0]]) == want
            assert (idx[0][cnt[0]:] == -1).all() and np.isinf(dist[0][cnt[0]:]).all()
            for j, i in enumerate(want):
                assert abs(d64[0][j] - float(exact[i])) <= 1e-12 * max(1.0, abs(float(exact[i])))


def test_range_count_beyond_capacity_keeps_the_lowest_ids():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((500, 8)).astype(np.float32)
    ot = O.Table(O.F32, x, np.zeros((1, 500), np.int32))
    q = rng.standard_normal((2, 8)).astype(np.float32)
    full = O.scan_range(ot, q, [], 16.0, 500, O.L2SQ)
    cut = O.scan_range(ot, q, [], 16.0, 7, O.L2SQ)
    for b in range(2):
        assert cut[3][b] == full[3][b] > 7
        assert np.array_equal(cut[0][b], full[0][b][:7])
        assert np.array_equal(cut[1][b], full[1][b][:7])


def test_range_sets_nest_and_match_the_topk_order_statistics():
    rng = np.random.default_rng(7)
    n, d, k = 2000, 16, 50
    x = rng.standard_normal((n, d)).astype(np.float32)
    a = rng.integers(0, 5, (1, n)).astype(np.int32)
    ot = O.Table(O.F32, x, a)
    q = rng.standard_normal((3, d)).astype(np.float32)
    pred = [(0, 0, 4)]
    ti, _, td64, _ = O.scan_topk(ot, q, pred, k, O.L2SQ)
    prev = None
    for j in (0, 9, 49):
        # just above the (j+1)-th smallest distance: exactly the rows at or
        # below it, i.e. the top-(j+1) set plus any row tied with it
        thr = np.nextafter(td64[:, j], np.inf)
        idx, _, _, cnt = O.scan_range(ot, q, pred, thr, n, O.L2SQ)
        for b in range(3):
            got = set(idx[b][:cnt[b]])
            assert np.unique(td64[b]).size == k  # continuous data: no ties
            assert got == set(ti[b][:j + 1]) and cnt[b] == j + 1
            assert list(idx[b][:cnt[b]]) == sorted(got)
            if prev is not None:
                assert prev[b] <= got
        prev = [set(idx[b][:cnt[b]]) for b in range(3)]


def test_range_closed_forms():
    d = 8
    e = np.eye(d, dtype=np.float32)
    x = np.concatenate([e, -e, e]).astype(np.float32)        # rows 0..7 basis, 8..15 negated, 16..23 again
    ot = O.Table(O.F32, x, np.zeros((1, 3 * d), np.int32))
    q = e[[2]]
    # cosine similarity > 0.5 on unit vectors = IP distance < -0.5: the copies of e_2
    idx, dist, _, cnt = O.scan_range(ot, q, [], -0.5, 10, O.IP)
    assert cnt[0] == 2 and list(idx[0][:2]) == [2, 18] and list(dist[0][:2]) == [-1.0, -1.0]
    # orthogonal rows have similarity exactly 0: similarity > 0 is the same set
    assert O.scan_range(ot, q, [], -0.0, 10, O.IP)[3][0] == 2
    # similarity > -2 selects everything; > 1 nothing
    assert O.scan_range(ot, q, [], 2.0, 30, O.IP)[3][0] == 3 * d
    assert O.scan_range(ot, q, [], -1.0, 30, O.IP)[3][0] == 0
    # squared L2 below 0 is empty (strict), just above 0 the exact copies
    assert O.scan_range(ot, q, [], 0.0, 30, O.L2SQ)[3][0] == 0
    idx, dist, _, cnt = O.scan_range(ot, q, [], 1e-30, 30, O.L2SQ)
    assert cnt[0] == 2 and list(idx[0][:2]) == [2, 18] and dist[0][0] == 0.0
    # +inf threshold: every qualifying row, -inf: none
    assert O.scan_range(ot, q, [], np.inf, 30, O.L2SQ)[3][0] == 3 * d
    assert O.scan_range(ot, q, [], -np.inf, 30, O.L2SQ)[3][0] == 0


def test_range_with_predicate_is_the_intersection():
    rng = np.random.default_rng(8)
    n, d = 3000, 12
    x = rng.standard_normal((n, d)).astype(np.float32)
    a = np.stack([rng.integers(0, 10, n), rng.integers(-3, 3, n)]).astype(np.int32)
    ot = O.Table(O.F32, x, a)
    q = rng.standard_normal((2, d)).astype(np.float32)
    pred = [(0, 2, 7), (1, -1, 2)]
    sel = set(O.select(ot, pred))
    allr = O.scan_range(ot, q, [], 18.0, n, O.L2SQ)
    filt = O.scan_range(ot, q, pred, 18.0, n, O.L2SQ)
    for b in range(2):
        want = sorted(set(allr[0][b][:allr[3][b]]) & sel)
        assert list(filt[0][b][:filt[3][b]]) == want
