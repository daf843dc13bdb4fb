"""Pins of the oracle's partition index and its filtered probe (the
probe-based access path of Section 4; pre-filtering of Section 4.1).

The index is k-means over the stored vectors (Lloyd's iteration: exact
nearest-centroid assignment, centroid = mean of its partition).  Pinned by
brute-force argmin, correctly rounded means (math.fsum), the monotone k-means
objective and the list layout; the probe by its closed forms: probing every
partition is the exact scan, the candidates nest as more partitions are
visited (so recall cannot fall), and the stopping rules."""

import math

import numpy as np
import pytest

import oracle as O


@pytest.fixture(scope="module")
def data():
    rng = np.random.default_rng(21)
    n, d = 3000, 12
    centres = rng.standard_normal((12, d)) * 3
    x = (centres[rng.integers(0, 12, n)] + rng.standard_normal((n, d))).astype(np.float32)
    a = rng.integers(0, 20, (1, n)).astype(np.int32)
    return x, a, O.Table(O.F32, x, a)


def _sse(x, cent, assign):
    return float(sum(((x[i].astype(np.float64) - cent[assign[i]]) ** 2).sum() for i in range(x.shape[0])))


def test_index_assignment_means_and_lists(data):
    x, a, t = data
    nlist = 24
    cent, assign, off, ids = O.ivf_build(t, nlist, 4)
    d2 = ((x[:, None, :].astype(np.float64) - cent[None, :, :].astype(np.float64)) ** 2).sum(-1)
    best = d2.argmin(1)
    srt = np.sort(d2, axis=1)
    clear = (srt[:, 1] - srt[:, 0]) > 1e-9 * srt[:, 1]
    assert np.array_equal(assign[clear], best[clear])
    # the lists: every row once, partitions ascending, offsets = counts
    assert np.array_equal(np.sort(ids), np.arange(x.shape[0]))
    assert np.array_equal(np.diff(off), np.bincount(assign, minlength=nlist))
    for c in range(nlist):
        m = ids[off[c]:off[c + 1]]
        assert np.all(np.diff(m) > 0) and np.all(assign[m] == c)


def test_centroids_are_partition_means(data):
    x, a, t = data
    cent0 = x[[(i * x.shape[0]) // 10 for i in range(10)]]
    assign = O._nearest_centroid(x, cent0)
    cent = O._centroid_means(x, assign, cent0)
    for c in range(10):
        m = np.nonzero(assign == c)[0]
        for j in range(x.shape[1]):
            want = np.float32(math.fsum(float(v) for v in x[m, j]) / m.size)
            assert abs(cent[c, j] - want) <= np.spacing(np.abs(want))


def test_kmeans_objective_does_not_increase(data):
    x, a, t = data
    prev = np.inf
    for iters in range(0, 5):
        cent, assign, _, _ = O.ivf_build(t, 16, iters)
        s = _sse(x, cent, assign)
        assert s <= prev * (1 + 1e-12)
        prev = s


def test_probing_every_partition_is_the_scan(data):
    x, a, t = data
    cent, assign, off, ids = O.ivf_build(t, 16, 3)
    q = x[[5, 700, 2999]] + np.float32(0.25)
    for pred in ([], [(0, 3, 9)]):
        got = O.ivf_probe(t, cent, off, ids, q, pred, 10, O.L2SQ, 16, 1, x.shape[0])
        ref = O.scan_topk(t, q, pred, 10, O.L2SQ)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        assert (got[2] == 16).all()


def test_probe_candidates_nest_and_stopping_rules(data):
    x, a, t = data
    cent, assign, off, ids = O.ivf_build(t, 16, 3)
    q = x[[11, 1500]] - np.float32(0.5)
    pred = [(0, 0, 5)]
    exact = O.scan_topk(t, q, pred, 10, O.L2SQ)[0]
    prev_rec = -1.0
    for nprobe in (1, 2, 4, 8, 16):
        got = O.ivf_probe(t, cent, off, ids, q, pred, 10, O.L2SQ, nprobe, 1, x.shape[0])
        assert (got[2] == nprobe).all()
        rec = np.mean([len(set(got[0][b]) & set(exact[b])) / 10 for b in range(2)])
        assert rec >= prev_rec
        prev_rec = rec
    assert prev_rec == 1.0
    # past nprobe the walk goes on only while fewer than min_cand rows
    # qualified: a selective predicate makes it visit more partitions
    sel = [(0, 0, 1)]
    few = O.ivf_probe(t, cent, off, ids, q, sel, 10, O.L2SQ, 1, 1, x.shape[0])
    more = O.ivf_probe(t, cent, off, ids, q, sel, 10, O.L2SQ, 1, 60, x.shape[0])
    assert (few[2] == 1).all() and (more[2] > 1).all() and (more[3] >= 60).all()
    # cap_c: a partition that would take the visited rows past the cap is not
    # visited (the first one always is)
    got = O.ivf_probe(t, cent, off, ids, q, pred, 10, O.L2SQ, 16, 1, 1)
    assert (got[2] == 1).all()
