"""Pins for the FP64 oracle: checks against facts that do not come from the
oracle itself (closed forms, exact integer arithmetic, library codecs and
distances, brute force on tiny inputs, invariants, a hand-worked example).

Each test is chosen so that a plausible slip in ``oracle/oracle.c`` -- a
dropped term, a wrong sign, an inclusive/exclusive bound, a swapped tie-break,
a transposed operand -- fails at least one of them.
"""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import torch
from scipy.spatial.distance import cdist

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
I32_MIN, I32_MAX = -(2 ** 31), 2 ** 31 - 1


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


# ------------------------------------------------------------------ codecs
def test_bf16_decode_exhaustive_vs_torch():
    codes = np.arange(65536, dtype=np.uint16)
    mine = O.bf16_values(codes)
    ref = torch.from_numpy(codes.view(np.int16).copy()).view(torch.bfloat16).double().numpy()
    nan = np.isnan(ref)
    assert np.array_equal(nan, np.isnan(mine))
    assert np.array_equal(mine[~nan], ref[~nan])


def test_e4m3_decode_exhaustive_vs_torch_and_ocp_points():
    codes = np.arange(256, dtype=np.uint8)
    mine = O.e4m3_values(codes)
    ref = torch.from_numpy(codes.copy()).view(torch.float8_e4m3fn).double().numpy()
    nan = np.isnan(ref)
    assert np.array_equal(nan, np.isnan(mine))
    assert nan.sum() == 2 and nan[0x7F] and nan[0xFF]
    assert np.array_equal(mine[~nan], ref[~nan])
    # OCP e4m3fn landmarks: max normal 448, min normal 2^-6, min subnormal 2^-9
    assert mine[0x7E] == 448.0 and mine[0x08] == 2.0 ** -6 and mine[0x01] == 2.0 ** -9
    assert mine[0x38] == 1.0 and mine[0x80] == 0.0 and math.copysign(1, mine[0x80]) < 0
    assert np.all(np.diff(mine[:0x7F]) > 0)


def _bf16_probe_values(rng):
    # random patterns, exact ties (low half 0x8000), just-below/above ties,
    # subnormals, extremes around the overflow threshold
    pats = rng.integers(0, 2 ** 32, size=20000, dtype=np.uint64).astype(np.uint32)
    pats = pats[(pats & 0x7F800000) != 0x7F800000]
    hi = pats & 0xFFFF0000
    extra = np.concatenate([hi | 0x8000, hi | 0x7FFF, hi | 0x8001, hi])
    edge = np.array([0x7F7F0000, 0x7F7F7FFF, 0x7F7F8000, 0x7F7FFFFF, 0x00000001, 0x00008000,
                     0x00018000, 0x80008000, 0x80000000, 0x00000000, 0x3F808000, 0x3F818000],
                    dtype=np.uint32)
    allp = np.concatenate([pats, extra.astype(np.uint32), edge])
    return allp.view(np.float32)


def test_bf16_encode_rne_vs_torch():
    x = _bf16_probe_values(np.random.default_rng(7))
    mine, overflow = O.encode_bf16(x)
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(mine, ref)
    # 0x7F7F8000 (midpoint above max, max is odd) and 0x7F7FFFFF overflow
    assert overflow == int(np.sum(np.isinf(torch.from_numpy(x).to(torch.bfloat16).float().numpy())))
    assert overflow >= 2


def test_e4m3_encode_rne_vs_torch_in_range_and_saturation():
    vals = O.e4m3_values(np.arange(0x7F, dtype=np.uint8))  # 0 .. 448 ascending
    mids = (vals[:-1] + vals[1:]) / 2.0                     # exact ties
    rng = np.random.default_rng(11)
    rand = rng.uniform(-448, 448, 20000)
    small = rng.uniform(-2 ** -5, 2 ** -5, 5000)
    probe = np.concatenate([vals, -vals, mids, -mids, np.nextafter(mids, 0), np.nextafter(mids, 1e9),
                            rand, small]).astype(np.float32).astype(np.float64)
    mine = O.e4m3_encode(probe)
    ref = torch.from_numpy(probe.astype(np.float32)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    # torch keeps the sign of zero results the same way (sign of the input)
    assert np.array_equal(mine, ref)
    # ties go to the even code: between codes c and c+1 the even one wins
    tie_codes = O.e4m3_encode(mids)
    assert np.all(tie_codes % 2 == 0)
    # saturation (torch's cast gives NaN there, the quantiser clamps to +-448)
    sat = O.e4m3_encode([448.0, 449.0, 464.0, 1e6, -1e30, -448.5])
    assert list(sat) == [0x7E, 0x7E, 0x7E, 0x7E, 0xFE, 0xFE]


def test_fp8_row_scale_definition():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((50, 33)).astype(np.float32)
    x[7] = 0.0
    codes, scale = O.encode_fp8_rows(x)
    amax = np.abs(x).max(axis=1)
    expect = np.where(amax == 0, np.float32(1), (amax / np.float32(448)).astype(np.float32))
    assert np.array_equal(scale, expect)
    dec = O.e4m3_values(codes.ravel()).reshape(codes.shape) * scale[:, None].astype(np.float64)
    # every stored value is within half an e4m3 step (relative 2^-4) of the input,
    # or within the subnormal spacing 2^-10 * scale
    err = np.abs(dec - x)
    bound = np.maximum(np.abs(x) * 2.0 ** -4, 2.0 ** -10 * scale[:, None])
    assert np.all(err <= bound * (1 + 1e-12))
    # the largest element of each non-zero row decodes to (about) 448 * scale
    i = np.argmax(np.abs(x), axis=1)
    top = np.abs(O.e4m3_values(codes[np.arange(50), i]))
    assert np.all(np.delete(top, 7) == 448.0) and np.all(codes[7] == 0)


def test_normalize_rows_vs_numpy_norm():
    rng = np.random.default_rng(5)
    x = (rng.standard_normal((300, 77)) * rng.uniform(0.01, 100, (300, 1))).astype(np.float32)
    x[4] = 0
    mine = O.normalize_rows(x)
    x64 = x.astype(np.float64)
    nrm = np.linalg.norm(x64, axis=1, keepdims=True)
    ref = np.where(nrm == 0, x64, x64 / np.where(nrm == 0, 1, nrm)).astype(np.float32)
    ulps = np.abs(mine.view(np.int32).astype(np.int64) - ref.view(np.int32).astype(np.int64))
    assert ulps.max() <= 1 and (ulps == 0).mean() > 0.999
    n_out = np.linalg.norm(mine.astype(np.float64), axis=1)
    assert np.all(np.abs(n_out[np.arange(300) != 4] - 1) < 80 * 2.0 ** -24)
    assert np.array_equal(mine[4], x[4])


# --------------------------------------------------------------- predicate
def test_select_brute_force_and_bounds():
    rng = np.random.default_rng(1)
    n = 3000
    a0 = rng.integers(-5, 6, n).astype(np.int32)
    a1 = rng.integers(I32_MIN, I32_MAX, n, dtype=np.int64).astype(np.int32)
    a1[:4] = [I32_MIN, I32_MAX, 0, -1]
    attr = np.stack([a0, a1])
    T = O.Table(O.F32, np.zeros((n, 1), np.float32), attr)
    cases = [
        [], [(0, 0, 1)], [(0, -5, 6)], [(0, 3, 3)], [(0, 6, -6)], [(0, -2, 2), (1, 0, 2 ** 40)],
        [(1, I32_MIN, I32_MIN + 1)], [(1, I32_MAX, I32_MAX + 1)], [(1, I32_MIN, I32_MAX)],
        [(1, -2 ** 62, 2 ** 62)], [(0, 1, 4), (0, 2, 9), (1, -1, 1)],
    ]
    for pred in cases:
        got = O.select(T, pred)
        want = [i for i in range(n) if all(lo <= int(attr[c][i]) < hi for c, lo, hi in pred)]
        assert got.tolist() == want, pred
    assert O.select(T, [(1, I32_MAX, I32_MAX + 1)]).tolist() == [1]
    assert O.select(T, [(1, I32_MIN, I32_MAX)]).size == n - int(np.sum(a1 == I32_MAX))


# ---------------------------------------------------------------- distance
def test_distance_exact_on_integer_vectors():
    rng = np.random.default_rng(2)
    n, d = 40, 29
    x = rng.integers(-50, 51, (n, d)).astype(np.float32)
    q = rng.integers(-50, 51, d).astype(np.float32)
    T = O.Table(O.F32, x, np.zeros(n, np.int32))
    ids = np.arange(n)
    l2 = O.distances(T, q, ids, O.L2SQ)
    ip = O.distances(T, q, ids, O.IP)
    xi, qi = x.astype(np.int64), q.astype(np.int64)
    assert l2.tolist() == [float(sum((int(a) - int(b)) ** 2 for a, b in zip(qi, r))) for r in xi]
    assert ip.tolist() == [float(-sum(int(a) * int(b) for a, b in zip(qi, r))) for r in xi]


def test_distance_closed_forms_basis_vectors():
    d = 16
    E = np.eye(d, dtype=np.float32)
    T = O.Table(O.F32, E, np.zeros(d, np.int32))
    for i in (0, 5, d - 1):
        l2 = O.distances(T, E[i], np.arange(d), O.L2SQ)
        ip = O.distances(T, E[i], np.arange(d), O.IP)
        assert l2[i] == 0.0 and np.all(np.delete(l2, i) == 2.0)
        assert ip[i] == -1.0 and np.all(np.delete(ip, i) == 0.0)
        assert not np.any(np.signbit(np.delete(ip, i)))  # zero stored as +0.0


def test_distance_vs_longdouble_and_scipy():
    rng = np.random.default_rng(4)
    n, d = 200, 128
    x = rng.standard_normal((n, d)).astype(np.float32)
    q = rng.standard_normal(d).astype(np.float32)
    T = O.Table(O.F32, x, np.zeros(n, np.int32))
    l2 = O.distances(T, q, np.arange(n), O.L2SQ)
    ip = O.distances(T, q, np.arange(n), O.IP)
    xl, ql = x.astype(np.longdouble), q.astype(np.longdouble)
    l2_ref = ((xl - ql) ** 2).sum(axis=1)
    ip_ref = -(xl * ql).sum(axis=1)
    absip = np.abs(xl * ql).sum(axis=1)
    assert np.all(np.abs(l2 - l2_ref) <= (d + 2) * 2.0 ** -53 * l2_ref)
    assert np.all(np.abs(ip - ip_ref) <= (d + 2) * 2.0 ** -53 * absip)
    sq = cdist(q[None].astype(np.float64), x.astype(np.float64), "sqeuclidean")[0]
    assert np.allclose(l2, sq, rtol=1e-12, atol=0)


def test_distance_on_quantised_storage_matches_decoded_values():
    rng = np.random.default_rng(6)
    n, d = 64, 96
    x = rng.standard_normal((n, d)).astype(np.float32)
    q = rng.standard_normal(d).astype(np.float32)
    attr = np.zeros(n, np.int32)
    Tb = O.Table.build(x, attr, O.BF16)
    Tf = O.Table.build(x, attr, O.FP8)
    xb = torch.from_numpy(x).to(torch.bfloat16).double().numpy()          # library codec
    cf = torch.from_numpy(Tf.rows.copy()).view(torch.float8_e4m3fn).double().numpy()
    xf = cf * Tf.scale[:, None].astype(np.float64)
    for T, xs, codes, s in ((Tb, xb, xb, np.ones(n)), (Tf, xf, cf, Tf.scale.astype(np.float64))):
        ql = q.astype(np.longdouble)
        ip = O.distances(T, q, np.arange(n), O.IP)
        ref = -(np.asarray(codes, np.longdouble) * ql).sum(axis=1) * s
        assert np.allclose(ip, ref.astype(np.float64), rtol=1e-13, atol=1e-13)
        l2 = O.distances(T, q, np.arange(n), O.L2SQ)
        ref2 = ((np.asarray(xs, np.longdouble) - ql) ** 2).sum(axis=1)
        assert np.allclose(l2, ref2.astype(np.float64), rtol=1e-13, atol=0)


# ------------------------------------------------------------------- top-k
def _exact_rank(x_int, q_int, ids, metric):
    """Exact integer distances ranked by (distance, id) with Python ints."""
    out = []
    for i in ids:
        r = [int(v) for v in x_int[i]]
        if metric == O.L2SQ:
            dv = sum((int(a) - b) ** 2 for a, b in zip(q_int, r))
        else:
            dv = -sum(int(a) * b for a, b in zip(q_int, r))
        out.append((dv, int(i)))
    return sorted(out)


@pytest.mark.parametrize("metric", [O.L2SQ, O.IP])
def test_topk_exact_with_many_ties_integer_data(metric):
    rng = np.random.default_rng(8)
    n, d = 500, 6
    x = rng.integers(-2, 3, (n, d)).astype(np.float32)   # lots of exact ties
    attr = np.stack([rng.integers(0, 10, n), rng.integers(0, 3, n)]).astype(np.int32)
    T = O.Table(O.F32, x, attr)
    q = rng.integers(-2, 3, (5, d)).astype(np.float32)
    pred = [(0, 2, 8), (1, 0, 2)]
    for k in (1, 7, 64, 400):
        idx, dist, dist64, nv = O.scan_topk(T, q, pred, k, metric, nthreads=3)
        sel = [i for i in range(n) if 2 <= attr[0, i] < 8 and 0 <= attr[1, i] < 2]
        for b in range(5):
            want = _exact_rank(x, q[b].astype(np.int64).tolist(), sel, metric)[:k]
            m = len(want)
            assert nv[b] == m
            assert idx[b, :m].tolist() == [i for _, i in want]
            assert dist64[b, :m].tolist() == [float(v) for v, _ in want]
            assert np.all(idx[b, m:] == -1) and np.all(np.isinf(dist[b, m:]))


def test_topk_brute_force_lexsort_continuous():
    rng = np.random.default_rng(9)
    n, d = 64, 8
    x = rng.standard_normal((n, d)).astype(np.float32)
    attr = rng.integers(0, 4, n).astype(np.int32)
    q = rng.standard_normal((4, d)).astype(np.float32)
    T = O.Table(O.F32, x, attr)
    for metric in (O.L2SQ, O.IP):
        idx, dist, dist64, _ = O.scan_topk(T, q, [(0, 1, 3)], 10, metric)
        sel = np.nonzero((attr >= 1) & (attr < 3))[0]
        xl = x[sel].astype(np.longdouble)
        for b in range(4):
            ql = q[b].astype(np.longdouble)
            dv = ((xl - ql) ** 2).sum(1) if metric == O.L2SQ else -(xl * ql).sum(1)
            order = np.lexsort((sel, dv.astype(np.float64)))
            assert idx[b].tolist() == sel[order][:10].tolist()
            assert np.array_equal(dist[b], dv[order][:10].astype(np.float64).astype(np.float32))


def test_topk_invariants_and_planted_queries():
    rng = np.random.default_rng(10)
    n, d = 2000, 24
    x = rng.standard_normal((n, d)).astype(np.float32)
    attr = rng.integers(0, 100, n).astype(np.int32)
    T = O.Table(O.F32, x, attr)
    pred = [(0, 0, 30)]
    sel = set(np.nonzero(attr < 30)[0].tolist())
    inside = sorted(sel)[17]
    outside = int(np.nonzero(attr >= 30)[0][3])
    dup = sorted(sel)[40]
    x2 = x.copy()
    x2[dup] = x2[inside]                      # planted duplicate -> tie at distance 0
    T2 = O.Table(O.F32, x2, attr)
    q = np.stack([x2[inside], x2[outside]])
    idx, dist, _, nv = O.scan_topk(T2, q, pred, 50, O.L2SQ)
    lo, hi = sorted((inside, dup))
    assert idx[0, 0] == lo and idx[0, 1] == hi and dist[0, 0] == 0 and dist[0, 1] == 0
    assert outside not in idx[1].tolist() and dist[1, 0] > 0
    for b in range(2):
        assert set(idx[b].tolist()) <= sel
        assert np.all(np.diff(dist[b].astype(np.float64)) >= 0)
    # the unfiltered scan does find the planted non-qualifying row first
    idx_all, dist_all, _, _ = O.scan_topk(T2, q[1:], [], 5, O.L2SQ)
    assert idx_all[0, 0] == outside and dist_all[0, 0] == 0


def test_pushdown_equivalence_eq3():
    """sigma_eps(v x sigma_theta(R)): ranking the materialised selection
    without a predicate gives the filtered scan (ids mapped back)."""
    rng = np.random.default_rng(12)
    n, d = 3000, 40
    x = rng.standard_normal((n, d)).astype(np.float32)
    attr = rng.integers(0, 1000, (2, n)).astype(np.int32)
    q = rng.standard_normal((6, d)).astype(np.float32)
    pred = [(0, 100, 600), (1, 0, 500)]
    T = O.Table(O.F32, x, attr)
    sel = O.select(T, pred)
    Ts = O.Table(O.F32, x[sel], np.zeros(sel.size, np.int32))
    for metric in (O.L2SQ, O.IP):
        a_idx, a_d, _, _ = O.scan_topk(T, q, pred, 33, metric)
        b_idx, b_d, _, _ = O.scan_topk(Ts, q, [], 33, metric)
        assert np.array_equal(a_idx, sel[b_idx])
        assert np.array_equal(a_d, b_d)


def test_ip_on_normalised_table_is_cosine_ranking():
    rng = np.random.default_rng(13)
    n, d = 500, 64
    x = (rng.standard_normal((n, d)) * rng.uniform(0.1, 10, (n, 1))).astype(np.float32)
    q = rng.standard_normal((3, d)).astype(np.float32)
    T = O.Table.build(x, np.zeros(n, np.int32), O.F32, normalize=True)
    idx, _, _, _ = O.scan_topk(T, q, [], 20, O.IP)
    cos_d = cdist(q.astype(np.float64), x.astype(np.float64), "cosine")
    for b in range(3):
        assert idx[b].tolist() == np.argsort(cos_d[b], kind="stable")[:20].tolist()


def test_per_query_predicates_and_k_equal_single_calls():
    rng = np.random.default_rng(14)
    n, d = 1500, 16
    x = rng.standard_normal((n, d)).astype(np.float32)
    attr = rng.integers(0, 50, (2, n)).astype(np.int32)
    T = O.Table(O.F32, x, attr)
    q = rng.standard_normal((4, d)).astype(np.float32)
    preds = [[(0, 0, 10)], [], [(0, 5, 45), (1, 3, 4)], [(1, 60, 70)]]
    ks = [3, 12, 100, 5]
    idx, dist, _, nv = O.scan_topk(T, q, preds, ks, O.L2SQ)
    for b in range(4):
        i1, d1, _, n1 = O.scan_topk(T, q[b], preds[b], ks[b], O.L2SQ)
        assert nv[b] == n1[0]
        assert np.array_equal(idx[b, :ks[b]], i1[0]) and np.array_equal(dist[b, :ks[b]], d1[0])
        assert np.all(idx[b, ks[b]:] == -1)
    assert nv[3] == 0 and np.all(idx[3] == -1)


def test_hand_worked_golden_example():
    with open(os.path.join(HERE, "golden", "hand_example.json")) as f:
        g = json.load(f)
    x = np.array(g["rows"], np.float32)
    T = O.Table(O.F32, x, np.array(g["attr"], np.int32))
    p = g["predicate"]
    pred = [(p["col"], p["lo"], p["hi"])]
    assert O.select(T, pred).tolist() == g["qualifying_ids"]
    for name, metric in (("L2SQ", O.L2SQ), ("IP", O.IP)):
        e = g["expected"][name]
        idx, dist, _, nv = O.scan_topk(T, np.array(g["query"], np.float32), pred, e["k"], metric)
        assert idx[0].tolist() == e["ids"]
        assert dist[0].tolist() == [float(v) for v in e["dist"]]
        assert nv[0] == e["nvalid"]
        assert not np.any(np.signbit(dist[0][dist[0] == 0]))


def test_k_larger_than_table_and_empty_selection():
    x = np.arange(12, dtype=np.float32).reshape(4, 3)
    T = O.Table(O.F32, x, np.array([1, 2, 3, 4], np.int32))
    idx, dist, _, nv = O.scan_topk(T, np.zeros(3, np.float32), [], 9, O.L2SQ)
    assert idx[0].tolist() == [0, 1, 2, 3, -1, -1, -1, -1, -1] and nv[0] == 4
    idx, dist, _, nv = O.scan_topk(T, np.zeros(3, np.float32), [(0, 5, 9)], 2, O.L2SQ)
    assert idx[0].tolist() == [-1, -1] and nv[0] == 0 and np.all(np.isinf(dist))


def test_fraction_exactness_of_fp8_ip_distance():
    """FP8 IP distance = -(scale * sum q_j c_j); with dyadic inputs the FP64
    result equals the exact rational value."""
    rng = np.random.default_rng(15)
    n, d = 20, 12
    x = (rng.integers(-64, 65, (n, d)) / 8.0).astype(np.float32)
    q = (rng.integers(-64, 65, d) / 16.0).astype(np.float32)
    T = O.Table.build(x, np.zeros(n, np.int32), O.FP8)
    got = O.distances(T, q, np.arange(n), O.IP)
    codes = O.e4m3_values(T.rows.ravel()).reshape(n, d)
    for i in range(n):
        exact = -Fraction(float(T.scale[i])) * sum(Fraction(float(a)) * Fraction(float(c))
                                                    for a, c in zip(q, codes[i]))
        assert got[i] == float(exact)


# ------------------------------------------------- summation order, pinned
# The oracle's FP64 distance is one chain over the coordinates in ascending
# order, one fused multiply-add each.  Emulated here with exact rationals
# (Python's int division rounds correctly), independently of the C code, on
# rows whose exact distances tie and whose FP64 sums round differently with
# the order of the terms.  The same rows ranked by a blockwise butterfly sum
# (per 16-byte block a chain, then a 64-lane xor butterfly of plain adds)
# come out in a different order, so the GPU test on these inputs detects a
# rerank that does not follow the definition's order.
def _emu_values(ot, i):
    if ot.dtype == O.F32:
        return [float(v) for v in ot.rows[i]], 1.0
    if ot.dtype == O.BF16:
        return [float(v) for v in O.bf16_values(ot.rows[i])], 1.0
    return [float(v) for v in O.e4m3_values(ot.rows[i])], float(ot.scale[i])


def _emu_fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _emu_chain(q, xs, sc, l2, js):
    acc = 0.0
    for j in js:
        if l2:
            t = float(q[j]) - sc * xs[j]
            acc = _emu_fma(t, t, acc)
        else:
            acc = _emu_fma(float(q[j]), xs[j], acc)
    return acc


def _emu_finish(acc, sc, l2):
    return (acc if l2 else -(sc * acc)) + 0.0


@pytest.mark.parametrize("dtype,metric", [(O.F32, O.L2SQ), (O.F32, O.IP), (O.BF16, O.IP), (O.FP8, O.IP)])
@pytest.mark.parametrize("B,seed", [(1, 13), (16, 27)])
def test_distance_is_the_ascending_fma_chain_on_tied_rows(dtype, metric, B, seed):
    import planted
    x, a, q, pos = planted.planted(metric == O.L2SQ, B, seed)
    ot = O.Table.build(x, a, dtype)
    V = {O.F32: 4, O.BF16: 8, O.FP8: 16}[dtype]
    l2 = metric == O.L2SQ
    differs = 0
    for b in range(min(B, 3)):
        seq, bfly = [], []
        for p in pos:
            xs, sc = _emu_values(ot, p)
            seq.append(_emu_finish(_emu_chain(q[b], xs, sc, l2, range(len(xs))), sc, l2))
            part = [_emu_chain(q[b], xs, sc, l2, range(c * V, (c + 1) * V)) for c in range(len(xs) // V)]
            part += [0.0] * (64 - len(part))
            m = 32
            while m:
                part = [part[l_] + part[l_ ^ m] for l_ in range(64)]
                m //= 2
            bfly.append(_emu_finish(part[0], sc, l2))
        seq = np.array(seq)
        assert np.array_equal(O.distances(ot, q[b], pos, metric), seq)
        top_seq = np.lexsort((pos, seq))[:100]
        top_bfly = np.lexsort((pos, np.array(bfly)))[:100]
        differs += not np.array_equal(top_seq, top_bfly)
    assert differs > 0
