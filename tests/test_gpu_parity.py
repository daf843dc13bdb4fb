"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.  Ids must match exactly; distances within 1e-5 relative
(the returned float is the FP64 distance rounded, so it is in fact expected
to match bit for bit, which is checked too)."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2403_15807_amd import inputs, vrs

pytestmark = pytest.mark.gpu

I32_MIN = -(2 ** 31)
RTOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _ready(oracle_lib):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return oracle_lib


def _check(res, ref, what=""):
    gi, gd = res.idx.cpu().numpy(), res.dist.cpu().numpy()
    ri, rd = ref[0], ref[1]
    assert gi.shape == ri.shape, what
    bad = np.nonzero((gi != ri).any(axis=1))[0]
    assert bad.size == 0, f"{what}: id mismatch in queries {bad[:8]}: gpu {gi[bad[0]][:12]} oracle {ri[bad[0]][:12]}"
    fin = np.isfinite(rd)
    assert np.array_equal(np.isfinite(gd), fin), what
    rel = np.abs(gd[fin].astype(np.float64) - rd[fin]) / np.maximum(np.abs(rd[fin]), 1e-30)
    assert (rel <= RTOL).all() or rd[fin].size == 0, f"{what}: max rel {rel.max()}"
    zero = rd[fin] == 0
    assert np.all(gd[fin][zero] == 0)
    assert np.array_equal(gd, rd), f"{what}: distances not bit-identical"
    nv = res.n_valid.cpu().numpy()
    assert np.array_equal(nv, ref[3]), what


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# ------------------------------------------------------------------ build
@pytest.mark.parametrize("store", [vrs.F32, vrs.BF16, vrs.FP8E4M3])
@pytest.mark.parametrize("normalize", [False, True])
def test_build_table_bit_exact(store, normalize):
    rng = np.random.default_rng(1)
    n, d = 3001, 100
    x = (rng.standard_normal((n, d)) * rng.uniform(0.01, 30, (n, 1))).astype(np.float32)
    x[5] = 0.0
    x[6, :7] = [1e-30, -1e-30, 3e-39, -0.0, 448.0, 1e-8, -5e-9]
    a = rng.integers(0, 10, (1, n)).astype(np.int32)
    T = vrs.Table(_dev(x), _dev(a), store=store, normalize=normalize)
    rows, scale = T.export()
    torch.cuda.synchronize()
    ot = O.Table.build(x, a, {vrs.F32: O.F32, vrs.BF16: O.BF16, vrs.FP8E4M3: O.FP8}[store], normalize)
    got = rows.cpu().numpy()
    if store == vrs.F32:
        assert np.array_equal(got.view(np.uint32), ot.rows.view(np.uint32))
    elif store == vrs.BF16:
        assert np.array_equal(got.view(np.uint16), ot.rows)
    else:
        assert np.array_equal(got, ot.rows)
        assert np.array_equal(scale.cpu().numpy().view(np.uint32), ot.scale.view(np.uint32))
    T.close()


def test_build_rejects_nonfinite():
    x = np.ones((100, 8), np.float32)
    x[3, 2] = np.nan
    with pytest.raises(vrs.VrsError) as e:
        vrs.Table(_dev(x), None)
    assert e.value.status == vrs.VRS_E_NONFINITE
    x[3, 2] = 3.4e38  # finite in float32, rounds past the largest bfloat16
    vrs.Table(_dev(x), None).close()
    with pytest.raises(vrs.VrsError) as e:
        vrs.Table(_dev(x), None, store=vrs.BF16)
    assert e.value.status == vrs.VRS_E_NONFINITE


# -------------------------------------------------------------- predicate
def test_select_matches_oracle():
    rng = np.random.default_rng(2)
    n = 70001  # several selection blocks and a ragged tail
    a = np.stack([rng.integers(0, 100, n), rng.integers(-5, 5, n)]).astype(np.int32)
    a[1, :3] = [I32_MIN, 2 ** 31 - 1, 0]
    T = vrs.Table(_dev(np.zeros((n, 4), np.float32)), _dev(a))
    ot = O.Table(O.F32, np.zeros((n, 4), np.float32), a)
    for pred in ([], [(0, 0, 10)], [(0, 10, 10)], [(0, 50, 40)], [(1, I32_MIN, I32_MIN + 1)],
                 [(1, 2 ** 31 - 1, 2 ** 40)], [(0, -2 ** 40, 2 ** 40), (1, 0, 3)],
                 [(0, 3, 97), (1, -4, 4), (0, 5, 90)]):
        got = T.select(pred).cpu().numpy()
        assert np.array_equal(got, O.select(ot, pred)), pred


# ------------------------------------------------------------------ scans
def _config0(n=100_000, d=128, C=100, B=16, seed_cfg=0):
    x = inputs.table(seed_cfg, n, d, C)
    a = inputs.attributes(seed_cfg, n, 1, 100)
    q = inputs.queries(seed_cfg, B, d, C)
    return x, a, q


@pytest.fixture(scope="module")
def cfg0():
    x, a, q = _config0()
    T = vrs.Table(_dev(x), _dev(a))
    ot = O.Table(O.F32, x, a)
    pred = [(0, I32_MIN, 10)]
    ref = O.scan_topk(ot, q, pred, 10, O.L2SQ)
    return x, a, q, T, ot, pred, ref


@pytest.mark.parametrize("strategy", [vrs.STRATEGY_AUTO, vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER])
@pytest.mark.parametrize("tile", list(range(-1, 8)))
def test_config0_l2_top10(cfg0, strategy, tile):
    x, a, q, T, ot, pred, ref = cfg0
    r = T.scan_topk(_dev(q), pred, 10, vrs.L2SQ, strategy=strategy, tile=tile)
    torch.cuda.synchronize()
    _check(r, ref, f"strategy {strategy} tile {tile}")


def test_config0_deterministic_and_strategy_invariant(cfg0):
    x, a, q, T, ot, pred, ref = cfg0
    outs = []
    for strategy in (vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER, vrs.STRATEGY_MASK):
        r = T.scan_topk(_dev(q), pred, 10, vrs.L2SQ, strategy=strategy)
        outs.append((r.idx.cpu().numpy(), r.dist.cpu().numpy().view(np.uint32)))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


def test_query_alone_equals_query_in_batch(cfg0):
    x, a, q, T, ot, pred, ref = cfg0
    full = T.scan_topk(_dev(q), pred, 10, vrs.L2SQ)
    for b in (0, 7, 15):
        one = T.scan_topk(_dev(q[b:b + 1]), pred, 10, vrs.L2SQ)
        assert torch.equal(one.idx[0], full.idx[b]) and torch.equal(one.dist[0], full.dist[b])


@pytest.mark.parametrize("metric", [vrs.L2SQ, vrs.IP])
@pytest.mark.parametrize("k", [1, 100, 256])
def test_ragged_shapes_and_k(metric, k):
    rng = np.random.default_rng(3)
    n, d, B = 33333, 100, 5  # d pads to 128, n is ragged for every tile
    x = inputs.table(1, n, d, 50)
    a = inputs.attributes(1, n, 2, 1000)
    q = inputs.queries(1, B, d, 50)
    T = vrs.Table(_dev(x), _dev(a), normalize=(metric == vrs.IP))
    ot = O.Table.build(x, a, O.F32, normalize=(metric == vrs.IP))
    pred = [(0, 100, 900), (1, 0, 700)]
    ref = O.scan_topk(ot, q, pred, k, metric)
    for strategy in (vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER):
        r = T.scan_topk(_dev(q), pred, k, metric, strategy=strategy)
        _check(r, ref, f"metric {metric} k {k} strategy {strategy}")


@pytest.mark.parametrize("B", [8, 70, 130])
@pytest.mark.parametrize("metric", [vrs.L2SQ, vrs.IP])
def test_mfma_query_tiles(B, metric):
    # several 64-query tiles with a ragged last tile, ragged row count
    n, d = 50001, 128
    x = inputs.table(4, n, d, 200)
    a = inputs.attributes(4, n, 2, 1000)
    q = inputs.queries(4, B, d, 200)
    T = vrs.Table(_dev(x), _dev(a), normalize=(metric == vrs.IP))
    ot = O.Table.build(x, a, O.F32, normalize=(metric == vrs.IP))
    pred = [(0, 0, 600), (1, 100, 1000)]
    for k in (1, 10, 100):
        ref = O.scan_topk(ot, q, pred, k, metric)
        for strategy in (vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER):
            for tile in (4, 5, 6, 7):
                r = T.scan_topk(_dev(q), pred, k, metric, strategy=strategy, tile=tile)
                _check(r, ref, f"B {B} metric {metric} k {k} strategy {strategy} tile {tile}")


@pytest.mark.parametrize("d", [384, 768, 1536])
@pytest.mark.parametrize("B", [5, 16, 70])
def test_mfma_f32_wide_rows_in_coordinate_chunks(d, B):
    # float32 rows wider than 256 coordinates: the FP32 MFMA screen takes
    # them 128 coordinates at a time (B <= 16: the small-batch form)
    n = 12001
    x = inputs.table(13, n, d, 100)
    a = inputs.attributes(13, n, 1, 1000)
    q = inputs.queries(13, B, d, 100)
    for metric in (vrs.L2SQ, vrs.IP):
        T = vrs.Table(_dev(x), _dev(a), normalize=(metric == vrs.IP))
        ot = O.Table.build(x, a, O.F32, normalize=(metric == vrs.IP))
        pred = [(0, 0, 700)]
        for k in (1, 100):
            ref = O.scan_topk(ot, q, pred, k, metric)
            for strategy in (vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER):
                _, su, tu = T.plan(B, pred, k, metric, strategy=strategy, tile=4, chooser=vrs.CHOOSER_HEURISTIC)
                assert (su, tu) == (strategy, 4), "the FP32 MFMA tile must be available"
                r = T.scan_topk(_dev(q), pred, k, metric, strategy=strategy, tile=4)
                _check(r, ref, f"d {d} B {B} metric {metric} k {k} strategy {strategy}")


def test_fewer_qualifying_rows_than_k_and_empty():
    x, a, q = _config0(n=5000, B=3)
    T = vrs.Table(_dev(x), _dev(a))
    ot = O.Table(O.F32, x, a)
    for pred in ([(0, 7, 8)], [(0, 200, 300)], [(0, 0, 0)]):
        # attr==7 keeps ~50 rows < k=100
        ref = O.scan_topk(ot, q, pred, 100, O.L2SQ)
        for strategy in (vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER):
            r = T.scan_topk(_dev(q), pred, 100, vrs.L2SQ, strategy=strategy)
            _check(r, ref, f"pred {pred}")


def test_planted_duplicates_and_queries():
    x, a, q = _config0(n=20000, B=4)
    sel = np.nonzero(a[0] < 10)[0]
    outside = np.nonzero(a[0] >= 10)[0]
    x = x.copy()
    for j in range(1, 40):                 # 40 identical rows -> 40-way tie at distance 0
        x[sel[j * 3]] = x[sel[0]]
    q = q.copy()
    q[0] = x[sel[0]]
    q[1] = x[outside[5]]                    # planted in a non-qualifying row
    T = vrs.Table(_dev(x), _dev(a))
    ot = O.Table(O.F32, x, a)
    pred = [(0, 0, 10)]
    ref = O.scan_topk(ot, q, pred, 10, O.L2SQ)
    assert ref[1][0, 0] == 0 and ref[1][0, 9] == 0
    r = T.scan_topk(_dev(q), pred, 10, vrs.L2SQ)
    _check(r, ref, "planted")
    assert int(outside[5]) not in r.idx[1].tolist()


@pytest.mark.parametrize("store", [vrs.BF16, vrs.FP8E4M3, vrs.F32])
@pytest.mark.parametrize("d", [256, 200])
def test_ip_quantised_storage(store, d):
    # streaming (tile 3) and MFMA (tile 4) screening, ragged 64-query tiles
    n, B = 40000, 70
    x = inputs.table(2, n, d, 200)
    a = inputs.attributes(2, n, 2, 10 ** 6)
    q = inputs.queries(2, B, d, 200)
    T = vrs.Table(_dev(x), _dev(a), store=store, normalize=True)
    ot = O.Table.build(x, a, {vrs.F32: O.F32, vrs.BF16: O.BF16, vrs.FP8E4M3: O.FP8}[store], True)
    for sel in (0.3, 0.01):
        w = inputs.two_term_width(sel, 10 ** 6)
        pred = [(0, 0, w), (1, 0, w)]
        for k in (10, 100):
            ref = O.scan_topk(ot, q, pred, k, O.IP)
            for tile in (3, 4):
                for strategy in (vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER):
                    r = T.scan_topk(_dev(q), pred, k, vrs.IP, tile=tile, strategy=strategy)
                    _check(r, ref, f"store {store} d {d} sel {sel} k {k} tile {tile} strategy {strategy}")


def test_forced_certificate_failure_uses_exact_fallback():
    # k' = k and a 200-way exact tie around the k-th position: the screening
    # lists cannot certify, the FP64 fallback must produce the exact answer
    x, a, q = _config0(n=30000, B=4)
    x = x.copy()
    sel = np.nonzero(a[0] < 10)[0]
    for j in range(1, 200):
        x[sel[j * 7]] = x[sel[0]]
    q = q.copy()
    q[:2] = x[sel[0]] + np.float32(0.01)
    T = vrs.Table(_dev(x), _dev(a))
    ot = O.Table(O.F32, x, a)
    pred = [(0, 0, 10)]
    ref = O.scan_topk(ot, q, pred, 50, O.L2SQ)
    r = T.scan_topk(_dev(q), pred, 50, vrs.L2SQ, kprime_mult=1)
    _check(r, ref, "fallback")
    assert r.certified[:2].sum().item() == 0


def test_batched_per_query_predicates_and_k():
    n, d, B = 50000, 64, 37
    x = inputs.table(3, n, d, 100)
    a = inputs.attributes(3, n, 2, 10 ** 6)
    q = inputs.queries(3, B, d, 100)
    bp = inputs.batched_predicates(3, B, 10 ** 6, s_min=1e-3)
    preds = [[(0, int(bp.lo[b, 0]), int(bp.hi[b, 0])), (1, int(bp.lo[b, 1]), int(bp.hi[b, 1]))]
             for b in range(B)]
    preds[3] = []                       # no predicate
    preds[4] = [(0, 10, 5)]             # empty
    T = vrs.Table(_dev(x), _dev(a), normalize=True)
    ot = O.Table.build(x, a, O.F32, normalize=True)
    kmax = int(bp.k.max())
    ref = O.scan_topk(ot, q, preds, bp.k, O.IP, out_stride=kmax)
    r = T.scan_topk_batched(_dev(q), vrs.preds_tensor(preds), _dev(bp.k), kmax, vrs.IP)
    _check(r, ref, "batched")


@pytest.mark.parametrize("store", [vrs.BF16, vrs.FP8E4M3])
def test_lowprec_mfma_one_coordinate_chunk_partial_query_tile(store):
    # d = 64 is a single coordinate chunk per row, and B = 80 leaves the last
    # 64-query tile with 16 queries (one busy wave, three idle ones): the
    # idle waves run ahead into the next tile while the busy one is still
    # reading the current tile's row records.
    n, d, B = 300_000, 64, 80
    x = inputs.table(4, n, d, 500)
    a = inputs.attributes(4, n, 2, 10 ** 6)
    q = inputs.queries(4, B, d, 500)
    T = vrs.Table(_dev(x), _dev(a), store=store, normalize=True)
    ot = O.Table.build(x, a, O.BF16 if store == vrs.BF16 else O.FP8, True)
    for sel, k in ((0.04, 100), (1.0, 10)):
        w = inputs.two_term_width(sel, 10 ** 6)
        pred = [(0, 0, w), (1, 0, w)]
        ref = O.scan_topk(ot, q, pred, k, O.IP)
        for tile in (4, 6):
            for strategy in (vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER):
                r = T.scan_topk(_dev(q), pred, k, vrs.IP, tile=tile, strategy=strategy)
                _check(r, ref, f"store {store} sel {sel} k {k} tile {tile} strategy {strategy}")


@pytest.mark.parametrize("B", [1, 9])
def test_lowprec_largest_k_prime(B):
    # bfloat16 rows at k = 256 take k' = 1024: the widest screening lists,
    # merge bound over up to 4096 heads and the four-keys-per-thread sort
    n, d, k = 30000, 96, 256
    x = inputs.table(6, n, d, 40)
    a = inputs.attributes(6, n, 2, 1000)
    q = inputs.queries(6, B, d, 40)
    T = vrs.Table(_dev(x), _dev(a), store=vrs.BF16, normalize=True)
    ot = O.Table.build(x, a, O.BF16, True)
    pred = [(0, 0, 900)]
    ref = O.scan_topk(ot, q, pred, k, O.IP)
    for strategy in (vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER):
        r = T.scan_topk(_dev(q), pred, k, vrs.IP, strategy=strategy)
        _check(r, ref, f"B {B} strategy {strategy}")


@pytest.mark.parametrize("store,metric", [(vrs.F32, vrs.L2SQ), (vrs.F32, vrs.IP), (vrs.BF16, vrs.IP),
                                          (vrs.FP8E4M3, vrs.IP)])
def test_two_pass_mfma_screening(store, metric):
    # one and two MFMA screening passes (prefix of every chunk, merged bound,
    # the rest) give the oracle's result, also when the first pass sees fewer
    # qualifying rows than k' (dense and very selective predicates, gather)
    n, d, B = 90001, 128, 150
    x = inputs.table(7, n, d, 60)
    a = inputs.attributes(7, n, 2, 10 ** 6)
    q = inputs.queries(7, B, d, 60)
    normalize = metric == vrs.IP
    T = vrs.Table(_dev(x), _dev(a), store=store, normalize=normalize)
    ot = O.Table.build(x, a, {vrs.F32: O.F32, vrs.BF16: O.BF16, vrs.FP8E4M3: O.FP8}[store], normalize)
    om = O.L2SQ if metric == vrs.L2SQ else O.IP
    for sel, k in ((1.0, 100), (0.3, 10), (0.002, 100)):
        w = inputs.two_term_width(sel, 10 ** 6)
        pred = [(0, 0, w), (1, 0, w)] if sel < 1.0 else []
        ref = O.scan_topk(ot, q, pred, k, om)
        for tile in (4, 7):
            for strategy in (vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER):
                for passes in (1, 2):
                    r = T.scan_topk(_dev(q), pred, k, metric, tile=tile, strategy=strategy, passes=passes)
                    _check(r, ref, f"store {store} sel {sel} k {k} tile {tile} strategy {strategy} passes {passes}")


@pytest.mark.parametrize("store, metric", [(vrs.F32, vrs.L2SQ), (vrs.BF16, vrs.IP)])
def test_two_pass_bound_inside_a_run_of_ties(store, metric):
    # every vector appears 8 times (scattered over the table) and the
    # queries are table vectors, so the (k'+1)-th screening key sits inside
    # a run of equal distances: the second pass admits keys up to and
    # including the first pass's bound key (distance, then row id) and
    # must reproduce the oracle's ids exactly with one and two passes
    rng = np.random.default_rng(23)
    base = inputs.table(9, 20000, 128, 40)
    perm = rng.permutation(8 * 20000)
    x = np.ascontiguousarray(np.tile(base, (8, 1))[perm])
    n = x.shape[0]
    a = inputs.attributes(9, n, 2, 10 ** 6)
    q = np.ascontiguousarray(base[rng.integers(0, 20000, 40)])
    normalize = metric == vrs.IP
    T = vrs.Table(_dev(x), _dev(a), store=store, normalize=normalize)
    ot = O.Table.build(x, a, {vrs.F32: O.F32, vrs.BF16: O.BF16}[store], normalize)
    om = O.L2SQ if metric == vrs.L2SQ else O.IP
    for k in (1, 100):
        ref = O.scan_topk(ot, q, [], k, om)
        for tile in (4, 7):
            for passes in (1, 2):
                r = T.scan_topk(_dev(q), [], k, metric, tile=tile, strategy=vrs.STRATEGY_MASK, passes=passes)
                _check(r, ref, f"store {store} k {k} tile {tile} passes {passes}")


@pytest.mark.parametrize("metric", [vrs.L2SQ, vrs.IP])
def test_one_query_stream_bound_from_published_heads(metric):
    # one-query streaming scans over enough row chunks (>= k'+1) bound each
    # chunk's list by the k'+1-th smallest best key any chunk has published;
    # with 4 copies of every vector the bound falls inside runs of tied
    # distances, and ids must still match the oracle exactly
    rng = np.random.default_rng(31)
    base = inputs.table(12, 75000, 96, 50)
    x = np.ascontiguousarray(np.tile(base, (4, 1))[rng.permutation(4 * 75000)])
    n = x.shape[0]
    a = inputs.attributes(12, n, 2, 10 ** 6)
    normalize = metric == vrs.IP
    T = vrs.Table(_dev(x), _dev(a), normalize=normalize)
    ot = O.Table.build(x, a, O.F32, normalize)
    om = O.L2SQ if metric == vrs.L2SQ else O.IP
    q = np.ascontiguousarray(np.concatenate([base[rng.integers(0, 75000, 3)], inputs.queries(12, 3, 96, 50)]))
    for sel in (1.0, 0.2):
        w = inputs.two_term_width(sel, 10 ** 6)
        pred = [(0, 0, w), (1, 0, w)] if sel < 1.0 else []
        for k in (1, 10, 50):
            for strategy in (vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER):
                for i in range(q.shape[0]):
                    qi = q[i:i + 1]
                    ref = O.scan_topk(ot, qi, pred, k, om)
                    r = T.scan_topk(_dev(qi), pred, k, metric, tile=0, strategy=strategy)
                    _check(r, ref, f"metric {metric} sel {sel} k {k} strategy {strategy} query {i}")


def test_batch_limit_is_an_argument_error(cfg0):
    T = cfg0[3]
    assert T.workspace_bytes(vrs.MAX_BATCH, 10) > 0
    with pytest.raises(vrs.VrsError):
        T.workspace_bytes(vrs.MAX_BATCH + 1, 10)
    with pytest.raises(vrs.VrsError):
        T.batched_workspace_bytes(vrs.MAX_BATCH + 1, 10)


def test_fp8_subnormal_codes_rerank_exactly():
    # one large coordinate per row sets the row scale (max|x| / 448), so the
    # small coordinates encode to subnormal e4m3 codes (|x| / scale < 2^-6):
    # screening, rerank and fallback must still reproduce the oracle's FP64
    # distances of the stored codes bit for bit
    rng = np.random.default_rng(11)
    n, d, B = 6000, 64, 9
    x = (rng.standard_normal((n, d)) * 1e-5).astype(np.float32)
    x[np.arange(n), rng.integers(0, d, n)] = rng.uniform(0.5, 2.0, n).astype(np.float32)
    a = inputs.attributes(3, n, 1, 1000)
    q = rng.standard_normal((B, d)).astype(np.float32)
    T = vrs.Table(_dev(x), _dev(a), store=vrs.FP8E4M3)
    ot = O.Table.build(x, a, O.FP8, False)
    mag = T.export()[0].cpu().numpy() & 0x7F
    assert ((mag > 0) & (mag < 8)).sum() > n  # plenty of subnormal codes
    for k in (1, 50):
        ref = O.scan_topk(ot, q, [], k, O.IP)
        for strategy in (vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER):
            for kp in (0, 1):  # k' = k forces the exact fallback pass too
                r = T.scan_topk(_dev(q), [], k, vrs.IP, strategy=strategy, kprime_mult=kp)
                _check(r, ref, f"k {k} strategy {strategy} kprime_mult {kp}")


@pytest.mark.parametrize("store", [vrs.F32, vrs.BF16])
def test_dense_gather_plan_fits_its_workspace(store):
    # gather at a high estimated selectivity: the planner's row estimate
    # (1.25 x the estimated qualifying rows) exceeds the table, and its chunk
    # count must still fit the workspace sized for the whole table; the
    # workspace here is exactly the advertised size
    n, d, B, k = 40000, 128, 8, 100
    x = inputs.table(4, n, d, 100)
    a = inputs.attributes(4, n, 2, 10 ** 6)
    q = inputs.queries(4, B, d, 100)
    T = vrs.Table(_dev(x), _dev(a), store=store, normalize=True)
    ot = O.Table.build(x, a, {vrs.F32: O.F32, vrs.BF16: O.BF16}[store], True)
    w = inputs.two_term_width(0.9, 10 ** 6)
    pred = [(0, 0, w), (1, 0, w)]
    ref = O.scan_topk(ot, q, pred, k, O.IP)
    for tile in (4, 5, 6, 7):
        o = vrs.vrs_opts()
        o.strategy, o.tile = vrs.STRATEGY_GATHER, tile
        ws = torch.empty(T.workspace_bytes(B, k, o), dtype=torch.uint8, device="cuda")
        r = T.scan_topk(_dev(q), pred, k, vrs.IP, strategy=vrs.STRATEGY_GATHER, tile=tile, ws=ws)
        _check(r, ref, f"store {store} tile {tile}")
