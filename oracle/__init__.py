"""FP64 CPU oracle for the filtered exact top-k scan (ctypes binding).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are its only users.  The product library never imports,
links or calls anything here, and nothing here imports the product.

The arithmetic lives in ``oracle.c`` (plain C, FP64, loops over the paper's
Section 3 definitions); this module compiles it with gcc and marshals numpy
arrays.  ``mlp.py`` holds the FP64 reference of the access-path chooser's
network.

Parity status of every function is pinned by ``tests/test_oracle_*.py``.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

F32, BF16, FP8 = 0, 1, 2
L2SQ, IP = 0, 1

_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` next to it."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-fast-math", "-pthread", SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.oracle_abi_version.restype = C.c_int
        L.oracle_bf16_value.restype = C.c_double
        L.oracle_bf16_value.argtypes = [C.c_uint16]
        L.oracle_e4m3_value.restype = C.c_double
        L.oracle_e4m3_value.argtypes = [C.c_uint8]
        L.oracle_e4m3_from_f64.restype = C.c_uint8
        L.oracle_e4m3_from_f64.argtypes = [C.c_double]
        L.oracle_encode_bf16.restype = C.c_int64
        L.oracle_encode_bf16.argtypes = [P, C.c_int64, P]
        L.oracle_encode_fp8_rows.restype = None
        L.oracle_encode_fp8_rows.argtypes = [P, C.c_int64, C.c_int32, P, P]
        L.oracle_normalize_rows.restype = None
        L.oracle_normalize_rows.argtypes = [P, C.c_int64, C.c_int32, P]
        L.oracle_select.restype = C.c_int64
        L.oracle_select.argtypes = [P, C.c_int64, C.c_int32, P, P, P, P]
        L.oracle_distances.restype = None
        L.oracle_distances.argtypes = [C.c_int32, C.c_int64, C.c_int32, P, P, P, P, C.c_int64,
                                       C.c_int32, P]
        L.oracle_scan_topk.restype = C.c_int
        L.oracle_scan_topk.argtypes = [C.c_int32, C.c_int64, C.c_int32, P, P, P, P, C.c_int32,
                                       C.c_int32, P, P, P, P, P, C.c_int32, C.c_int32, C.c_int32,
                                       P, P, P, P]
        L.oracle_scan_range.restype = C.c_int
        L.oracle_scan_range.argtypes = [C.c_int32, C.c_int64, C.c_int32, P, P, P, P, C.c_int32,
                                        C.c_int32, P, P, P, P, P, C.c_int32, C.c_int32, C.c_int32,
                                        P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------- codecs
def bf16_values(codes) -> np.ndarray:
    codes = np.asarray(codes, dtype=np.uint16).ravel()
    return np.array([lib().oracle_bf16_value(int(c)) for c in codes], dtype=np.float64)


def e4m3_values(codes) -> np.ndarray:
    codes = np.asarray(codes, dtype=np.uint8).ravel()
    return np.array([lib().oracle_e4m3_value(int(c)) for c in codes], dtype=np.float64)


def e4m3_encode(values) -> np.ndarray:
    values = np.asarray(values, dtype=np.float64).ravel()
    return np.array([lib().oracle_e4m3_from_f64(float(v)) for v in values], dtype=np.uint8)


def encode_bf16(x):
    """float32 array -> (uint16 codes, number of finite values that overflowed)."""
    x = _c(x, np.float32)
    out = np.empty(x.shape, dtype=np.uint16)
    ov = lib().oracle_encode_bf16(_p(x), x.size, _p(out))
    return out, int(ov)


def encode_fp8_rows(x):
    """float32 ``[n, d]`` -> (uint8 codes ``[n, d]``, float32 scales ``[n]``)."""
    x = _c(x, np.float32)
    n, d = x.shape
    codes = np.empty((n, d), dtype=np.uint8)
    scale = np.empty(n, dtype=np.float32)
    lib().oracle_encode_fp8_rows(_p(x), n, d, _p(codes), _p(scale))
    return codes, scale


def normalize_rows(x):
    x = _c(x, np.float32)
    n, d = x.shape
    out = np.empty_like(x)
    lib().oracle_normalize_rows(_p(x), n, d, _p(out))
    return out


# ---------------------------------------------------------------- table
class Table:
    """A stored table as the oracle sees it: ``dtype`` in {F32, BF16, FP8},
    ``rows`` (float32, uint16 or uint8 ``[n, d]``), ``scale`` (FP8 only) and
    int32 attributes ``[n_attr, n]``."""

    def __init__(self, dtype, rows, attr, scale=None):
        self.dtype = int(dtype)
        want = {F32: np.float32, BF16: np.uint16, FP8: np.uint8}[self.dtype]
        self.rows = _c(rows, want)
        self.n, self.d = self.rows.shape
        attr = np.asarray(attr, dtype=np.int32)
        if attr.ndim == 1:
            attr = attr[None, :]
        self.attr = _c(attr, np.int32)
        assert self.attr.shape[1] == self.n
        self.scale = None if scale is None else _c(scale, np.float32)
        if self.dtype == FP8:
            assert self.scale is not None and self.scale.shape == (self.n,)

    @classmethod
    def build(cls, x, attr, dtype=F32, normalize=False):
        """The oracle's own stored table from float32 input rows: optional row
        normalisation, then the storage codec."""
        x = _c(x, np.float32)
        if normalize:
            x = normalize_rows(x)
        if dtype == F32:
            return cls(F32, x, attr)
        if dtype == BF16:
            codes, ov = encode_bf16(x)
            if ov:
                raise ValueError("bfloat16 overflow")
            return cls(BF16, codes, attr)
        codes, scale = encode_fp8_rows(x)
        return cls(FP8, codes, attr, scale)


def _terms(preds, B):
    """``preds``: one predicate for all queries or a list of B predicates;
    a predicate is a list of (col, lo, hi) triples."""
    if preds is None or (len(preds) > 0 and isinstance(preds[0], tuple)) or len(preds) == 0:
        preds = [list(preds or [])] * B
    assert len(preds) == B
    tmax = max(1, max(len(p) for p in preds))
    nterms = np.array([len(p) for p in preds], dtype=np.int32)
    cols = np.zeros((B, tmax), dtype=np.int32)
    lo = np.zeros((B, tmax), dtype=np.int64)
    hi = np.zeros((B, tmax), dtype=np.int64)
    for b, p in enumerate(preds):
        for t, (c, l, h) in enumerate(p):
            cols[b, t], lo[b, t], hi[b, t] = c, l, h
    return tmax, nterms, cols, lo, hi


def select(table: Table, pred):
    """Ascending ids of the rows satisfying the conjunction ``pred``."""
    _, nterms, cols, lo, hi = _terms(pred, 1)
    out = np.empty(table.n, dtype=np.int32)
    c = lib().oracle_select(_p(table.attr), table.n, int(nterms[0]), _p(cols[0]), _p(lo[0]),
                            _p(hi[0]), _p(out))
    return out[:c].copy()


def distances(table: Table, q, ids, metric):
    q = _c(q, np.float32).ravel()
    assert q.size == table.d
    ids = _c(ids, np.int64)
    out = np.empty(ids.size, dtype=np.float64)
    lib().oracle_distances(table.dtype, table.n, table.d, _p(table.rows), _p(table.scale), _p(q),
                           _p(ids), ids.size, int(metric), _p(out))
    return out


def scan_topk(table: Table, q, preds, k, metric, nthreads=None, out_stride=None):
    """Exact filtered top-k.  ``preds``: one predicate (list of (col, lo, hi))
    for every query, or a list with one predicate per query; ``k``: an int or
    one int per query.  Returns ``(idx int64 [B, K], dist float32 [B, K],
    dist64 float64 [B, K], nvalid int64 [B])`` with ``K = max k``."""
    q = _c(q, np.float32)
    if q.ndim == 1:
        q = q[None, :]
    B, d = q.shape
    assert d == table.d
    ks = np.broadcast_to(np.asarray(k, dtype=np.int32), (B,)).copy()
    K = int(out_stride or (ks.max() if B else 1))
    tmax, nterms, cols, lo, hi = _terms(preds, B)
    idx = np.empty((B, K), dtype=np.int64)
    dist = np.empty((B, K), dtype=np.float32)
    dist64 = np.empty((B, K), dtype=np.float64)
    nvalid = np.empty(B, dtype=np.int64)
    if nthreads is None:
        nthreads = len(os.sched_getaffinity(0))
    rc = lib().oracle_scan_topk(table.dtype, table.n, table.d, _p(table.rows), _p(table.scale),
                                _p(table.attr), _p(q), B, tmax, _p(nterms), _p(cols), _p(lo),
                                _p(hi), _p(ks), K, int(metric), int(nthreads), _p(idx),
                                _p(dist), _p(dist64), _p(nvalid))
    if rc != 0:
        raise MemoryError("oracle_scan_topk ran out of memory")
    return idx, dist, dist64, nvalid


def scan_range(table: Table, q, preds, thr, cap, metric, nthreads=None):
    """Threshold selection: for every query, the qualifying rows whose FP64
    distance is below its threshold, ascending by id.  ``thr``: a float or
    one per query; ``cap``: ids kept per query.  Returns ``(idx int64
    [B, cap], dist float32 [B, cap], dist64 float64 [B, cap], count int64
    [B])``, padded with -1 / +inf; ``count`` counts every selected row."""
    q = _c(q, np.float32)
    if q.ndim == 1:
        q = q[None, :]
    B, d = q.shape
    assert d == table.d
    th = np.ascontiguousarray(np.broadcast_to(np.asarray(thr, dtype=np.float64), (B,)))
    tmax, nterms, cols, lo, hi = _terms(preds, B)
    cap = int(cap)
    idx = np.empty((B, max(cap, 1)), dtype=np.int64)
    dist = np.empty((B, max(cap, 1)), dtype=np.float32)
    dist64 = np.empty((B, max(cap, 1)), dtype=np.float64)
    count = np.empty(B, dtype=np.int64)
    if nthreads is None:
        nthreads = len(os.sched_getaffinity(0))
    lib().oracle_scan_range(table.dtype, table.n, table.d, _p(table.rows), _p(table.scale),
                            _p(table.attr), _p(q), B, tmax, _p(nterms), _p(cols), _p(lo), _p(hi),
                            _p(th), cap, int(metric), int(nthreads), _p(idx), _p(dist), _p(dist64),
                            _p(count))
    return idx[:, :cap], dist[:, :cap], dist64[:, :cap], count


def stored_as_f32(table: Table) -> np.ndarray:
    """The stored vectors as float32 rows: float32 and bfloat16 values are
    exact; an FP8 value (scale * code) is rounded to the nearest float32."""
    if table.dtype == F32:
        return table.rows.copy()
    if table.dtype == BF16:
        return bf16_values(table.rows).reshape(table.n, table.d).astype(np.float32)
    vals = e4m3_values(table.rows).reshape(table.n, table.d)
    return (vals * table.scale.astype(np.float64)[:, None]).astype(np.float32)


def join_topk(r_table: Table, s_table: Table, preds, k, metric, nthreads=None):
    """Vector join: for every row of ``r_table`` (its stored vector as a
    float32 query), the exact filtered top-k rows of ``s_table``.  Returns
    what ``scan_topk`` returns, one row per row of ``r_table``."""
    assert r_table.d == s_table.d
    return scan_topk(s_table, stored_as_f32(r_table), preds, k, metric, nthreads=nthreads)


# ------------------------------------------------------------ probe path
# A partition index over the vector column (the probe-based access path of
# Section 4: data organised so that similar vectors sit together; here
# k-means partitions, squared L2 on the stored vectors) and its filtered
# probe with pre-filtering (Section 4.1: the relational predicate decides
# which rows may enter the result, not which partitions are visited).

def _nearest_centroid(x32, cent):
    """Exact nearest centroid of every row by (FP64 squared L2, centroid id)."""
    zr = np.zeros((1, x32.shape[0]), np.int32)
    zc = np.zeros((1, cent.shape[0]), np.int32)
    idx = join_topk(Table(F32, x32, zr), Table(F32, cent, zc), [], 1, L2SQ)[0]
    return idx[:, 0].astype(np.int32)


def _centroid_means(x32, assign, old):
    """Mean of each partition's rows: FP64 running sum in ascending row
    order, divided by the count, rounded to float32; an empty partition keeps
    its previous centroid."""
    cent = old.copy()
    for c in range(old.shape[0]):
        members = np.nonzero(assign == c)[0]
        if members.size:
            s = np.cumsum(x32[members].astype(np.float64), axis=0)[-1]
            cent[c] = (s / float(members.size)).astype(np.float32)
    return cent


def ivf_build(table: Table, nlist: int, iters: int):
    """k-means partition index: initial centroids are the stored rows at
    positions floor(i n / nlist); each iteration assigns every row to its
    exact nearest centroid and moves the centroids to their partitions'
    means; the final assignment uses the final centroids.  Returns
    (centroids float32 [nlist, d], assign int32 [n], list_off int64
    [nlist + 1], list_ids int32 [n]) with every partition's rows ascending."""
    x32 = stored_as_f32(table)
    n = table.n
    cent = x32[[(i * n) // nlist for i in range(nlist)]].copy()
    for _ in range(iters):
        cent = _centroid_means(x32, _nearest_centroid(x32, cent), cent)
    assign = _nearest_centroid(x32, cent)
    order = np.argsort(assign, kind="stable").astype(np.int32)
    counts = np.bincount(assign, minlength=nlist)
    list_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return cent, assign, list_off, order


def ivf_probe(table: Table, cent, list_off, list_ids, q, preds, k, metric, nprobe, min_cand, cap_c):
    """Filtered probe: each query walks the partitions in the order of their
    centroids' distance to it (exact, by FP64 squared L2 and centroid id; at
    most min(nlist, 256) of them); a visited partition contributes its rows
    that satisfy the predicate.  The first nprobe partitions are visited;
    past them the walk continues only while fewer than min_cand rows
    qualified (pre-filtering: a selective predicate makes the probe visit
    more of the index).  A partition that would take the rows visited past
    cap_c ends the walk (the first partition is always visited).  The result
    is the exact top-k of the collected rows by (FP64 distance, id).
    Returns (idx int64 [B, k], dist float32 [B, k], partitions visited int64
    [B], candidates int64 [B])."""
    q = _c(q, np.float32)
    B = q.shape[0]
    zc = np.zeros((1, cent.shape[0]), np.int32)
    walk = min(cent.shape[0], 256)
    coarse = scan_topk(Table(F32, cent, zc), q, [], walk, L2SQ)[0]
    _, nterms, cols, lo, hi = _terms(preds, B)
    idx = np.full((B, k), -1, np.int64)
    dist = np.full((B, k), np.inf, np.float32)
    taken = np.zeros(B, np.int64)
    ncand = np.zeros(B, np.int64)
    for b in range(B):
        cand, visited = [], 0
        for lst in coarse[b]:
            if lst < 0:
                break
            if taken[b] >= nprobe and len(cand) >= min_cand:
                break
            members = list_ids[list_off[lst]:list_off[lst + 1]]
            if taken[b] >= 1 and visited + members.size > cap_c:
                break
            ok = np.ones(members.size, bool)
            for t in range(nterms[b]):
                v = table.attr[cols[b, t], members].astype(np.int64)
                ok &= (lo[b, t] <= v) & (v < hi[b, t])
            cand.extend(members[ok].tolist())
            visited += members.size
            taken[b] += 1
        ncand[b] = len(cand)
        if cand:
            ids = np.array(cand, np.int64)
            d64 = distances(table, q[b], ids, metric)
            order = np.lexsort((ids, d64))[:k]
            idx[b, :order.size] = ids[order]
            dist[b, :order.size] = d64[order].astype(np.float32)
    return idx, dist, taken, ncand
