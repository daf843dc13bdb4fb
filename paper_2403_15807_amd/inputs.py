"""Seeded synthetic inputs for the filtered top-k scan.

This module only draws random numbers: it holds none of the search
arithmetic (no distances, no predicates, no ranking, no quantisation, no
normalisation), so both the FP64 oracle tests and the GPU path may use it.

The paper evaluates on synthetic data generated with a fixed seed (Section 5,
"Dataset"); the inputs here follow the same idea with clustered Gaussian
vectors so that nearest neighbours are meaningful:

* ``n_clusters`` centres, each ~ N(0, I_d) in float64;
* every table row picks a centre uniformly and adds ``sigma`` * N(0, I_d)
  noise, the sum rounded once to float32;
* queries are fresh draws from the same mixture (not table rows);
* relational attributes are i.i.d. uniform int32 in ``[0, attr_range)``,
  stored column-major ``[n_attr][n]``.

Rows are generated in fixed chunks of ``CHUNK`` rows, each chunk from its own
child seed, so a table of ``n`` rows is a prefix of any larger table drawn with
the same arguments and chunks can be generated on several threads.
"""

from __future__ import annotations

import concurrent.futures as _cf
import os
from dataclasses import dataclass

import numpy as np

BASE_SEED = 240315807
CHUNK = 1 << 20

# Stream identifiers inside one configuration's seed space.
_S_CENTERS, _S_ROWS, _S_ATTR, _S_QUERY, _S_PRED = 0, 1, 2, 3, 4


def _rng(cfg: int, stream: int, chunk: int = 0) -> np.random.Generator:
    ss = np.random.SeedSequence(entropy=BASE_SEED, spawn_key=(cfg, stream, chunk))
    return np.random.Generator(np.random.PCG64(ss))


def _threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def centers(cfg: int, n_clusters: int, d: int) -> np.ndarray:
    """Cluster centres, float64 ``[n_clusters, d]``."""
    return _rng(cfg, _S_CENTERS).standard_normal((n_clusters, d))


_SUB = 1 << 16  # rows per noise block inside a chunk (bounds temporary memory)


def _rows_chunk(cfg, c, lo, hi, d, cent, sigma, out):
    g = _rng(cfg, _S_ROWS, c)
    lab = g.integers(0, cent.shape[0], size=hi - lo)
    for a in range(0, hi - lo, _SUB):
        b = min(hi - lo, a + _SUB)
        z = g.standard_normal((b - a, d))
        out[lo + a:lo + b] = (cent[lab[a:b]] + sigma * z).astype(np.float32)


def table(cfg: int, n: int, d: int, n_clusters: int, sigma: float = 0.1) -> np.ndarray:
    """Clustered Gaussian table, float32 ``[n, d]`` row-major."""
    cent = centers(cfg, n_clusters, d)
    out = np.empty((n, d), dtype=np.float32)
    jobs = [(c, c * CHUNK, min(n, (c + 1) * CHUNK)) for c in range((n + CHUNK - 1) // CHUNK)]
    if len(jobs) <= 1:
        for c, lo, hi in jobs:
            _rows_chunk(cfg, c, lo, hi, d, cent, sigma, out)
        return out
    with _cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(lambda j: _rows_chunk(cfg, j[0], j[1], j[2], d, cent, sigma, out), jobs))
    return out


def queries(cfg: int, b: int, d: int, n_clusters: int, sigma: float = 0.1,
            stream_offset: int = 0) -> np.ndarray:
    """``b`` fresh draws from the table's mixture, float32 ``[b, d]``."""
    cent = centers(cfg, n_clusters, d)
    g = _rng(cfg, _S_QUERY, stream_offset)
    lab = g.integers(0, n_clusters, size=b)
    z = g.standard_normal((b, d))
    return (cent[lab] + sigma * z).astype(np.float32)


def _attr_chunk(cfg, c, lo, hi, n_attr, attr_range, out):
    g = _rng(cfg, _S_ATTR, c)
    out[:, lo:hi] = g.integers(0, attr_range, size=(n_attr, hi - lo), dtype=np.int32)


def attributes(cfg: int, n: int, n_attr: int, attr_range: int) -> np.ndarray:
    """i.i.d. uniform int32 attributes, column-major ``[n_attr, n]``."""
    out = np.empty((n_attr, n), dtype=np.int32)
    jobs = [(c, c * CHUNK, min(n, (c + 1) * CHUNK)) for c in range((n + CHUNK - 1) // CHUNK)]
    if len(jobs) <= 1:
        for c, lo, hi in jobs:
            _attr_chunk(cfg, c, lo, hi, n_attr, attr_range, out)
        return out
    with _cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(lambda j: _attr_chunk(cfg, j[0], j[1], j[2], n_attr, attr_range, out), jobs))
    return out


def two_term_width(selectivity: float, attr_range: int) -> int:
    """Width ``w`` of ``[0, w)`` on each of two independent uniform columns so
    that the conjunction keeps about ``selectivity`` of the rows."""
    return int(max(1, min(attr_range, round(attr_range * float(selectivity) ** 0.5))))


@dataclass
class BatchedPredicates:
    """Per-query two-term ranges ``lo[b, t] <= A[t][i] < hi[b, t]`` and ``k[b]``."""
    lo: np.ndarray        # int64 [B, 2]
    hi: np.ndarray        # int64 [B, 2]
    k: np.ndarray         # int32 [B]
    target_sel: np.ndarray  # float64 [B], the drawn selectivity


def batched_predicates(cfg: int, b: int, attr_range: int, s_min: float = 1e-4,
                       s_max: float = 1.0, k_choices=(1, 10, 100)) -> BatchedPredicates:
    """Per-query selectivity ``s ~ logU[s_min, s_max]`` split over two columns
    as ``s0 = s**u``, ``s1 = s**(1-u)`` with ``u ~ U[0, 1]``, at random offsets,
    and ``k`` uniform over ``k_choices``."""
    g = _rng(cfg, _S_PRED)
    s = np.exp(g.uniform(np.log(s_min), np.log(s_max), size=b))
    u = g.uniform(0.0, 1.0, size=b)
    widths = np.stack([np.round(attr_range * s ** u), np.round(attr_range * s ** (1.0 - u))], axis=1)
    widths = np.clip(widths, 1, attr_range).astype(np.int64)
    lo = (g.uniform(0.0, 1.0, size=(b, 2)) * (attr_range - widths + 1)).astype(np.int64)
    lo = np.minimum(lo, attr_range - widths)
    hi = lo + widths
    k = np.asarray(k_choices, dtype=np.int32)[g.integers(0, len(k_choices), size=b)]
    return BatchedPredicates(lo=lo, hi=hi, k=k, target_sel=s)


@dataclass
class ChooserWorkload:
    """One scan configuration of the chooser's training or held-out set."""
    n: int
    d: int
    b: int
    sel: float
    k: int
    dtype: int      # 0 float32, 1 bfloat16, 2 FP8
    seed: int       # query / predicate stream for this workload


CHOOSER_DIMS = (64, 128, 768, 1536)
CHOOSER_MAX_ROWS = {64: 10_000_000, 128: 10_000_000, 768: 4_000_000, 1536: 2_000_000}


def chooser_workloads(cfg: int, count: int, n_min: int = 100_000, b_max: int = 4096):
    """``count`` workloads: n ~ logU[n_min, max rows for d], d uniform over
    CHOOSER_DIMS, B ~ logU-integer[1, b_max], selectivity ~ logU[1e-4, 1]
    with probability 3/4 and U[0.3, 1] otherwise (the dense end, where the
    masked and gathered scans trade places), k uniform over {1, 10, 100},
    storage dtype uniform over {f32, bf16, fp8}."""
    g = _rng(cfg, _S_PRED, 7)
    out = []
    for i in range(count):
        d = int(CHOOSER_DIMS[g.integers(0, len(CHOOSER_DIMS))])
        n_max = CHOOSER_MAX_ROWS[d]
        n = int(round(np.exp(g.uniform(np.log(n_min), np.log(n_max)))))
        b = int(min(b_max, max(1, int(np.floor(np.exp(g.uniform(0.0, np.log(b_max + 1))))))))
        sel = float(np.exp(g.uniform(np.log(1e-4), 0.0)))
        if g.uniform() < 0.25:
            sel = float(g.uniform(0.3, 1.0))
        k = int((1, 10, 100)[g.integers(0, 3)])
        dtype = int(g.integers(0, 3))
        out.append(ChooserWorkload(n=n, d=d, b=b, sel=sel, k=k, dtype=dtype, seed=int(g.integers(0, 2 ** 31))))
    return out
