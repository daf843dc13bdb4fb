"""ctypes binding of ``libvrs.so`` (include/vrs.h), same names as the C ABI.

Argument marshalling only: every step of a scan runs in the library's gfx950
kernels.  PyTorch supplies device memory (queries, outputs, workspace through
its caching allocator) and the HIP stream.  There is no CPU fallback: if the
library is missing or no GPU is visible, calls raise.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvrs.so")
CHOOSER_WEIGHTS = os.path.join(HERE, "chooser_weights.bin")

VRS_OK, VRS_E_ARG, VRS_E_NONFINITE, VRS_E_NOMEM, VRS_E_UNSUPPORTED, VRS_E_HIP, VRS_E_WORKSPACE = range(7)
L2SQ, IP = 0, 1
F32, BF16, FP8E4M3 = 0, 1, 2
STRATEGY_AUTO, STRATEGY_MASK, STRATEGY_GATHER = 0, 1, 2
CHOOSER_LEARNED, CHOOSER_HEURISTIC = 0, 1
MAX_TERMS = 4
MAX_BATCH = 65535  # largest B of one call (VRS_MAX_BATCH)
NOALLOC_SCRATCH_BYTES = 64 << 20  # static workspace of vrs_scan_topk_noalloc (VRS_NOALLOC_SCRATCH_BYTES)

EXPORTS = [
    "vrs_build_table", "vrs_destroy_table", "vrs_table_info", "vrs_table_export",
    "vrs_scan_workspace_bytes", "vrs_select_workspace_bytes", "vrs_select", "vrs_scan_topk",
    "vrs_scan_topk_batched", "vrs_num_tiles", "vrs_chooser_load", "vrs_last_error",
    "vrs_profile", "vrs_stage_times", "vrs_mlp_forward", "vrs_mlp_backward", "vrs_mlp_adam",
    "vrs_chooser_set", "vrs_chooser_clear", "vrs_plan", "vrs_table_view",
    "vrs_batched_workspace_bytes", "vrs_batched_num_configs", "vrs_batched_tune",
    "vrs_batched_graph_create", "vrs_graph_launch", "vrs_graph_config", "vrs_graph_destroy",
    "vrs_range_workspace_bytes", "vrs_scan_range", "vrs_join_workspace_bytes", "vrs_join_topk",
    "vrs_index_build", "vrs_index_destroy", "vrs_index_info", "vrs_index_export", "vrs_probe_workspace_bytes",
    "vrs_probe_topk", "vrs_plan_access", "vrs_scan_topk_noalloc", "vrs_chooser_pick",
    "vrs_scan_graph_create",
]
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS = 6, 64, 16, 5648
NUM_STAGES = 6
STAGES = ["prep", "select", "screen", "merge", "rerank", "fallback"]


class VrsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"vrs status {status}: {msg}")
        self.status = status


class vrs_range(C.Structure):
    _fields_ = [("col", C.c_int32), ("_pad", C.c_int32), ("lo", C.c_int64), ("hi", C.c_int64)]


class vrs_pred(C.Structure):
    _fields_ = [("nterms", C.c_int32), ("_pad", C.c_int32), ("term", vrs_range * MAX_TERMS)]


class vrs_opts(C.Structure):
    _fields_ = [("strategy", C.c_int32), ("tile", C.c_int32), ("chooser", C.c_int32),
                ("kprime_mult", C.c_int32), ("n_valid", C.c_void_p), ("certified", C.c_void_p),
                ("passes", C.c_int32), ("_pad", C.c_int32), ("err_ratio", C.c_void_p)]


_lib = None


def lib() -> C.CDLL:
    """Load libvrs.so (built by ``paper_2403_15807_amd._build.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, S = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        sig = {
            "vrs_build_table": [P, I64, I32, P, I32, I32, I32, P, P],
            "vrs_destroy_table": [P],
            "vrs_table_info": [P, P, P, P, P, P],
            "vrs_table_export": [P, P, P, P],
            "vrs_scan_workspace_bytes": [P, I32, I32, P, P],
            "vrs_select_workspace_bytes": [P, P],
            "vrs_select": [P, P, P, P, P, S, P],
            "vrs_scan_topk": [P, P, I32, P, I32, I32, P, P, P, S, P, P],
            "vrs_scan_topk_batched": [P, P, I32, P, P, I32, I32, P, P, P, S, P, P],
            "vrs_num_tiles": [],
            "vrs_chooser_load": [C.c_char_p],
            "vrs_last_error": [],
            "vrs_profile": [I32],
            "vrs_stage_times": [P, P],
            "vrs_mlp_forward": [P, P, I32, P, P, P],
            "vrs_mlp_backward": [P, P, P, P, P, P, I32, I32, P, P, P, P, P],
            "vrs_mlp_adam": [P, P, P, P, I32, C.c_float, C.c_float, C.c_float, C.c_float, P],
            "vrs_chooser_set": [P, P, P],
            "vrs_chooser_clear": [],
            "vrs_plan": [P, I32, P, I32, I32, P, P, P, P],
            "vrs_table_view": [P, I64, P],
            "vrs_range_workspace_bytes": [P, I32, I32, P],
            "vrs_join_workspace_bytes": [P, P, I32, P, P],
            "vrs_index_build": [P, I32, I32, P, P],
            "vrs_index_destroy": [P],
            "vrs_index_info": [P, P, P],
            "vrs_index_export": [P, P, P, P, P],
            "vrs_probe_workspace_bytes": [P, I32, I32, I32, I64, P],
            "vrs_plan_access": [P, I32, P, I32, I32, I64, P, P, P],
            "vrs_scan_topk_noalloc": [P, P, I32, P, I32, I32, P, P, P, P],
            "vrs_chooser_pick": [P, P, P],
            "vrs_probe_topk": [P, P, I32, P, I32, I32, I32, I64, I64, P, P, P, P, S, P],
            "vrs_join_topk": [P, P, P, I32, I32, P, P, P, S, P, P],
            "vrs_scan_range": [P, P, I32, P, I32, P, I32, P, P, P, P, S, P, P],
            "vrs_batched_workspace_bytes": [P, I32, I32, I32, P, P],
            "vrs_batched_num_configs": [],
            "vrs_batched_tune": [P, P, I32, P, P, I32, I32, P, P, P, S, P, P, P, P],
            "vrs_batched_graph_create": [P, P, I32, P, P, I32, I32, P, P, P, S, P, P, P],
            "vrs_scan_graph_create": [P, P, I32, P, I32, I32, P, P, P, S, P, P, P],
            "vrs_graph_launch": [P, P],
            "vrs_graph_config": [P],
            "vrs_graph_destroy": [P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int32
        L.vrs_last_error.restype = C.c_char_p
        _lib = L
        # trained access-path chooser shipped with the package (see chooser.py)
        if os.path.exists(CHOOSER_WEIGHTS):
            L.vrs_chooser_load(CHOOSER_WEIGHTS.encode())
    return _lib


def _check(st: int):
    if st != VRS_OK:
        raise VrsError(st, lib().vrs_last_error().decode())


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def make_pred(terms) -> vrs_pred:
    """``terms``: iterable of ``(col, lo, hi)`` meaning ``lo <= A[col][i] < hi``."""
    terms = list(terms or [])
    if len(terms) > MAX_TERMS:
        raise ValueError(f"at most {MAX_TERMS} terms")
    p = vrs_pred()
    p.nterms = len(terms)
    for i, (c, lo, hi) in enumerate(terms):
        p.term[i].col, p.term[i].lo, p.term[i].hi = int(c), int(lo), int(hi)
    return p


def preds_tensor(pred_list, device="cuda") -> torch.Tensor:
    """Pack a list of predicates into a device byte tensor of ``vrs_pred``."""
    n = len(pred_list)
    buf = (vrs_pred * max(n, 1))()
    for i, terms in enumerate(pred_list):
        buf[i] = make_pred(terms)
    raw = bytes(C.string_at(C.addressof(buf), C.sizeof(vrs_pred) * n))
    return torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)


@dataclass
class ScanResult:
    idx: torch.Tensor
    dist: torch.Tensor
    n_valid: torch.Tensor
    certified: torch.Tensor
    err_ratio: torch.Tensor | None = None


@dataclass
class RangeResult:
    idx: torch.Tensor
    dist: torch.Tensor
    count: torch.Tensor


class Table:
    """A library-owned table (``vrs_build_table``), or a row-prefix view of
    one (``Table.view``)."""

    def __init__(self, vec: torch.Tensor | None, attr: torch.Tensor | None = None, store: int = F32,
                 normalize: bool = False, stream=None):
        if vec is None:  # filled in by view()
            return
        if not (vec.is_cuda and vec.dtype == torch.float32 and vec.dim() == 2):
            raise ValueError("vec must be a float32 [n, d] CUDA tensor")
        vec = vec.contiguous()
        n, d = vec.shape
        if attr is not None:
            if attr.dim() == 1:
                attr = attr[None, :]
            if not (attr.is_cuda and attr.dtype == torch.int32 and attr.shape[1] == n):
                raise ValueError("attr must be an int32 [n_attr, n] CUDA tensor")
            attr = attr.contiguous()
        n_attr = 0 if attr is None else attr.shape[0]
        h = C.c_void_p()
        _check(lib().vrs_build_table(_ptr(vec), n, d, _ptr(attr), n_attr, int(store),
                                     int(bool(normalize)), _stream(stream), C.byref(h)))
        self._h = h
        self.n, self.d, self.n_attr, self.store = n, d, n_attr, int(store)
        mx = C.c_double()
        _check(lib().vrs_table_info(h, None, None, None, None, C.byref(mx)))
        self.max_norm = mx.value

    @property
    def handle(self):
        return self._h

    def view(self, n: int) -> "Table":
        """Non-owning view of the first n rows (keep the parent alive)."""
        h = C.c_void_p()
        _check(lib().vrs_table_view(self._h, int(n), C.byref(h)))
        v = Table(None)
        v._h, v._parent = h, self
        v.n, v.d, v.n_attr, v.store, v.max_norm = int(n), self.d, self.n_attr, self.store, self.max_norm
        return v

    def plan(self, B: int, terms, k: int, metric: int = L2SQ, strategy: int = STRATEGY_AUTO,
             tile: int = -1, chooser: int = CHOOSER_LEARNED):
        """(features[6], strategy, tile) the planner picks for such a call."""
        o = vrs_opts()
        o.strategy, o.tile, o.chooser = strategy, tile, chooser
        f = (C.c_float * 6)()
        st, tl = C.c_int32(), C.c_int32()
        p = make_pred(terms)
        _check(lib().vrs_plan(self._h, B, C.byref(p), k, metric, C.byref(o), f, C.byref(st), C.byref(tl)))
        return list(f), st.value, tl.value

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().vrs_destroy_table(self._h))
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().vrs_destroy_table(self._h)
        except Exception:
            pass

    # -------------------------------------------------------------- helpers
    def export(self, stream=None):
        dt = {F32: torch.float32, BF16: torch.int16, FP8E4M3: torch.uint8}[self.store]
        rows = torch.empty((self.n, self.d), dtype=dt, device="cuda")
        scale = torch.empty(self.n, dtype=torch.float32, device="cuda") if self.store == FP8E4M3 else None
        _check(lib().vrs_table_export(self._h, _ptr(rows), _ptr(scale), _stream(stream)))
        return rows, scale

    def workspace_bytes(self, B: int, k_max: int, opts: vrs_opts | None = None) -> int:
        out = C.c_size_t()
        _check(lib().vrs_scan_workspace_bytes(self._h, B, k_max, None if opts is None else C.byref(opts),
                                              C.byref(out)))
        return out.value

    def workspace(self, B: int, k_max: int, opts: vrs_opts | None = None) -> torch.Tensor:
        return torch.empty(max(self.workspace_bytes(B, k_max, opts), 256), dtype=torch.uint8, device="cuda")

    def select(self, terms, stream=None):
        nb = C.c_size_t()
        _check(lib().vrs_select_workspace_bytes(self._h, C.byref(nb)))
        ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device="cuda")
        ids = torch.empty(self.n, dtype=torch.int32, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        p = make_pred(terms)
        _check(lib().vrs_select(self._h, C.byref(p), _ptr(ids), _ptr(cnt), _ptr(ws), ws.numel(),
                                _stream(stream)))
        return ids[: int(cnt.item())]

    def _opts(self, B, strategy, tile, chooser, kprime_mult, n_valid, certified, passes=0, err_ratio=None):
        o = vrs_opts()
        o.strategy, o.tile, o.chooser, o.kprime_mult, o.passes = strategy, tile, chooser, kprime_mult, passes
        o.n_valid = n_valid.data_ptr()
        o.certified = certified.data_ptr()
        o.err_ratio = None if err_ratio is None else err_ratio.data_ptr()
        return o

    def scan_topk(self, q: torch.Tensor, terms, k: int, metric: int = L2SQ, strategy: int = STRATEGY_AUTO,
                  tile: int = -1, chooser: int = CHOOSER_LEARNED, kprime_mult: int = 0,
                  ws: torch.Tensor | None = None, out: tuple | None = None, stream=None,
                  passes: int = 0, diag: bool = False) -> ScanResult:
        """Filtered exact top-k of the queries ``q`` [B, d] (one predicate);
        ``passes`` forces one- or two-pass MFMA screening (0 = planner's choice);
        ``diag`` also returns the screening error ratio per query (``err_ratio``)."""
        q = q.contiguous()
        B = q.shape[0]
        if out is None:
            idx = torch.empty((B, k), dtype=torch.int64, device="cuda")
            dist = torch.empty((B, k), dtype=torch.float32, device="cuda")
            nv = torch.empty(B, dtype=torch.int32, device="cuda")
            cert = torch.empty(B, dtype=torch.uint8, device="cuda")
        else:
            idx, dist, nv, cert = out
        er = torch.empty(B, dtype=torch.float32, device="cuda") if diag else None
        o = self._opts(B, strategy, tile, chooser, kprime_mult, nv, cert, passes, er)
        if ws is None:
            ws = self.workspace(B, k, o)
        p = make_pred(terms)
        _check(lib().vrs_scan_topk(self._h, _ptr(q), B, C.byref(p), k, metric, _ptr(idx), _ptr(dist),
                                   _ptr(ws), ws.numel(), C.byref(o), _stream(stream)))
        return ScanResult(idx, dist, nv, cert, er)

    def scan_graph(self, q: torch.Tensor, terms, k: int, metric: int = L2SQ, strategy: int = STRATEGY_AUTO,
                   tile: int = -1, chooser: int = CHOOSER_LEARNED, kprime_mult: int = 0,
                   ws: torch.Tensor | None = None, out: tuple | None = None, stream=None,
                   passes: int = 0) -> "BatchedGraph":
        """Capture ``scan_topk`` for these buffers into a HIP graph
        (``vrs_scan_graph_create``); ``launch()`` replays it.  Write new query
        vectors into ``q`` between replays; the results land in ``result``."""
        q = q.contiguous()
        B = q.shape[0]
        if out is None:
            out = (torch.empty((B, k), dtype=torch.int64, device="cuda"),
                   torch.empty((B, k), dtype=torch.float32, device="cuda"),
                   torch.empty(B, dtype=torch.int32, device="cuda"),
                   torch.empty(B, dtype=torch.uint8, device="cuda"))
        idx, dist, nv, cert = out
        o = self._opts(B, strategy, tile, chooser, kprime_mult, nv, cert, passes)
        if ws is None:
            ws = self.workspace(B, k, o)
        p = make_pred(terms)
        h = C.c_void_p()
        _check(lib().vrs_scan_graph_create(self._h, _ptr(q), B, C.byref(p), k, metric, _ptr(idx), _ptr(dist),
                                           _ptr(ws), ws.numel(), C.byref(o), _stream(stream), C.byref(h)))
        return BatchedGraph(h, (q, ws, self, o), ScanResult(idx, dist, nv, cert))

    def range_workspace_bytes(self, B: int, cap: int) -> int:
        out = C.c_size_t()
        _check(lib().vrs_range_workspace_bytes(self._h, B, cap, C.byref(out)))
        return out.value

    def scan_range(self, q: torch.Tensor, terms, thr, cap: int, metric: int = IP,
                   strategy: int = STRATEGY_AUTO, ws: torch.Tensor | None = None, out: tuple | None = None,
                   stream=None) -> RangeResult:
        """Threshold selection: per query, the qualifying rows whose exact
        distance is below ``thr`` (a float, or one per query), ascending by
        id, at most ``cap`` of them; ``count`` counts them all."""
        q = q.contiguous()
        B = q.shape[0]
        th = torch.as_tensor(thr, dtype=torch.float64).reshape(-1).expand(B).contiguous().to("cuda")
        if out is None:
            idx = torch.empty((B, cap), dtype=torch.int64, device="cuda")
            dist = torch.empty((B, cap), dtype=torch.float32, device="cuda")
            cnt = torch.empty(B, dtype=torch.int64, device="cuda")
        else:
            idx, dist, cnt = out
        if ws is None:
            ws = torch.empty(max(self.range_workspace_bytes(B, cap), 256), dtype=torch.uint8, device="cuda")
        o = vrs_opts()
        o.strategy = strategy
        p = make_pred(terms)
        _check(lib().vrs_scan_range(self._h, _ptr(q), B, C.byref(p), metric, _ptr(th), cap, _ptr(idx),
                                    _ptr(dist), _ptr(cnt), _ptr(ws), ws.numel(), C.byref(o), _stream(stream)))
        return RangeResult(idx, dist, cnt)

    def join_workspace_bytes(self, S: "Table", k: int) -> int:
        nb = C.c_size_t()
        _check(lib().vrs_join_workspace_bytes(self._h, S.handle, k, None, C.byref(nb)))
        return nb.value

    def join_topk(self, S: "Table", terms, k: int, metric: int = L2SQ, strategy: int = STRATEGY_AUTO,
                  tile: int = -1, diag: bool = False, ws: torch.Tensor | None = None, stream=None) -> ScanResult:
        """Vector join: every row of this table (its stored vector) as a
        query against ``S``; one result row per row of this table."""
        n = self.n
        idx = torch.empty((n, k), dtype=torch.int64, device="cuda")
        dist = torch.empty((n, k), dtype=torch.float32, device="cuda")
        nv = torch.empty(n, dtype=torch.int32, device="cuda")
        cert = torch.empty(n, dtype=torch.uint8, device="cuda")
        er = torch.empty(n, dtype=torch.float32, device="cuda") if diag else None
        o = self._opts(n, strategy, tile, CHOOSER_LEARNED, 0, nv, cert, 0, er)
        if ws is None:
            nb = C.c_size_t()
            _check(lib().vrs_join_workspace_bytes(self._h, S.handle, k, C.byref(o), C.byref(nb)))
            ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device="cuda")
        p = make_pred(terms)
        _check(lib().vrs_join_topk(self._h, S.handle, C.byref(p), k, metric, _ptr(idx), _ptr(dist), _ptr(ws),
                                   ws.numel(), C.byref(o), _stream(stream)))
        return ScanResult(idx, dist, nv, cert, er)

    def batched_workspace_bytes(self, B: int, k_max: int, metric: int = IP, opts: vrs_opts | None = None) -> int:
        out = C.c_size_t()
        _check(lib().vrs_batched_workspace_bytes(self._h, B, k_max, metric,
                                                 None if opts is None else C.byref(opts), C.byref(out)))
        return out.value

    def _batched_args(self, q, k_max, metric, tile, kprime_mult, ws, out, passes=0, err_ratio=None):
        q = q.contiguous()
        B = q.shape[0]
        if out is None:
            out = (torch.empty((B, k_max), dtype=torch.int64, device="cuda"),
                   torch.empty((B, k_max), dtype=torch.float32, device="cuda"),
                   torch.empty(B, dtype=torch.int32, device="cuda"),
                   torch.empty(B, dtype=torch.uint8, device="cuda"))
        idx, dist, nv, cert = out
        o = self._opts(B, STRATEGY_MASK, tile, CHOOSER_HEURISTIC, kprime_mult, nv, cert, passes, err_ratio)
        if ws is None:
            ws = torch.empty(max(self.batched_workspace_bytes(B, k_max, metric, o), 256), dtype=torch.uint8,
                             device="cuda")
        return q, B, o, ws, (idx, dist, nv, cert)

    def scan_topk_batched(self, q: torch.Tensor, preds: torch.Tensor, ks: torch.Tensor, k_max: int,
                          metric: int = IP, tile: int = -1, kprime_mult: int = 0,
                          ws: torch.Tensor | None = None, out: tuple | None = None,
                          stream=None, passes: int = 0, diag: bool = False) -> ScanResult:
        """Per-query predicates (``preds_tensor``) and k (int32 device tensor).
        ``tile`` is a batched configuration index (-1: tuned or default);
        ``passes`` forces one- or two-pass dense screening (0 = by table size);
        ``diag`` also returns the screening error ratio per query."""
        er = torch.empty(q.shape[0], dtype=torch.float32, device="cuda") if diag else None
        q, B, o, ws, (idx, dist, nv, cert) = self._batched_args(q, k_max, metric, tile, kprime_mult, ws, out,
                                                                passes, er)
        _check(lib().vrs_scan_topk_batched(self._h, _ptr(q), B, _ptr(preds), _ptr(ks), k_max, metric,
                                           _ptr(idx), _ptr(dist), _ptr(ws), ws.numel(), C.byref(o),
                                           _stream(stream)))
        return ScanResult(idx, dist, nv, cert, er)

    def batched_tune(self, q, preds, ks, k_max: int, metric: int = IP, kprime_mult: int = 0,
                     ws=None, out=None, stream=None):
        """Autotune the batched configuration on these inputs: (best, ms per
        configuration, ScanResult of the best)."""
        q, B, o, ws, (idx, dist, nv, cert) = self._batched_args(q, k_max, metric, -1, kprime_mult, ws, out)
        n = batched_num_configs()
        ms = (C.c_float * n)()
        best = C.c_int32()
        _check(lib().vrs_batched_tune(self._h, _ptr(q), B, _ptr(preds), _ptr(ks), k_max, metric, _ptr(idx),
                                      _ptr(dist), _ptr(ws), ws.numel(), C.byref(o), _stream(stream),
                                      C.byref(best), ms))
        return best.value, list(ms), ScanResult(idx, dist, nv, cert)

    def batched_graph(self, q, preds, ks, k_max: int, metric: int = IP, tile: int = -1,
                      kprime_mult: int = 0, ws=None, out=None, stream=None) -> "BatchedGraph":
        """Capture the batched launch for these buffers into a HIP graph."""
        q, B, o, ws, res = self._batched_args(q, k_max, metric, tile, kprime_mult, ws, out)
        h = C.c_void_p()
        idx, dist, nv, cert = res
        _check(lib().vrs_batched_graph_create(self._h, _ptr(q), B, _ptr(preds), _ptr(ks), k_max, metric,
                                              _ptr(idx), _ptr(dist), _ptr(ws), ws.numel(), C.byref(o),
                                              _stream(stream), C.byref(h)))
        return BatchedGraph(h, (q, preds, ks, ws, self), ScanResult(idx, dist, nv, cert))


class Index:
    """A partition index over a table's vector column (``vrs_index_build``);
    keep the table alive while the index is used."""

    def __init__(self, table: "Table", nlist: int, iters: int = 10, stream=None):
        h = C.c_void_p()
        _check(lib().vrs_index_build(table.handle, int(nlist), int(iters), _stream(stream), C.byref(h)))
        self._h, self.table = h, table
        nl, ml = C.c_int32(), C.c_int64()
        _check(lib().vrs_index_info(h, C.byref(nl), C.byref(ml)))
        self.nlist, self.max_list = nl.value, ml.value

    def export(self, stream=None):
        cent = torch.empty((self.nlist, self.table.d), dtype=torch.float32, device="cuda")
        off = torch.empty(self.nlist + 1, dtype=torch.int64, device="cuda")
        ids = torch.empty(self.table.n, dtype=torch.int32, device="cuda")
        _check(lib().vrs_index_export(self._h, _ptr(cent), _ptr(off), _ptr(ids), _stream(stream)))
        return cent, off, ids

    def workspace_bytes(self, B: int, k: int, nprobe: int, cap_c: int) -> int:
        nb = C.c_size_t()
        _check(lib().vrs_probe_workspace_bytes(self._h, B, k, nprobe, cap_c, C.byref(nb)))
        return nb.value

    def probe_topk(self, q: torch.Tensor, terms, k: int, metric: int = L2SQ, nprobe: int = 16,
                   min_cand: int | None = None, cap_c: int = 1 << 16, ws: torch.Tensor | None = None,
                   out: tuple | None = None, stream=None):
        """Filtered probe: (idx [B, k], dist [B, k], partitions visited [B])."""
        q = q.contiguous()
        B = q.shape[0]
        if out is None:
            out = (torch.empty((B, k), dtype=torch.int64, device="cuda"),
                   torch.empty((B, k), dtype=torch.float32, device="cuda"),
                   torch.empty(B, dtype=torch.int32, device="cuda"))
        idx, dist, taken = out
        if ws is None:
            ws = torch.empty(max(self.workspace_bytes(B, k, nprobe, cap_c), 256), dtype=torch.uint8, device="cuda")
        p = make_pred(terms)
        _check(lib().vrs_probe_topk(self._h, _ptr(q), B, C.byref(p), k, metric, nprobe,
                                    int(min_cand if min_cand is not None else k), int(cap_c), _ptr(idx),
                                    _ptr(dist), _ptr(taken), _ptr(ws), ws.numel(), _stream(stream)))
        return idx, dist, taken

    def plan_access(self, B: int, terms, k: int, nprobe: int = 16, cap_c: int = 1 << 16):
        """(estimated scan ms, estimated probe ms, probe faster?)"""
        sc, pr, up = C.c_double(), C.c_double(), C.c_int32()
        p = make_pred(terms)
        _check(lib().vrs_plan_access(self._h, B, C.byref(p), k, nprobe, cap_c, C.byref(sc), C.byref(pr),
                                     C.byref(up)))
        return sc.value, pr.value, bool(up.value)

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().vrs_index_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().vrs_index_destroy(self._h)
        except Exception:
            pass


class BatchedGraph:
    """A captured launch sequence (batched form or single-predicate scan);
    ``launch()`` replays it on a stream.  The buffers it was captured with
    are kept alive here."""

    def __init__(self, h, keep, result: ScanResult):
        self._h = h
        self._keep = keep
        self.result = result

    @property
    def config(self) -> int:
        return int(lib().vrs_graph_config(self._h))

    def launch(self, stream=None):
        _check(lib().vrs_graph_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().vrs_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().vrs_graph_destroy(self._h)
        except Exception:
            pass


def batched_num_configs() -> int:
    return int(lib().vrs_batched_num_configs())


def profile(enable: bool):
    _check(lib().vrs_profile(int(bool(enable))))


def stage_times():
    """Accumulated (ms, calls) per stage since the last read."""
    ms = (C.c_double * NUM_STAGES)()
    calls = (C.c_int64 * NUM_STAGES)()
    _check(lib().vrs_stage_times(ms, calls))
    return {STAGES[i]: (ms[i], calls[i]) for i in range(NUM_STAGES)}


def mlp_forward(params: torch.Tensor, x: torch.Tensor, act: torch.Tensor | None = None, stream=None):
    y = torch.empty((x.shape[0], MLP_OUT), dtype=torch.float32, device=x.device)
    _check(lib().vrs_mlp_forward(_ptr(params), _ptr(x), x.shape[0], _ptr(y), _ptr(act), _stream(stream)))
    return y


def mlp_backward(params, x, y, act, target, mask, stream=None):
    """Returns (grad [MLP_PARAMS], loss [1]) of the masked mean squared error."""
    nb = x.shape[0]
    count = int(mask.sum().item())
    sig = torch.empty((nb, MLP_OUT + 2 * MLP_HIDDEN), dtype=torch.float32, device=x.device)
    sq = torch.empty(nb, dtype=torch.float32, device=x.device)
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check(lib().vrs_mlp_backward(_ptr(params), _ptr(x), _ptr(y), _ptr(act), _ptr(target), _ptr(mask),
                                  nb, count, _ptr(sig), _ptr(sq), _ptr(grad), _ptr(loss), _stream(stream)))
    return grad, loss


def mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().vrs_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr),
                              float(beta1), float(beta2), float(eps), _stream(stream)))


def chooser_set(params, mean, std):
    import numpy as np
    p = np.ascontiguousarray(params, dtype=np.float32)
    mu = np.ascontiguousarray(mean, dtype=np.float32)
    sd = np.ascontiguousarray(std, dtype=np.float32)
    _check(lib().vrs_chooser_set(p.ctypes.data, mu.ctypes.data, sd.ctypes.data))


def chooser_clear():
    _check(lib().vrs_chooser_clear())


def chooser_pick(feats, allowed) -> int:
    """The installed network's pick among the allowed arms (host inference,
    as the planner runs it); -1 without a network."""
    import numpy as np
    f = np.ascontiguousarray(feats, dtype=np.float32)
    al = np.ascontiguousarray(allowed, dtype=np.uint8)
    arm = C.c_int32()
    _check(lib().vrs_chooser_pick(f.ctypes.data, al.ctypes.data, C.byref(arm)))
    return arm.value


def num_tiles() -> int:
    return int(lib().vrs_num_tiles())


def chooser_load(path: str) -> bool:
    return lib().vrs_chooser_load(path.encode()) == VRS_OK
