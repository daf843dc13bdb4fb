"""Benchmark: filtered exact top-k queries/s on one MI355X.

Default workload (``--workload scan``): 10,000,000 x 128 float32 vectors
drawn from a mixture of 1000 Gaussians (sigma 0.1), two int32 attributes
uniform in [0, 10^6), a two-term range predicate of the requested
selectivity, squared-L2 top-100, one query per batch.  A step is one
``vrs_scan_topk`` call over one batch (the whole hot path: query prep,
predicate pass, screening, merge, FP64 rerank and certificate, fallback);
inputs are resident in HBM before timing starts.  The same line carries a
sweep of the workload's grid (batch 1/16/128/1024, selectivity 0.01%..100%,
mask and gather, L2 and inner product on normalised rows), each point timed
the same way.

``--workload batched``: 2,000,000 x 1536 bfloat16 rows (normalised), 4096
queries each with its own two-term range predicate (selectivity log-uniform
in [1e-4, 1]) and k in {1, 10, 100}; a step is one replay of the
HIP-graph-captured batched launch, with the autotuned configuration; the
plain path's per-query launches are timed beside it.

Prints one JSON line with the throughput, the roofline position of the
dominant kernel (screening) measured with HIP events on the scan's stream,
and the FP64 CPU oracle timed on a bounded sample of the same workload on the
host's cores.
"""

from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
CSRC = os.path.join(ROOT, "paper_2403_15807_amd", "csrc")

HBM_PEAK_GBS = 8000.0
MFMA_F32_PEAK_TFLOPS = 157.3
MFMA_BF16_PEAK_TFLOPS = 2500.0
ATTR = 10 ** 6

# Sources that make up each screening kernel (a traffic figure measured on an
# older version of them is not reported).
KERNEL_SOURCES = {
    "screen_stream": ["k_stream.hip", "topk_sized.h"],
    "screen_mfma_f32": ["k_mfma.hip", "wave_topk.h"],
    "screen_mfma_bf16": ["k_mfma_bf16.hip", "wave_topk.h"],
    "range_screen": ["k_range.hip", "exact64.h"],
}



def timed_then_profiled(fn, reps, torch, vrs):
    """Time `reps` calls with no instrumentation, then repeat them with the
    library's per-stage event profiling on (the events cost time of their own,
    so they stay out of the timed loop).  Returns (seconds, stage times)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    vrs.stage_times()  # drop anything recorded before
    vrs.profile(True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    vrs.profile(False)
    return elapsed, vrs.stage_times()

def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(kernel):
    """Hash of the kernel's source file and the device headers it uses (host
    structures elsewhere may change without changing the kernel)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel] + ["common.h"]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch from a committed counter summary under profiles/
    (FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel calibration), if it
    was taken on the current kernel source; else None."""
    want = source_hash(kernel)
    pat = re.compile(r"^traffic kernel=(\S+) workload=(\S+) source=(\S+) bytes_per_launch=(\d+)")
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        with open(path) as fh:
            for line in fh:
                m = pat.match(line.strip())
                if m and m.group(1) == kernel and m.group(2) == workload and m.group(3) == want:
                    return int(m.group(4))
    return None


def screen_kernel_name(store, used_mfma):
    if not used_mfma:
        return "screen_stream"
    return "screen_mfma_f32" if store == "f32" else "screen_mfma_bf16"


def roofline(n_sel, n, d, B, store, gather, n_terms, screen_ms, launches=1):
    """Roofline of the screening kernel.  ``screen_ms`` is its average
    launch duration; a scan that screens in ``launches`` passes splits one
    step's algorithmic work over them, so the work per launch is the step's
    divided by ``launches`` (achieved = step work / step screening time)."""
    row_bytes = d * {"f32": 4, "bf16": 2, "fp8": 1}[store] + (4 if store == "fp8" else 0)
    bytes_alg = (n_sel * row_bytes + (n_sel * 4 if gather else n * 4 * n_terms) + B * d * 4) / launches
    flops_alg = 2.0 * B * n_sel * d / launches
    hbm_gbs = bytes_alg / (screen_ms * 1e-3) / 1e9
    tflops = flops_alg / (screen_ms * 1e-3) / 1e12
    mfma_peak = MFMA_F32_PEAK_TFLOPS if store == "f32" else MFMA_BF16_PEAK_TFLOPS
    if flops_alg / bytes_alg < mfma_peak * 1e12 / (HBM_PEAK_GBS * 1e9):
        r = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(hbm_gbs / HBM_PEAK_GBS, 4)}
    else:
        r = {"bound": "mfma", "achieved": round(tflops, 2), "peak": mfma_peak, "unit": "TFLOP/s",
             "frac": round(tflops / mfma_peak, 4)}
    r["alg_bytes_per_launch"] = int(bytes_alg)
    r["alg_flops_per_launch"] = int(flops_alg)
    return r


def mfma_used(T, vrs, B, pred, k, metric, strategy, tile):
    _, _, t = T.plan(B, pred, k, metric, strategy=strategy, tile=tile)
    return vrs.num_tiles() > t >= 4


# ---------------------------------------------------------------- scan form
def bench_scan(args):
    import torch

    from paper_2403_15807_amd import inputs, vrs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    metric = vrs.L2SQ if args.metric == "l2" else vrs.IP
    strategy = {"auto": vrs.STRATEGY_AUTO, "mask": vrs.STRATEGY_MASK, "gather": vrs.STRATEGY_GATHER}[args.strategy]
    n = args.n or 10_000_000
    d = args.d or 128
    B = args.batch or 1
    cfg_id = args.cfg if args.cfg >= 0 else (1 if args.store == "f32" else 2)
    t0 = time.time()
    x = inputs.table(cfg_id, n, d, args.clusters)
    attr = inputs.attributes(cfg_id, n, 2, ATTR)
    q = inputs.queries(cfg_id, B, d, args.clusters)
    w = inputs.two_term_width(args.sel, ATTR)
    pred = [(0, 0, w), (1, 0, w)]
    log(f"generated {n}x{d} in {time.time() - t0:.1f}s")

    xd = torch.from_numpy(x).to(dev)
    ad = torch.from_numpy(attr).to(dev)
    t0 = time.time()
    store = {"f32": vrs.F32, "bf16": vrs.BF16, "fp8": vrs.FP8E4M3}[args.store]
    T = vrs.Table(xd, ad, store=store, normalize=(metric == vrs.IP))
    T_other = None
    if args.sweep and args.store == "f32":
        # the sweep's other metric (IP on L2-normalised rows, or L2 on raw rows)
        T_other = vrs.Table(xd, ad, store=store, normalize=(metric != vrs.IP))
    torch.cuda.synchronize()
    log(f"table(s) built in {time.time() - t0:.2f}s")
    del xd
    torch.cuda.empty_cache()
    n_sel = int(T.select(pred).numel())
    realized = n_sel / n
    qd = torch.from_numpy(q).to(dev)
    k = args.k
    idx = torch.empty((B, k), dtype=torch.int64, device=dev)
    dist = torch.empty((B, k), dtype=torch.float32, device=dev)
    nv = torch.empty(B, dtype=torch.int32, device=dev)
    cert = torch.empty(B, dtype=torch.uint8, device=dev)
    o = vrs.vrs_opts()
    o.strategy, o.tile = strategy, args.tile
    ws = T.workspace(B, k, o)
    out = (idx, dist, nv, cert)

    def step():
        T.scan_topk(qd, pred, k, metric, strategy=strategy, tile=args.tile, ws=ws, out=out, passes=args.passes)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    elapsed, stages = timed_then_profiled(step, args.steps, torch, vrs)
    log(f"timed {args.steps} steps in {elapsed:.3f}s")
    ms_step = elapsed * 1e3 / args.steps
    qps = B * args.steps / elapsed
    certified = float(cert.float().mean().item())
    diag = diagnostics(T, qd, pred, k, metric, strategy, args.tile, ws, args.passes, idx, torch)
    # end to end: the call plus the copy of its results to host memory
    e2e = []
    for _ in range(min(args.steps, 10)):
        t1 = time.perf_counter()
        step()
        idx.cpu(), dist.cpu()
        e2e.append(time.perf_counter() - t1)
    diag["end_to_end_ms_with_d2h"] = round(float(np.median(e2e)) * 1e3, 4)

    used_gather = stages["select"][1] > 0
    used_mfma = mfma_used(T, vrs, B, pred, k, metric, strategy, args.tile)
    screen_ms = stages["screen"][0] / max(1, stages["screen"][1])
    launches = max(1, round(stages["screen"][1] / args.steps))
    roof = roofline(n_sel, n, d, B, args.store, used_gather, len(pred), screen_ms, launches)
    roof["launches_per_step"] = launches
    kname = screen_kernel_name(args.store, used_mfma)
    wkey = f"scan-{n}x{d}-{args.store}-{args.metric}-b{B}-s{args.sel:g}-k{k}-{'gather' if used_gather else 'mask'}"
    tb = traffic_from_profiles(kname, wkey)
    roof["traffic"] = tb
    roof["kernel"] = kname
    roof["kernel_ms"] = round(screen_ms, 4)
    roof["traffic_key"] = wkey

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {args.copy_calibration} MiB")
        del src, dst

    sweep = sweep_check = None
    if args.sweep:
        sweep, checks = run_sweep(args, T, T_other, n, d, metric, vrs, torch, dev)
        if not args.no_cpu:
            sweep_check = sweep_oracle_check(args, x, attr, checks, metric, vrs)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_scan(args, x, attr, q, pred, k, metric, B, idx, vrs)

    precision = None
    if args.recall and args.store != "f32":
        precision = precision_report(args, x, attr, q, pred, k, metric, B, idx, dist, vrs)

    rec = {
        "metric": "filtered exact top-k queries/s (N=10M,d=128)",
        "value": round(qps, 2),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.store,
        "data": "synthetic",
        "config": {"workload": f"clustered-gaussian N={n} d={d} {args.store} top-{k} {args.metric}",
                   "batch": B, "selectivity_target": args.sel, "selectivity": round(realized, 6),
                   "strategy": "gather" if used_gather else "mask", "k": k},
        "roofline": roof,
        "cpu_baseline": cpu,
        "stages_ms_per_step": {s: round(v[0] / max(1, args.steps), 4) for s, v in stages.items()},
        "stages_note": "per-stage HIP events, from a second pass of the same steps; the timed pass runs without them",
        "certified_frac": certified,
        "fallback_rate": round(1.0 - certified, 6),
        "diagnostics": diag,
    }
    if sweep is not None:
        rec["sweep"] = sweep
        rec["sweep_check"] = sweep_check
    if precision is not None:
        rec["precision"] = precision
    print(json.dumps(rec), flush=True)


def diagnostics(T, qd, pred, k, metric, strategy, tile, ws, passes, idx, torch):
    """One untimed call with the screening-error diagnostic: the largest
    |screening - exact| / bound over every reranked key of every query, the
    certified fraction, and that the result equals the timed calls' one."""
    r = T.scan_topk(qd, pred, k, metric, strategy=strategy, tile=tile, ws=ws, passes=passes, diag=True)
    torch.cuda.synchronize()
    return {"err_ratio_max": float(r.err_ratio.max().item()),
            "certified_frac": float(r.certified.float().mean().item()),
            "same_ids_as_timed": bool(torch.equal(r.idx, idx))}


def run_sweep(args, T, T_other, n, d, metric, vrs, torch, dev):
    """The workload's grid, each point warmup 1 + 3 timed calls."""
    from paper_2403_15807_amd import inputs
    points = []
    sels = [1e-4, 1e-3, 1e-2, 0.1, 0.5, 1.0]
    batches = [1, 16, 128, 1024]
    tables = [(args.metric, T, metric)]
    if T_other is not None:
        om = "ip" if metric == vrs.L2SQ else "l2"
        tables.append((om, T_other, vrs.IP if metric == vrs.L2SQ else vrs.L2SQ))
    qs_h = {B: inputs.queries(1, B, d, args.clusters, stream_offset=7) for B in batches}
    qs = {B: torch.from_numpy(v).to(dev) for B, v in qs_h.items()}
    checks = []  # (metric name, query, predicate, ids) for the oracle
    t_start = time.time()
    for mname, TT, mm in tables:
        for B in batches:
            for s in sels:
                w = inputs.two_term_width(s, ATTR)
                pred = [(0, 0, w), (1, 0, w)]
                n_sel = int(TT.select(pred).numel())
                strategies = [("mask", vrs.STRATEGY_MASK), ("gather", vrs.STRATEGY_GATHER)]
                if mname != args.metric:
                    strategies = [("auto", vrs.STRATEGY_AUTO)]
                ids_first = None
                for sname, st in strategies:
                    o = vrs.vrs_opts()
                    o.strategy, o.tile = st, -1
                    ws = TT.workspace(B, args.k, o)
                    res = TT.scan_topk(qs[B], pred, args.k, mm, strategy=st, ws=ws)
                    torch.cuda.synchronize()
                    ids = res.idx.cpu().numpy()
                    if ids_first is None:
                        ids_first = ids
                        checks.append((mname, qs_h[B][0], pred, ids[0]))
                    elif not np.array_equal(ids, ids_first):
                        raise SystemExit(f"sweep: {sname} ids differ from mask at B={B} sel={s} {mname}")
                    reps = 3
                    el, stg = timed_then_profiled(
                        lambda: TT.scan_topk(qs[B], pred, args.k, mm, strategy=st, ws=ws), reps, torch, vrs)
                    gather = stg["select"][1] > 0
                    sms = stg["screen"][0] / max(1, stg["screen"][1])
                    nl = max(1, round(stg["screen"][1] / reps))
                    r = roofline(n_sel, n, d, B, args.store, gather, 2, sms, nl)
                    points.append({"metric": mname, "batch": B, "sel": s, "strategy": sname,
                                   "used": "gather" if gather else "mask",
                                   "qps": round(B * reps / el, 1), "ms": round(el * 1e3 / reps, 4),
                                   "screen_ms": round(sms * nl, 4), "passes": nl,
                                   "bound": r["bound"], "frac": r["frac"]})
    log(f"sweep: {len(points)} points in {time.time() - t_start:.1f}s (mask and gather ids equal at every point)")
    return points, checks


def sweep_oracle_check(args, x, attr, checks, metric, vrs):
    """Query 0 of every sweep point against the FP64 oracle (one call per
    metric, each query with its point's predicate)."""
    import oracle as O
    cores = len(os.sched_getaffinity(0))
    ok, t0 = 0, time.perf_counter()
    for mname in sorted(set(c[0] for c in checks)):
        cs = [c for c in checks if c[0] == mname]
        ot = O.Table.build(x, attr, O.F32, normalize=(mname == "ip"))
        q = np.stack([c[1] for c in cs])
        ref = O.scan_topk(ot, q, [c[2] for c in cs], args.k, O.IP if mname == "ip" else O.L2SQ, nthreads=cores)
        ok += sum(bool(np.array_equal(ref[0][i], c[3])) for i, c in enumerate(cs))
        del ot
    log(f"sweep oracle check: {ok}/{len(checks)} points match in {time.perf_counter() - t0:.1f}s")
    return {"points_checked": len(checks), "points_matching_oracle": ok,
            "what": "query 0 of every sweep point against the FP64 oracle; mask and gather ids equal at every point"}


def cpu_baseline_scan(args, x, attr, q, pred, k, metric, B, idx, vrs):
    import oracle as O
    cores = len(os.sched_getaffinity(0))
    nq = args.cpu_queries or min(3 * cores, 48)  # about 10-20 s of oracle work
    ot = O.Table.build(x, attr, {"f32": O.F32, "bf16": O.BF16, "fp8": O.FP8}[args.store],
                       normalize=(metric == vrs.IP))
    qs = np.ascontiguousarray(q[np.arange(nq) % B])
    log(f"oracle: {nq} queries on {cores} cores")
    t0 = time.perf_counter()
    ref = O.scan_topk(ot, qs, pred, k, O.L2SQ if metric == vrs.L2SQ else O.IP, nthreads=cores)
    cpu_s = time.perf_counter() - t0
    cpu = {"value": round(nq / cpu_s, 3), "unit": "queries/s", "cores": min(cores, nq), "kind": "oracle",
           "sample": f"{nq} queries of the same workload (full {x.shape[0]}-row table), FP64, {cpu_s:.1f}s wall"}
    gi = idx.cpu().numpy()
    same = all(np.array_equal(ref[0][i], gi[i % B]) for i in range(min(nq, B)))
    cpu["gpu_ids_match_oracle"] = bool(same)
    log(f"oracle done in {cpu_s:.1f}s, ids match: {same}")
    return cpu


def precision_report(args, x, attr, q, pred, k, metric, B, idx, dist, vrs):
    import oracle as O
    cores = len(os.sched_getaffinity(0))
    nq = min(B, args.cpu_queries or cores)
    qs = np.ascontiguousarray(q[:nq])
    mo = O.L2SQ if metric == vrs.L2SQ else O.IP
    t_r = O.Table.build(x, attr, O.F32, normalize=(metric == vrs.IP))
    r2 = O.scan_topk(t_r, qs, pred, k, mo, nthreads=cores)
    gi = idx.cpu().numpy()[:nq]
    gd = dist.cpu().numpy()[:nq].astype(np.float64)
    recall = float(np.mean([len(set(gi[i][gi[i] >= 0]) & set(r2[0][i][r2[0][i] >= 0])) /
                            max(1, int((r2[0][i] >= 0).sum())) for i in range(nq)]))
    fin = np.isfinite(r2[2]) & np.isfinite(gd)
    maxerr = float(np.max(np.abs(gd[fin] - r2[2][fin]))) if fin.any() else 0.0
    log(f"recall@{k} vs float32 rows: {recall:.4f}, max |dist err| {maxerr:.3g}")
    return {"queries": nq, "recall_at_k_vs_fp32_rows": round(recall, 4),
            "max_abs_dist_error_vs_fp32_rows": maxerr,
            "note": "ids are exact for the stored rows; this compares with the float32 rows"}


# ------------------------------------------------------------- batched form
def bench_batched(args):
    import torch

    import oracle as O
    from paper_2403_15807_amd import inputs, vrs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n = args.n or 2_000_000
    d = args.d or 1536
    B = args.batch or 4096
    store = {"f32": vrs.F32, "bf16": vrs.BF16, "fp8": vrs.FP8E4M3}[args.store if args.store != "f32" else "bf16"]
    sname = {vrs.BF16: "bf16", vrs.FP8E4M3: "fp8"}[store]
    t0 = time.time()
    x = inputs.table(3, n, d, 1000)
    attr = inputs.attributes(3, n, 2, ATTR)
    q = inputs.queries(3, B, d, 1000)
    bp = inputs.batched_predicates(3, B, ATTR)
    preds = [[(0, int(bp.lo[b, 0]), int(bp.hi[b, 0])), (1, int(bp.lo[b, 1]), int(bp.hi[b, 1]))]
             for b in range(B)]
    log(f"generated {n}x{d} and {B} predicates in {time.time() - t0:.1f}s")
    T = vrs.Table(torch.from_numpy(x).to(dev), torch.from_numpy(attr).to(dev), store=store, normalize=True)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    qd = torch.from_numpy(q).to(dev)
    pd = vrs.preds_tensor(preds)
    kd = torch.from_numpy(bp.k).to(dev)
    kmax = int(bp.k.max())
    # qualifying rows per query (for the useful-work rate)
    sel_rows = np.array([int(T.select(p).numel()) for p in preds], dtype=np.int64)
    log(f"selectivity: mean {sel_rows.mean() / n:.4f}, median {np.median(sel_rows) / n:.5f}")

    out = (torch.empty((B, kmax), dtype=torch.int64, device=dev),
           torch.empty((B, kmax), dtype=torch.float32, device=dev),
           torch.empty(B, dtype=torch.int32, device=dev), torch.empty(B, dtype=torch.uint8, device=dev))
    ws = torch.empty(T.batched_workspace_bytes(B, kmax, vrs.IP), dtype=torch.uint8, device=dev)
    t0 = time.time()
    best, cfg_ms, _ = T.batched_tune(qd, pd, kd, kmax, vrs.IP, ws=ws, out=out, kprime_mult=args.kprime_mult)
    log(f"autotuned in {time.time() - t0:.1f}s: config {best}, ms {['%.2f' % m for m in cfg_ms]}")
    G = T.batched_graph(qd, pd, kd, kmax, vrs.IP, tile=best, ws=ws, out=out, kprime_mult=args.kprime_mult)
    for _ in range(args.warmup):
        G.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        G.launch()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    qps = B * args.steps / elapsed
    ms_step = elapsed * 1e3 / args.steps
    log(f"graph: {ms_step:.3f} ms per batch, {qps:.0f} queries/s")

    # stage split (eager run of the same configuration, events per stage)
    vrs.stage_times()
    vrs.profile(True)
    for _ in range(3):
        T.scan_topk_batched(qd, pd, kd, kmax, vrs.IP, tile=best, ws=ws, out=out, kprime_mult=args.kprime_mult)
    torch.cuda.synchronize()
    vrs.profile(False)
    stages = vrs.stage_times()
    # the screening stage of one batch (dense and sparse kernels, both passes)
    screen_ms = stages["screen"][0] / 3
    launches = max(1, round(stages["screen"][1] / 3))
    pair_flops = 2.0 * d * float(sel_rows.sum())
    tf = pair_flops / (screen_ms * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": round(tf, 2), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None, "kernel": "screen (dense + sparse)",
            "kernel_ms": round(screen_ms / launches, 4), "launches_per_step": launches,
            "screen_ms_per_batch": round(screen_ms, 4), "alg_flops_per_batch": int(pair_flops),
            "note": "algorithmic work = 2 d per qualifying (query, row) pair, over the batch's screening time"}
    rd = T.scan_topk_batched(qd, pd, kd, kmax, vrs.IP, tile=best, ws=ws, diag=True, kprime_mult=args.kprime_mult)
    torch.cuda.synchronize()
    cert_b = rd.certified.cpu().numpy()
    sfrac = sel_rows / n
    diag = {"err_ratio_max": float(rd.err_ratio.max().item()),
            "certified_frac": float(cert_b.mean()),
            "same_ids_as_graph": bool(torch.equal(rd.idx, out[0])),
            "fallbacks_by_k": {int(kk): [int((bp.k == kk).sum()), int(((bp.k == kk) & (cert_b == 0)).sum())]
                               for kk in np.unique(bp.k)},
            "fallbacks_by_selectivity_decade": {
                f"{lo:g}-{lo * 10:g}": [int(((sfrac >= lo) & (sfrac < lo * 10)).sum()),
                                         int(((sfrac >= lo) & (sfrac < lo * 10) & (cert_b == 0)).sum())]
                for lo in (1e-5, 1e-4, 1e-3, 1e-2, 1e-1)}}

    # the plain path, one launch per query (own predicate and k), on a sample
    m = min(B, args.per_query_sample)
    for b in range(2):
        T.scan_topk(qd[b:b + 1], preds[b], int(bp.k[b]), vrs.IP)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(m):
        T.scan_topk(qd[b:b + 1], preds[b], int(bp.k[b]), vrs.IP)
    torch.cuda.synchronize()
    pq_qps = m / (time.perf_counter() - t0)
    log(f"per-query launches: {pq_qps:.1f} queries/s on {m} queries")

    cpu = None
    if not args.no_cpu:
        cores = len(os.sched_getaffinity(0))
        nq = args.cpu_queries or min(cores, 16)
        ot = O.Table.build(x, attr, O.BF16 if store == vrs.BF16 else O.FP8, normalize=True)
        rows = np.arange(nq)
        t0 = time.perf_counter()
        ref = O.scan_topk(ot, q[rows], [preds[i] for i in rows], bp.k[rows], O.IP, nthreads=cores, out_stride=kmax)
        cpu_s = time.perf_counter() - t0
        gi = out[0].cpu().numpy()[rows]
        cpu = {"value": round(nq / cpu_s, 3), "unit": "queries/s", "cores": min(cores, nq), "kind": "oracle",
               "sample": f"first {nq} queries of the batch with their own predicates and k, FP64, {cpu_s:.1f}s wall",
               "gpu_ids_match_oracle": bool(np.array_equal(gi, ref[0]))}
        log(f"oracle {cpu_s:.1f}s, ids match {cpu['gpu_ids_match_oracle']}")

    rec = {
        "metric": "filtered exact top-k queries/s (batched uneven form)",
        "value": round(qps, 2), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": sname, "data": "synthetic",
        "config": {"workload": f"clustered-gaussian N={n} d={d} {sname} normalised, {B} queries with own "
                               f"2-term range predicates (sel logU[1e-4,1]) and k in {{1,10,100}}, IP",
                   "batch": B, "autotuned_config": best, "config_ms": [round(v, 3) for v in cfg_ms]},
        "roofline": roof,
        "per_query_launches_qps": round(pq_qps, 2),
        "speedup_vs_per_query_launches": round(qps / pq_qps, 2),
        "cpu_baseline": cpu,
        "fallback_rate": round(1.0 - diag["certified_frac"], 6),
        "diagnostics": diag,
        "stages_ms_per_step": {s: round(v[0] / 3, 4) for s, v in stages.items()},
    }
    print(json.dumps(rec), flush=True)

# ----------------------------------------------------------- precision form
def bench_precision(args):
    """4M x 768 normalised rows stored as float32, bfloat16 and FP8 e4m3 with
    row scales; 256 queries per call; IP top-k for k in {10, 100} at
    selectivity 1% and 30%.  The float32 form's ids equal the FP64 oracle on
    the float32 rows (checked on sampled queries); the bf16 / FP8 forms' ids
    are exact for their stored rows and are reported against the float32
    form: recall@k, and the largest |returned distance - FP64 distance of the
    same row on the float32 rows|."""
    import torch

    import oracle as O
    from paper_2403_15807_amd import inputs, vrs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n, d, B = args.n or 4_000_000, args.d or 768, args.batch or 256
    t0 = time.time()
    x = inputs.table(2, n, d, 2000)
    attr = inputs.attributes(2, n, 2, ATTR)
    q = inputs.queries(2, B, d, 2000)
    log(f"generated {n}x{d} in {time.time() - t0:.1f}s")
    xd, ad = torch.from_numpy(x).to(dev), torch.from_numpy(attr).to(dev)
    tables = {name: vrs.Table(xd, ad, store=st, normalize=True)
              for name, st in (("f32", vrs.F32), ("bf16", vrs.BF16), ("fp8", vrs.FP8E4M3))}
    del xd
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    qd = torch.from_numpy(q).to(dev)
    cores = len(os.sched_getaffinity(0))
    ot = O.Table.build(x, attr, O.F32, normalize=True)  # the float32 rows (R2)
    rows = np.arange(min(B, args.cpu_queries or cores))
    results, head = [], None
    for sel, k in ((0.01, 10), (0.01, 100), (0.3, 10), (0.3, 100)):
        w = inputs.two_term_width(sel, ATTR)
        pred = [(0, 0, w), (1, 0, w)]
        n_sel = int(tables["f32"].select(pred).numel())
        ref_ids = ref_d = None
        for name in ("f32", "bf16", "fp8"):
            T = tables[name]
            o = vrs.vrs_opts()
            ws = T.workspace(B, k, o)
            r = T.scan_topk(qd, pred, k, vrs.IP, ws=ws)
            torch.cuda.synchronize()
            el, stg = timed_then_profiled(lambda: T.scan_topk(qd, pred, k, vrs.IP, ws=ws), args.steps, torch, vrs)
            rd = T.scan_topk(qd, pred, k, vrs.IP, ws=ws, diag=True)
            torch.cuda.synchronize()
            ids, dist = rd.idx.cpu().numpy(), rd.dist.cpu().numpy().astype(np.float64)
            gather = stg["select"][1] > 0
            sms = stg["screen"][0] / max(1, stg["screen"][1])
            nl = max(1, round(stg["screen"][1] / args.steps))
            roof = roofline(n_sel, n, d, B, name, gather, 2, sms, nl)
            e = {"store": name, "sel": sel, "k": k, "qps": round(B * args.steps / el, 1),
                 "ms": round(el * 1e3 / args.steps, 4), "screen_ms": round(sms * nl, 4),
                 "strategy": "gather" if gather else "mask", "bound": roof["bound"], "frac": roof["frac"],
                 "certified_frac": float(rd.certified.float().mean().item()),
                 "err_ratio_max": float(rd.err_ratio.max().item())}
            if name == "f32":
                ref_ids, ref_d = ids, dist
                orc = O.scan_topk(ot, q[rows], pred, k, O.IP, nthreads=cores)
                e["ids_match_fp64_oracle_on_sample"] = bool(np.array_equal(orc[0], ids[rows]))
                e["oracle_sample"] = int(rows.size)
            else:
                rec_ = [len(set(ids[b][ids[b] >= 0]) & set(ref_ids[b][ref_ids[b] >= 0])) /
                        max(1, int((ref_ids[b] >= 0).sum())) for b in range(B)]
                err = 0.0
                for b in range(B):
                    v = ids[b] >= 0
                    if v.any():
                        d64 = O.distances(ot, q[b], ids[b][v], O.IP)
                        err = max(err, float(np.max(np.abs(dist[b][v] - d64))))
                e["recall_at_k_vs_fp32_form"] = round(float(np.mean(rec_)), 4)
                e["max_abs_dist_error_vs_fp64_on_fp32_rows"] = err
            results.append(e)
            log(json.dumps(e))
            if name == "bf16" and sel == 0.3 and k == 100:
                head = (e, roof)
    e, roof = head
    kname = "screen_mfma_bf16"
    wkey = f"scan-{n}x{d}-bf16-ip-b{B}-s0.3-k100-{e['strategy']}"
    roof["traffic"] = traffic_from_profiles(kname, wkey)
    roof["kernel"] = kname
    roof["traffic_key"] = wkey
    rec = {
        "metric": "filtered exact top-k queries/s (precision form)",
        "value": e["qps"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": e["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"clustered-gaussian N={n} d={d} normalised, stored f32 / bf16 / fp8, "
                               f"IP, batch {B}, k in {{10, 100}}, selectivity 1% and 30%; value = bf16, 30%, k=100",
                   "batch": B},
        "roofline": roof,
        "precision": results,
        "note": "ids of every form are exact for its stored rows; recall and distance error compare the "
                "bf16/fp8 forms with the float32 form (= FP64 oracle on the float32 rows)",
    }
    print(json.dumps(rec), flush=True)


# ------------------------------------------------------- threshold selection
def bench_range(args):
    """Threshold selection on the 10M x 128 table: cosine similarity > t (IP
    distance < -t on L2-normalised rows and queries), the evaluation's
    similarity predicate of the paper (Section 5), with the two-term range
    predicate of the requested selectivity."""
    import torch

    import oracle as O
    from paper_2403_15807_amd import inputs, vrs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n, d, B = args.n or 10_000_000, args.d or 128, args.batch or 1
    t0 = time.time()
    x = inputs.table(1, n, d, args.clusters)
    attr = inputs.attributes(1, n, 2, ATTR)
    q = inputs.queries(1, B, d, args.clusters, stream_offset=3)
    q = (q / np.linalg.norm(q.astype(np.float64), axis=1, keepdims=True)).astype(np.float32)
    log(f"generated {n}x{d} in {time.time() - t0:.1f}s")
    T = vrs.Table(torch.from_numpy(x).to(dev), torch.from_numpy(attr).to(dev), normalize=True)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    qd = torch.from_numpy(q).to(dev)
    thr = -args.cos
    w = inputs.two_term_width(args.sel, ATTR)
    pred = [(0, 0, w), (1, 0, w)]
    n_sel = int(T.select(pred).numel())
    cap = args.cap
    ws = torch.empty(T.range_workspace_bytes(B, cap), dtype=torch.uint8, device=dev)
    out = (torch.empty((B, cap), dtype=torch.int64, device=dev), torch.empty((B, cap), dtype=torch.float32, device=dev),
           torch.empty(B, dtype=torch.int64, device=dev))
    strategy = {"auto": vrs.STRATEGY_AUTO, "mask": vrs.STRATEGY_MASK, "gather": vrs.STRATEGY_GATHER}[args.strategy]

    def step():
        T.scan_range(qd, pred, thr, cap, vrs.IP, strategy=strategy, ws=ws, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    el, stages = timed_then_profiled(step, args.steps, torch, vrs)
    gather = stages["select"][1] > 0
    screen_ms = stages["screen"][0] / max(1, stages["screen"][1])
    roof = roofline(n_sel, n, d, B, "f32", gather, 2, screen_ms)
    roof["kernel"] = "range_screen"
    roof["kernel_ms"] = round(screen_ms, 4)
    wkey = f"range-{n}x{d}-f32-ip-b{B}-s{args.sel:g}-cos{args.cos:g}-{'gather' if gather else 'mask'}"
    roof["traffic"] = traffic_from_profiles("range_screen", wkey)
    roof["traffic_key"] = wkey
    counts = out[2].cpu().numpy()
    cpu = None
    if not args.no_cpu:
        cores = len(os.sched_getaffinity(0))
        nq = min(B, args.cpu_queries or cores)
        ot = O.Table.build(x, attr, O.F32, normalize=True)
        reps = max(1, (args.cpu_queries or cores) // nq)
        qs = np.ascontiguousarray(np.tile(q[:nq], (reps, 1)))
        t0 = time.perf_counter()
        ref = O.scan_range(ot, qs, pred, thr, cap, O.IP, nthreads=cores)
        cpu_s = time.perf_counter() - t0
        gi = out[0].cpu().numpy()
        same = bool(np.array_equal(ref[0][:nq], gi[:nq]) and np.array_equal(ref[3][:nq], counts[:nq]))
        cpu = {"value": round(qs.shape[0] / cpu_s, 3), "unit": "queries/s", "cores": min(cores, qs.shape[0]),
               "kind": "oracle", "sample": f"{qs.shape[0]} queries of the same workload, FP64, {cpu_s:.1f}s wall",
               "gpu_ids_match_oracle": same}
        log(f"oracle {cpu_s:.1f}s, ids match {same}")
    rec = {
        "metric": "threshold selection queries/s (cosine > t, N=10M, d=128)",
        "value": round(B * args.steps / el, 2), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(el * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"clustered-gaussian N={n} d={d} f32 normalised, cosine > {args.cos}, "
                               f"2-term predicate selectivity {args.sel:g}", "batch": B, "cap": cap,
                   "strategy": "gather" if gather else "mask", "selectivity": round(n_sel / n, 6)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "selected_rows_per_query": [int(c) for c in counts[:8]],
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
    }
    print(json.dumps(rec), flush=True)


# --------------------------------------------------------------- vector join
def bench_join(args):
    """kNN join: the first R rows of the 10M x 128 table, each as a query,
    against the whole table (squared L2, top-k)."""
    import torch

    import oracle as O
    from paper_2403_15807_amd import inputs, vrs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n, d, nr, k = args.n or 10_000_000, args.d or 128, args.join_rows, args.k
    x = inputs.table(1, n, d, args.clusters)
    attr = inputs.attributes(1, n, 2, ATTR)
    S = vrs.Table(torch.from_numpy(x).to(dev), torch.from_numpy(attr).to(dev))
    R = S.view(nr)
    torch.cuda.synchronize()
    w = inputs.two_term_width(args.sel, ATTR)
    pred = [(0, 0, w), (1, 0, w)]
    n_sel = int(S.select(pred).numel())
    ws = torch.empty(R.join_workspace_bytes(S, k), dtype=torch.uint8, device=dev)
    r = R.join_topk(S, pred, k, vrs.L2SQ, ws=ws)
    torch.cuda.synchronize()
    args.steps = min(args.steps, 10)  # (a join takes about half a second)
    el, stages = timed_then_profiled(lambda: R.join_topk(S, pred, k, vrs.L2SQ, ws=ws), args.steps, torch, vrs)
    r = R.join_topk(S, pred, k, vrs.L2SQ, ws=ws)
    screen_ms = stages["screen"][0] / max(1, stages["screen"][1])
    launches = max(1, round(stages["screen"][1] / args.steps))
    batches = (nr + 8191) // 8192
    flops = 2.0 * nr * n_sel * d
    tf = flops / (stages["screen"][0] / args.steps * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": round(tf, 2), "peak": MFMA_F32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / MFMA_F32_PEAK_TFLOPS, 4), "traffic": None, "kernel": "screen_mfma_f32",
            "kernel_ms": round(screen_ms, 4), "launches_per_step": launches,
            "note": "2 d flops per (R row, qualifying S row), over the step's screening time"}
    cpu = None
    if not args.no_cpu:
        cores = len(os.sched_getaffinity(0))
        nq = args.cpu_queries or cores
        ot = O.Table(O.F32, x, attr)
        rows = np.linspace(0, nr - 1, nq).astype(int)
        t0 = time.perf_counter()
        ref = O.scan_topk(ot, x[rows], pred, k, O.L2SQ, nthreads=cores)
        cpu_s = time.perf_counter() - t0
        same = bool(np.array_equal(ref[0], r.idx.cpu().numpy()[rows]))
        cpu = {"value": round(nq / cpu_s, 3), "unit": "R rows/s", "cores": min(cores, nq), "kind": "oracle",
               "sample": f"{nq} rows of R against the full table, FP64, {cpu_s:.1f}s wall",
               "gpu_ids_match_oracle": same}
        log(f"oracle {cpu_s:.1f}s, ids match {same}")
    rec = {
        "metric": "vector join R rows/s (kNN join against N=10M, d=128)",
        "value": round(nr * args.steps / el, 2), "unit": "R rows/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": round(el * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"first {nr} rows of a clustered-gaussian N={n} d={d} f32 table joined with the "
                               f"whole table, squared L2, top-{k}, 2-term predicate selectivity {args.sel:g}",
                   "batches_of_R": batches},
        "roofline": roof,
        "cpu_baseline": cpu,
        "stages_ms_per_step": {kk: round(v[0] / args.steps, 4) for kk, v in stages.items()},
    }
    print(json.dumps(rec), flush=True)


# ----------------------------------------------------------- probe vs scan
def bench_probe(args):
    """Scan vs probe (Section 5.3's question, Figs. 7-8): the 10M x 128 table
    with one attribute, a one-column range predicate of selectivity 1e-4..1,
    top-k; the exact scan
    (the planner's mask or gather) against the filtered probe of a k-means
    partition index (nprobe nearest partitions, walk extended until k rows
    qualify), at one query and at a batch; recall of the probe against the
    scan's exact answer."""
    import torch

    from paper_2403_15807_amd import inputs, vrs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n, d, k = args.n or 10_000_000, args.d or 128, args.k
    nlist = args.nlist
    nprobes = [int(v) for v in str(args.nprobe).split(",")]
    x = inputs.table(10, n, d, args.clusters)
    attr = inputs.attributes(10, n, 1, ATTR)
    T = vrs.Table(torch.from_numpy(x).to(dev), torch.from_numpy(attr).to(dev))
    torch.cuda.synchronize()
    t0 = time.time()
    ix = vrs.Index(T, nlist, iters=args.iters)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log(f"index: {nlist} partitions, {args.iters} iterations in {build_s:.2f}s, largest {ix.max_list}")
    cent, off, _ = [t.cpu().numpy() for t in ix.export()]
    sizes = np.diff(off)
    size_biased = float((sizes.astype(np.float64) ** 2).sum() / n)

    def visited_rows(qh, taken):
        # rows in the partitions each query visited (its nearest centroids, FP64)
        dd = ((qh.astype(np.float64)[:, None, :] - cent.astype(np.float64)[None]) ** 2).sum(-1)
        order = np.argsort(dd, axis=1, kind="stable")
        return float(np.mean([sizes[order[b, :taken[b]]].sum() for b in range(qh.shape[0])]))

    def timed(fn, reps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) / reps * 1e3

    points = []
    for B in (1, 16, args.probe_batch):
        qh = inputs.queries(10, B, d, args.clusters)
        q = torch.from_numpy(qh).to(dev)
        for sel in (1e-4, 1e-3, 1e-2, 0.1, 0.5, 1.0):
            pred = [(0, 0, max(1, int(round(sel * ATTR))))]
            ex = T.scan_topk(q, pred, k, vrs.L2SQ)
            o = vrs.vrs_opts()
            sws = T.workspace(B, k, o)
            scan_ms = timed(lambda: T.scan_topk(q, pred, k, vrs.L2SQ, ws=sws), args.steps)
            ei = ex.idx.cpu().numpy()
            for nprobe in nprobes:
                ws = torch.empty(ix.workspace_bytes(B, k, nprobe, args.cap_c), dtype=torch.uint8, device=dev)
                pr = ix.probe_topk(q, pred, k, vrs.L2SQ, nprobe, k, args.cap_c, ws=ws)
                torch.cuda.synchronize()
                probe_ms = timed(lambda: ix.probe_topk(q, pred, k, vrs.L2SQ, nprobe, k, args.cap_c, ws=ws,
                                                       out=pr), args.steps)
                pi = pr[0].cpu().numpy()
                taken = pr[2].cpu().numpy()
                rec = float(np.mean([len(set(pi[b][pi[b] >= 0]) & set(ei[b][ei[b] >= 0])) /
                                     max(1, int((ei[b] >= 0).sum())) for b in range(B)]))
                est_scan, est_probe, use_probe = ix.plan_access(B, pred, k, nprobe, args.cap_c)
                chosen = probe_ms if use_probe else scan_ms
                points.append({"batch": B, "sel": sel, "nprobe": nprobe, "scan_ms": round(scan_ms, 4),
                               "probe_ms": round(probe_ms, 4), "probe_recall": round(rec, 4),
                               "partitions_visited_mean": round(float(taken.mean()), 2),
                               "rows_visited_mean": round(visited_rows(qh, taken)),
                               "faster": "probe" if probe_ms < scan_ms else "scan",
                               "model_scan_ms": round(est_scan, 4), "model_probe_ms": round(est_probe, 4),
                               "model_pick": "probe" if use_probe else "scan",
                               "model_regret": round(chosen / min(scan_ms, probe_ms) - 1.0, 4)})
                log(json.dumps(points[-1]))
    head = [p for p in points if p["batch"] == 1 and p["sel"] == 1.0 and p["nprobe"] == nprobes[0]][0]
    rec = {
        "metric": f"filtered top-k queries/s, probe path (k-means partitions) vs exact scan (N={n})",
        "value": round(1e3 / head["probe_ms"], 2), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": head["probe_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"clustered-gaussian N={n} d={d} f32, one-column range predicate, squared L2, "
                               f"top-{k}; index {nlist} partitions ({args.iters} k-means iterations), probe "
                               f"{nprobes} partitions, more until k rows qualify, at most {args.cap_c} rows",
                   "index_build_s": round(build_s, 3), "largest_partition": ix.max_list,
                   "size_biased_partition": round(size_biased)},
        "points": points,
        "model_picks_faster": f"{sum(p['model_pick'] == p['faster'] for p in points)}/{len(points)}",
        "note": "value = probe queries/s at one query, selectivity 1; the scan is exact, the probe approximate",
    }
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=["scan", "batched", "precision", "range", "join", "probe"],
                    default="scan")
    ap.add_argument("--nlist", type=int, default=1024, help="probe workload: partitions")
    ap.add_argument("--nprobe", default="4,16", help="probe workload: partitions probed (comma list)")
    ap.add_argument("--iters", type=int, default=8, help="probe workload: k-means iterations")
    ap.add_argument("--cap-c", type=int, default=1 << 20, help="probe workload: visited-row budget")
    ap.add_argument("--probe-batch", type=int, default=256, help="probe workload: the batched point")
    ap.add_argument("--cos", type=float, default=0.9, help="range workload: cosine-similarity threshold")
    ap.add_argument("--cap", type=int, default=65536, help="range workload: result slots per query")
    ap.add_argument("--join-rows", type=int, default=16384, help="join workload: rows of R")
    ap.add_argument("--n", type=int, default=0, help="rows (default 10M scan, 2M batched)")
    ap.add_argument("--d", type=int, default=0, help="dimension (default 128 scan, 1536 batched)")
    ap.add_argument("--clusters", type=int, default=1000)
    ap.add_argument("--cfg", type=int, default=-1,
                    help="seed configuration index (default: 1 for float32, 2 for bf16/fp8)")
    ap.add_argument("--batch", type=int, default=0, help="queries per call (default 1 scan, 4096 batched)")
    ap.add_argument("--sel", type=float, default=1.0)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--metric", choices=["l2", "ip"], default="l2")
    ap.add_argument("--store", choices=["f32", "bf16", "fp8"], default="f32")
    ap.add_argument("--recall", action="store_true",
                    help="precision form: recall@k and max distance error of the stored-precision "
                         "result against the FP64 oracle on the float32 rows (sampled queries)")
    ap.add_argument("--strategy", choices=["auto", "mask", "gather"], default="auto")
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--passes", type=int, default=0, choices=[0, 1, 2],
                    help="MFMA screening passes (0 = planner's choice)")
    ap.add_argument("--cpu-queries", type=int, default=0,
                    help="oracle sample size (0 = 3 x #cores, at most 48, for the scan form)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sweep", dest="sweep", action="store_false",
                    help="skip the batch x selectivity x strategy sweep")
    ap.add_argument("--kprime-mult", type=int, default=0,
                    help="batched workload: k' = this times k for every query (0 = the library's rule)")
    ap.add_argument("--per-query-sample", type=int, default=256,
                    help="batched workload: queries timed through per-query launches")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of this many MiB (reference for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the scan shards by rows across GPUs by design, but this build runs on one).",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        bench_batched(args)
    elif args.workload == "precision":
        bench_precision(args)
    elif args.workload == "range":
        bench_range(args)
    elif args.workload == "join":
        bench_join(args)
    elif args.workload == "probe":
        bench_probe(args)
    else:
        bench_scan(args)


if __name__ == "__main__":
    main()
