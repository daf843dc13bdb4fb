"""Learned access-path chooser: timing harness, training, regret evaluation.

Workload-driven access-path selection (the paper's conclusion that the best
scan strategy depends on selectivity, dimensionality and the number of
concurrent queries, Sections 3.2 and 5) is learned from timings the scan
itself produces:

1. ``collect``: for random workloads (``inputs.chooser_workloads``) every
   valid arm (strategy x tile) is timed with HIP events on the scan's
   stream; arms a simple cost model predicts to be hopeless are not run and
   enter the data as censored upper bounds.
2. ``train``: the 6 -> 64 -> 64 -> 16 network is fitted to ln(ms) per arm
   (masked mean squared error, Adam) by the library's own HIP kernels
   (``vrs_mlp_forward/backward/adam``).
3. ``evaluate``: on held-out workloads, the time of the learned pick and of
   the selectivity-threshold heuristic's pick relative to the best arm by
   exhaustive timing (regret = t_pick / t_best - 1).

``python -m paper_2403_15807_amd.chooser --train 1250 --heldout 2000``
writes ``chooser_weights.bin`` (loaded by ``vrs_chooser_load``) and
``chooser_report.json`` next to this file.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import struct
import sys
import time

import numpy as np
import torch

from . import inputs, vrs

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "chooser_weights.bin")
REPORT = os.path.join(HERE, "chooser_report.json")
ATTR_RANGE = 10 ** 6
CFG_TRAIN, CFG_HELDOUT, CFG_TABLES = 40, 41, 42


def log(msg):
    print(f"[chooser] {msg}", file=sys.stderr, flush=True)


class Tables:
    """One library table per (d, dtype) at the largest row count used for d;
    smaller tables are row-prefix views."""

    def __init__(self):
        self.src, self.tab = {}, {}

    def get(self, d, dtype, n):
        if (d, dtype) not in self.tab:
            if d not in self.src:
                n_max = inputs.CHOOSER_MAX_ROWS[d]
                t0 = time.time()
                x = inputs.table(CFG_TABLES + d, n_max, d, 1000)
                a = inputs.attributes(CFG_TABLES + d, n_max, 2, ATTR_RANGE)
                self.src[d] = (torch.from_numpy(x).cuda(), torch.from_numpy(a).cuda())
                del x, a
                log(f"table source d={d} n={n_max} in {time.time() - t0:.1f}s")
            xd, ad = self.src[d]
            self.tab[(d, dtype)] = vrs.Table(xd, ad, store=dtype, normalize=True)
        return self.tab[(d, dtype)].view(n)


def _cost_model(w, strategy, tile):
    """Rough ms estimate used only to skip hopeless arms."""
    kind, qt = (0, [1, 2, 4, 8][tile]) if tile < 4 else (1, 64)
    rows = w.n * (w.sel if strategy == vrs.STRATEGY_GATHER else 1.0)
    bpe = {0: 4, 1: 2, 2: 1}[w.dtype]
    hbm = rows * w.d * bpe * (1 if kind == 1 else max(1, math.ceil(w.b / qt) / 8)) / 6e12
    if kind == 0:
        comp = 2.0 * w.b * rows * w.d / 40e12
    else:
        bpad = math.ceil(w.b / 64) * 64
        comp = 2.0 * bpad * rows * w.d / (70e12 if w.dtype == 0 else 600e12)
    return 1e3 * max(hbm, comp) + 0.1


def _arms():
    nt = vrs.num_tiles()
    return [(s, t) for s in (vrs.STRATEGY_MASK, vrs.STRATEGY_GATHER) for t in range(nt)]


def time_workload(tables, w, reps=2, censor_factor=8.0):
    """ln(ms) per arm (NaN = invalid), a censored flag per arm, and the raw
    planner features of the workload."""
    T = tables.get(w.d, w.dtype, w.n)
    q = torch.from_numpy(inputs.queries(CFG_TABLES + w.d, w.b, w.d, 1000, stream_offset=w.seed % 100000)).cuda()
    width = inputs.two_term_width(w.sel, ATTR_RANGE)
    pred = [(0, 0, width), (1, 0, width)]
    feats, _, _ = T.plan(w.b, pred, w.k, vrs.IP, chooser=vrs.CHOOSER_HEURISTIC)
    arms = _arms()
    nt = vrs.num_tiles()
    y = np.full(2 * nt, np.nan)
    cens = np.zeros(2 * nt, bool)
    order = sorted(range(len(arms)), key=lambda i: _cost_model(w, *arms[i]))
    best = math.inf
    idx = torch.empty((w.b, w.k), dtype=torch.int64, device="cuda")
    dist = torch.empty((w.b, w.k), dtype=torch.float32, device="cuda")
    nv = torch.empty(w.b, dtype=torch.int32, device="cuda")
    cert = torch.empty(w.b, dtype=torch.uint8, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ws = None
    for i in order:
        s, t = arms[i]
        _, s_used, t_used = T.plan(w.b, pred, w.k, vrs.IP, strategy=s, tile=t, chooser=vrs.CHOOSER_HEURISTIC)
        if s_used != s or t_used != t:
            continue  # arm not available for this table / k
        est = _cost_model(w, s, t)
        if est > censor_factor * best:
            y[i], cens[i] = math.log(est), True
            continue
        if ws is None:
            ws = T.workspace(w.b, w.k)
        times = []
        for r in range(reps + 1):
            e0.record()
            T.scan_topk(q, pred, w.k, vrs.IP, strategy=s, tile=t, chooser=vrs.CHOOSER_HEURISTIC,
                        ws=ws, out=(idx, dist, nv, cert))
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            times.append(ms)
            if r == 0 and ms > censor_factor * best and ms > 2.0:
                break
        ms = min(times[1:]) if len(times) > 1 else times[0]
        cens[i] = len(times) == 1
        y[i] = math.log(ms)
        best = min(best, ms)
    return np.array(feats, np.float64), y, cens


def collect(workloads, tables, label):
    F, Y, C = [], [], []
    t0 = time.time()
    for j, w in enumerate(workloads):
        f, y, c = time_workload(tables, w)
        F.append(f)
        Y.append(y)
        C.append(c)
        if (j + 1) % 25 == 0:
            log(f"{label}: {j + 1}/{len(workloads)} workloads, {time.time() - t0:.0f}s")
    return np.array(F), np.array(Y), np.array(C)


def train(F, Y, epochs=4000, lr=3e-3, seed=0):
    """Fit the network on the GPU with the library's kernels; returns
    (params, mean, std, final loss)."""
    mask = np.isfinite(Y)
    mean = F.mean(0)
    std = F.std(0)
    std[std < 1e-6] = 1.0
    X = ((F - mean) / std).astype(np.float32)
    T = np.where(mask, Y, 0.0).astype(np.float32)
    rng = np.random.default_rng(seed)
    p = np.zeros(vrs.MLP_PARAMS, np.float32)
    o = 0
    for fan_in, fan_out in ((6, 64), (64, 64), (64, 16)):
        lim = math.sqrt(6.0 / fan_in)
        p[o:o + fan_in * fan_out] = rng.uniform(-lim, lim, fan_in * fan_out) * (0.5 if fan_out == 16 else 1.0)
        o += fan_in * fan_out + fan_out
    p[-16:] = np.nanmean(np.where(mask, Y, np.nan), axis=0).astype(np.float32)
    p[-16:] = np.where(np.isfinite(p[-16:]), p[-16:], 0.0)
    dp = torch.from_numpy(p).cuda()
    dx, dt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    dm = torch.from_numpy(mask.astype(np.uint8)).cuda()
    m, v = torch.zeros_like(dp), torch.zeros_like(dp)
    act = torch.empty((X.shape[0], 2 * vrs.MLP_HIDDEN), dtype=torch.float32, device="cuda")
    loss = None
    for step in range(1, epochs + 1):
        y = vrs.mlp_forward(dp, dx, act)
        g, loss = vrs.mlp_backward(dp, dx, y, act, dt, dm)
        vrs.mlp_adam(dp, g, m, v, step, lr=lr * (0.1 if step > 0.8 * epochs else 1.0))
    return dp.cpu().numpy(), mean.astype(np.float32), std.astype(np.float32), float(loss.item())


def save(path, params, mean, std):
    with open(path, "wb") as f:
        f.write(b"VRSCHOOS")
        f.write(struct.pack("<ii", 1, vrs.MLP_PARAMS))
        f.write(np.asarray(params, "<f4").tobytes())
        f.write(np.asarray(mean, "<f4").tobytes())
        f.write(np.asarray(std, "<f4").tobytes())


def evaluate(workloads, F, Y, C, params, mean, std, tables):
    """Regret of the learned and heuristic picks against the best timed arm."""
    nt = vrs.num_tiles()
    res = {"learned": [], "heuristic": []}
    for j, w in enumerate(workloads):
        y = Y[j]
        if not np.isfinite(y).any():
            continue
        tbest = math.exp(np.nanmin(y))
        T = tables.get(w.d, w.dtype, w.n)
        width = inputs.two_term_width(w.sel, ATTR_RANGE)
        pred = [(0, 0, width), (1, 0, width)]
        vrs.chooser_set(params, mean, std)
        _, s_l, t_l = T.plan(w.b, pred, w.k, vrs.IP, chooser=vrs.CHOOSER_LEARNED)
        vrs.chooser_clear()
        _, s_h, t_h = T.plan(w.b, pred, w.k, vrs.IP, chooser=vrs.CHOOSER_HEURISTIC)
        for name, s, t in (("learned", s_l, t_l), ("heuristic", s_h, t_h)):
            a = (s - 1) * nt + t
            tp = math.exp(y[a]) if np.isfinite(y[a]) else tbest * 100.0
            res[name].append(tp / tbest - 1.0)
    out = {}
    for name, r in res.items():
        r = np.array(r)
        out[name] = {"mean_regret": float(r.mean()), "p95_regret": float(np.percentile(r, 95)),
                     "median_regret": float(np.median(r)), "frac_best": float((r < 1e-9).mean()),
                     "n": int(r.size)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=1250)
    ap.add_argument("--heldout", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=4000)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--report", default=REPORT)
    args = ap.parse_args()
    tables = Tables()
    wt = inputs.chooser_workloads(CFG_TRAIN, args.train)
    wh = inputs.chooser_workloads(CFG_HELDOUT, args.heldout)
    t0 = time.time()
    Ft, Yt, Ct = collect(wt, tables, "train")
    t_collect = time.time() - t0
    log(f"training set: {len(wt)} workloads, {int(np.isfinite(Yt).sum())} timed arms "
        f"({int(Ct.sum())} censored), {t_collect:.0f}s")
    t0 = time.time()
    params, mean, std, loss = train(Ft, Yt, epochs=args.epochs)
    t_train = time.time() - t0
    log(f"trained in {t_train:.1f}s, final masked MSE {loss:.4f}")
    save(args.out, params, mean, std)
    t0 = time.time()
    Fh, Yh, Ch = collect(wh, tables, "heldout")
    t_held = time.time() - t0
    ev = evaluate(wh, Fh, Yh, Ch, params, mean, std, tables)
    report = {"train_workloads": len(wt), "train_timed_arms": int(np.isfinite(Yt).sum()),
              "train_censored_arms": int(Ct.sum()), "heldout_workloads": len(wh),
              "heldout_timed_arms": int(np.isfinite(Yh).sum()), "final_train_mse_ln_ms": loss,
              "collect_train_s": round(t_collect, 1), "train_s": round(t_train, 2),
              "collect_heldout_s": round(t_held, 1), "regret": ev, "arms": vrs.num_tiles() * 2,
              "workload_ranges": {"n": "logU[1e5, 1e7] (d<=128), [1e5, 4e6] (768), [1e5, 2e6] (1536)",
                                  "d": list(inputs.CHOOSER_DIMS), "B": "logU-int[1, 4096]",
                                  "selectivity": "logU[1e-4, 1] (3/4), U[0.3, 1] (1/4)",
                                  "k": [1, 10, 100],
                                  "dtype": ["f32", "bf16", "fp8"], "metric": "IP (normalised rows)"}}
    with open(args.report, "w") as f:
        json.dump(report, f, indent=1)
    print(json.dumps(report["regret"]), flush=True)


if __name__ == "__main__":
    main()
