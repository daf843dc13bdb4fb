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


MFMA_TILES = range(4, 8)   # tile ids of the MFMA kernels (the rest stream), as the planner's table
STREAM_QT = [1, 2, 4, 8]   # queries per workgroup of the streaming tiles


def allowed_arms(f, y, nt):
    """The arms the planner offers the network for a workload, from its
    recorded features and timings: the arms available for the table and k
    (timed or censored), no gather arm when the estimated selectivity is at
    least 0.9, and no streaming tile that would re-read the table 8 or more
    times when an MFMA tile is available (the rules of the planner)."""
    valid = np.isfinite(y)
    B = int(round(math.exp(f[2])))
    est_sel = math.exp(f[3])
    any_mfma = bool(valid[[s * nt + t for s in (0, 1) for t in MFMA_TILES]].any())
    allowed = valid.copy()
    if est_sel >= 0.9:
        allowed[nt:] = False
    for t, qt in enumerate(STREAM_QT):
        if any_mfma and (B + qt - 1) // qt >= 8:
            allowed[t] = allowed[nt + t] = False
    return allowed


def heuristic_arm(f, y, nt):
    """The selectivity-threshold heuristic's arm: gather below an estimated
    selectivity of 0.5; MFMA tile 4 from 8 queries, else the streaming tile
    for the batch size."""
    valid = np.isfinite(y)
    B = int(round(math.exp(f[2])))
    est_sel = math.exp(f[3])
    if B >= 8 and valid[4]:
        tile = 4
    else:
        tile = 0 if B <= 1 else (1 if B <= 2 else (2 if B <= 4 else 3))
    return (1 if est_sel < 0.5 else 0) * nt + tile


def evaluate_recorded(F, Y, params, mean, std):
    """Regret (t_pick / t_best - 1) of the learned and heuristic picks on
    recorded timings (a censored arm counts at its cost-model bound, at least
    8 times the best).  Deterministic: the learned pick is the library's own
    host inference (vrs_chooser_pick)."""
    nt = Y.shape[1] // 2
    vrs.chooser_set(params, mean, std)
    rows = []
    for f, y in zip(F, Y):
        if not np.isfinite(y).any():
            continue
        tbest = math.exp(np.nanmin(y))
        al = allowed_arms(f, y, nt)
        a_l = vrs.chooser_pick(f, al)
        a_h = heuristic_arm(f, y, nt)
        r, t = [], []
        for a in (a_l, a_h):
            tp = math.exp(y[a]) if a >= 0 and np.isfinite(y[a]) else tbest * 100.0
            r.append(tp / tbest - 1.0)
            t.append(tp)
        rows.append((r[0], r[1], a_l, a_h, int(np.nanargmin(y)), tbest, t[0]))
    vrs.chooser_clear()
    return rows


def summarize(rows):
    out = {}
    for j, name in ((0, "learned"), (1, "heuristic")):
        r = np.array([x[j] for x in rows])
        out[name] = {"mean_regret": float(r.mean()), "p95_regret": float(np.percentile(r, 95)),
                     "median_regret": float(np.median(r)), "frac_best": float((r < 1e-9).mean()),
                     "n": int(r.size)}
    return out


def tail_analysis(F, Y, rows, top=12):
    """Where the learned pick's regret concentrates: by dtype, dimension,
    batch and selectivity buckets, and the worst workloads."""
    keep = [i for i in range(len(F)) if np.isfinite(Y[i]).any()]
    Fk = F[keep]
    reg = np.array([x[0] for x in rows])
    groups = {}
    def add(key, mask):
        if mask.any():
            groups[key] = {"n": int(mask.sum()), "mean": round(float(reg[mask].mean()), 4),
                           "p95": round(float(np.percentile(reg[mask], 95)), 4)}
    for dt, nm in ((0, "f32"), (1, "bf16"), (2, "fp8")):
        add(f"dtype={nm}", np.isclose(Fk[:, 5], dt))
    for d in (64, 128, 768, 1536):
        add(f"d={d}", np.isclose(np.exp(Fk[:, 1]), d, rtol=1e-3))
    B = np.exp(Fk[:, 2])
    for lo, hi in ((1, 8), (8, 64), (64, 512), (512, 5000)):
        add(f"B=[{lo},{hi})", (B >= lo - 1e-6) & (B < hi))
    s = np.exp(Fk[:, 3])
    for lo, hi in ((0, 1e-3), (1e-3, 1e-2), (1e-2, 0.1), (0.1, 0.5), (0.5, 1.01)):
        add(f"sel=[{lo:g},{hi:g})", (s >= lo) & (s < hi))
    # milliseconds lost to the pick, and how much of the total the tail holds
    lost = np.array([x[6] - x[5] for x in rows])
    best = np.array([x[5] for x in rows])
    tail = reg >= np.percentile(reg, 95)
    groups["ms_lost"] = {"mean": round(float(lost.mean()), 4), "median": round(float(np.median(lost)), 4),
                         "tail_p95_mean_best_ms": round(float(best[tail].mean()), 4),
                         "tail_p95_mean_lost_ms": round(float(lost[tail].mean()), 4),
                         "all_mean_best_ms": round(float(best.mean()), 4),
                         "total_lost_over_total_best": round(float(lost.sum() / best.sum()), 4)}
    worst = np.argsort(-reg)[:top]
    w = [{"N": int(round(math.exp(Fk[i, 0]))), "d": int(round(math.exp(Fk[i, 1]))),
          "B": int(round(math.exp(Fk[i, 2]))), "est_sel": float(math.exp(Fk[i, 3])),
          "k": int(round(math.exp(Fk[i, 4]))), "dtype": int(Fk[i, 5]), "regret": round(float(reg[i]), 3),
          "learned_arm": rows[i][2], "best_arm": rows[i][4], "best_ms": round(rows[i][5], 4),
          "learned_ms": round(rows[i][6], 4)} for i in worst]
    return {"groups": groups, "worst": w}


def load_weights(path):
    raw = open(path, "rb").read()
    assert raw[:8] == b"VRSCHOOS"
    n = struct.unpack("<ii", raw[8:16])[1]
    arr = np.frombuffer(raw[16:], "<f4")
    return arr[:n].copy(), arr[n:n + 6].copy(), arr[n + 6:n + 12].copy()


HELDOUT = os.path.join(HERE, "chooser_heldout.npz")
TRAINSET = os.path.join(HERE, "chooser_train.npz")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--phase", choices=["train", "heldout", "report"], required=True,
                    help="train: time the training workloads and fit the network (GPU); heldout: time the "
                         "held-out workloads exhaustively (GPU); report: regret on the recorded held-out "
                         "timings (host only)")
    ap.add_argument("--train", type=int, default=1350)
    ap.add_argument("--heldout", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=4000)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--report", default=REPORT)
    ap.add_argument("--trainset", default=TRAINSET, help="recorded training timings (.npz)")
    ap.add_argument("--heldout-file", default=HELDOUT, help="recorded held-out timings (.npz)")
    args = ap.parse_args()
    if args.phase == "train":
        tables = Tables()
        wt = inputs.chooser_workloads(CFG_TRAIN, args.train)
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
        np.savez_compressed(args.trainset, F=Ft, Y=Yt, C=Ct, collect_s=t_collect, train_s=t_train, loss=loss)
        return
    if args.phase == "heldout":
        tables = Tables()
        wh = inputs.chooser_workloads(CFG_HELDOUT, args.heldout)
        t0 = time.time()
        Fh, Yh, Ch = collect(wh, tables, "heldout")
        t_held = time.time() - t0
        # inference latency of the network on the GPU (one workload, the
        # library's forward kernel), HIP events
        params, mean, std = load_weights(args.out)
        dp = torch.from_numpy(params).cuda()
        x = torch.from_numpy(((Fh[:1] - mean) / std).astype(np.float32)).cuda()
        act = torch.empty((1, 2 * vrs.MLP_HIDDEN), dtype=torch.float32, device="cuda")
        vrs.mlp_forward(dp, x, act)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(100):
            vrs.mlp_forward(dp, x, act)
        e1.record()
        e1.synchronize()
        hip_us = e0.elapsed_time(e1) * 10.0
        np.savez_compressed(args.heldout_file, F=Fh, Y=Yh, C=Ch, collect_s=t_held, hip_infer_us=hip_us)
        log(f"held-out: {len(wh)} workloads in {t_held:.0f}s, HIP inference {hip_us:.1f} us")
        return
    # report (host only)
    params, mean, std = load_weights(args.out)
    H = np.load(args.heldout_file)
    Fh, Yh, Ch = H["F"], H["Y"], H["C"]
    rows = evaluate_recorded(Fh, Yh, params, mean, std)
    vrs.chooser_set(params, mean, std)
    f0 = Fh[0].astype(np.float32)
    al = np.ones(Yh.shape[1], np.uint8)
    t0 = time.perf_counter()
    for _ in range(10000):
        vrs.chooser_pick(f0, al)
    host_us = (time.perf_counter() - t0) / 10000 * 1e6
    vrs.chooser_clear()
    # the same Python marshalling around a call that returns at once (no network)
    t0 = time.perf_counter()
    for _ in range(10000):
        vrs.chooser_pick(f0, al)
    empty_us = (time.perf_counter() - t0) / 10000 * 1e6
    report = {"heldout_workloads": int(Fh.shape[0]), "heldout_timed_arms": int((np.isfinite(Yh) & ~Ch).sum()),
              "heldout_censored_arms": int(Ch.sum()), "collect_heldout_s": round(float(H["collect_s"]), 1),
              "regret": summarize(rows), "tail": tail_analysis(Fh, Yh, rows),
              "inference_us": {"host_pick_incl_python_call": round(host_us, 2),
                               "host_pick_net_of_python_call": round(host_us - empty_us, 2),
                               "hip_forward_one_workload_incl_python_launch": round(float(H["hip_infer_us"]), 2)},
              "arms": int(Yh.shape[1])}
    if os.path.exists(args.trainset):
        T = np.load(args.trainset)
        report.update({"train_workloads": int(T["F"].shape[0]),
                       "train_timed_arms": int((np.isfinite(T["Y"]) & ~T["C"]).sum()),
                       "train_censored_arms": int(T["C"].sum()), "collect_train_s": round(float(T["collect_s"]), 1),
                       "train_s": round(float(T["train_s"]), 2), "final_train_mse_ln_ms": float(T["loss"])})
    report["workload_ranges"] = {"n": "logU[1e5, 1e7] (d<=128), [1e5, 4e6] (768), [1e5, 2e6] (1536)",
                                 "d": list(inputs.CHOOSER_DIMS), "B": "logU-int[1, 4096]",
                                 "selectivity": "logU[1e-4, 1] (3/4), U[0.3, 1] (1/4)", "k": [1, 10, 100],
                                 "dtype": ["f32", "bf16", "fp8"], "metric": "IP (normalised rows)"}
    with open(args.report, "w") as f:
        json.dump(report, f, indent=1)
    print(json.dumps(report["regret"]), flush=True)


if __name__ == "__main__":
    main()
