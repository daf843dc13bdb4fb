// planner.cpp -- workspace layout, access-path choice and the launch
// sequence of one scan (see api.cpp for the ABI checks around it).
#include "planner.h"

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <cmath>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

namespace vrs {

namespace {

// VALU streaming tiles (queries per workgroup 1..8; wg_target = workgroups)
// and MFMA tiles (64 queries per workgroup; wg_target = quarter-rounds of
// resident workgroups: 4 = one full round, 8 = two, 2 = half a round).
const TileCfg kTiles[] = {
    {0, 1, 1024}, {0, 2, 1024}, {0, 4, 1024}, {0, 8, 1024},
    {1, 64, 4}, {1, 128, 4}, {1, 64, 8}, {1, 128, 8},
};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);
constexpr int kChooserMaxB = 4096;  // largest batch of the chooser's training workloads
constexpr size_t LDS_BUDGET = 64 * 1024;  // several workgroups per CU

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

double gamma_n(double n, double u) { return n * u / (1.0 - n * u); }

int screen_cb(int Kp) { return next_pow2(std::max(2 * Kp, Kp + 256)) - Kp; }

// Largest tile-compatible query count per workgroup that fits the LDS budget.
int fit_qt(int qt, int Kp, int CB, int dp) {
    while (qt > 1 && screen_stream_lds(qt, Kp, CB, dp) > LDS_BUDGET) qt >>= 1;
    return qt;
}

// est_rows: rows the screening kernel is expected to visit (the qualifying
// rows for gather, every row for mask); bounds the number of row chunks so
// that a workgroup always has enough rows to amortise its top-k state.  It
// is clamped to the table's rows: the workspace is sized for est_rows = n,
// and a plan must never need more chunks than that sizing assumed.
Plan make_plan(const vrs_table_s *t, int B, int kmax, const vrs_opts *opts, int tile,
               int strategy, int64_t est_rows = -1) {
    Plan P{};
    P.strategy = strategy;
    P.tile = tile;
    const int kmult = opts ? opts->kprime_mult : 0;
    P.kprime = kprime_rule(kmax, t->store, kmult);
    P.K = P.kprime + 1;
    P.Kp = next_pow2(P.K);
    const TileCfg &cfg = kTiles[tile];
    P.mfma = cfg.kind == 1;
    if (P.mfma) {
        P.CB = mfma_cb(P.Kp);
        P.qt = t->store == VRS_F32 ? cfg.qt : screen_mfma_bf16_qm();
        P.n_qtiles = (B + P.qt - 1) / P.qt;
        // (float32 batches of at most 16 queries run the small-batch form: one
        // 16-query group per workgroup)
        const int occ = t->store == VRS_F32 ? screen_mfma_occupancy(P.Kp, P.CB, B <= 16 ? 16 : P.qt) : 1;
        const int64_t slots = (int64_t)256 * occ * cfg.wg_target / 4;
        const int64_t rows = est_rows < 0 ? t->n : std::min<int64_t>(std::max<int64_t>(est_rows, 1), t->n);
        // at least 256 rows per chunk: a small selection still spreads over
        // many workgroups (with 1024 a 10,000-row selection ran as 8 chunks)
        int64_t max_chunks = std::max<int64_t>(1, rows / 256);
        int64_t nc = std::max<int64_t>(1, std::min<int64_t>(max_chunks, slots / P.n_qtiles));
        if (nc >= 8) nc = nc / 8 * 8;  // whole XCD groups: a row chunk's query tiles share an L2
        P.n_chunks = (int)nc;
        // two passes once a chunk holds 2048 rows or more (the first pass
        // screens a short prefix of every chunk; the extra merge costs tens
        // of microseconds)
        const int passes = opts ? opts->passes : 0;
        P.two_pass = passes == 2 || (passes != 1 && rows / nc >= 2048);
    } else {
        P.CB = screen_cb(P.Kp);
        P.qt = fit_qt(std::min(cfg.qt, next_pow2(B)), P.Kp, P.CB, t->dp);
        P.n_qtiles = (B + P.qt - 1) / P.qt;
        int64_t max_chunks = std::max<int64_t>(1, (t->n + 1023) / 1024);
        P.n_chunks = (int)std::max<int64_t>(1, std::min<int64_t>(max_chunks, cfg.wg_target / P.n_qtiles));
    }
    // exact fallback: about 64K rows per task, bounded scratch
    const size_t fb_cap = (size_t)256 << 20;
    int64_t want = std::max<int64_t>(1, (t->n + 65535) / 65536);
    int64_t cap = std::max<int64_t>(1, (int64_t)(fb_cap / ((size_t)B * kmax * 16)));
    P.fb_chunks = (int)std::min(want, cap);
    P.fb_rows_per_chunk = (int)((t->n + P.fb_chunks - 1) / P.fb_chunks);
    // workspace layout
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += a256(bytes);
        return r;
    };
    P.o_qp = take((size_t)B * t->dp * 4);
    P.o_qnorm = take((size_t)B * 8);
    P.o_qn2 = take((size_t)B * 4);
    P.o_qhl = take(t->store == VRS_F32 ? 0 : screen_mfma_bf16_qfrag_bytes(B, t->dp));
    P.o_gthr = take((size_t)B * 8);
    P.o_cbuf = take(P.mfma ? (size_t)B * P.n_chunks * P.CB * 8 : 0);
    P.o_bitmap = take((size_t)(t->n + 31) / 32 * 4);
    P.o_blk = take((size_t)((t->n + SEL_BLOCK_ROWS - 1) / SEL_BLOCK_ROWS) * 4);
    P.o_sel = take((size_t)t->n * 4);
    P.o_selcnt = take(8);
    P.o_part = take((size_t)B * P.n_chunks * P.K * 8);
    P.o_heads = take(P.mfma ? 0 : (size_t)B * P.n_chunks * 8);
    P.o_fills = take(P.mfma ? (size_t)B * P.n_chunks * 4 : 0);
    P.o_mid = take((size_t)B * ((P.n_chunks + 2047) / 2048) * P.K * 8);
    P.o_merged = take((size_t)B * P.K * 8);
    P.o_rrdist = take((size_t)B * P.K * 8);
    P.o_fail = take((size_t)B * 4);
    P.o_failcnt = take(8);
    P.o_fb = take((size_t)B * P.fb_chunks * kmax * 16);
    P.o_preds = take((size_t)B * sizeof(PredDev));
    P.o_kc = take((size_t)B * 4);
    P.o_kps = take((size_t)B * 4);
    P.total = o;
    return P;
}

bool tile_ok(const vrs_table_s *t, int B, int kmax, const vrs_opts *opts, int tile,
             int metric = VRS_IP) {
    if (kTiles[tile].kind == 0) return true;
    const int kmult = opts ? opts->kprime_mult : 0;
    const int Kp = next_pow2(kprime_rule(kmax, t->store, kmult) + 1);
    // Rows wider than 256 coordinates are multiplied in chunks, and every
    // 64-row tile re-reads its queries' slice of the chunk: offered only while
    // the batch's prepared queries fit one XCD's 4 MB L2 (at 1536 coordinates
    // and 2000 queries the chunked form ran 2.4x slower than the streaming
    // kernel).
    if (t->store == VRS_F32)
        return screen_mfma_supported(t->dp, t->store, Kp, mfma_cb(Kp)) &&
               (t->dp <= 256 || (int64_t)B * t->dp * 4 <= ((int64_t)4 << 20));
    return screen_mfma_bf16_supported(t->dp, t->store, metric, Kp, mfma_cb(Kp));
}

int default_tile(const vrs_table_s *t, int B, int kmax, const vrs_opts *opts,
                 int metric = VRS_IP) {
    if (B >= 8 && tile_ok(t, B, kmax, opts, 4, metric)) return 4;
    if (B <= 1) return 0;
    if (B <= 2) return 1;
    if (B <= 4) return 2;
    return 3;
}

}  // namespace

int mfma_cb(int Kp) { return next_pow2(std::max(2 * Kp, Kp + 128)) - Kp; }

void ensure_dyn_lds(const void *kernel, size_t bytes) {
    static std::mutex mu;
    static std::map<const void *, size_t> done;
    std::lock_guard<std::mutex> g(mu);
    size_t &d = done[kernel];
    if (bytes <= d) return;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
        d = bytes;
    else
        (void)hipGetLastError();
}

// ------------------------------------------------------------ stage timing
namespace {
struct ProfRec {
    int stage;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
thread_local bool g_prof_quiet = false;  // set while a launch sequence is captured
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;
hipEvent_t g_prof_open[VRS_NUM_STAGES];

hipEvent_t prof_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

void prof_begin(int stage, hipStream_t s) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (!g_prof_on || g_prof_quiet) return;
    hipEvent_t e = prof_event();
    if (e && hipEventRecord(e, s) == hipSuccess) g_prof_open[stage] = e;
}

void prof_end(int stage, hipStream_t s) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (!g_prof_on || g_prof_quiet || !g_prof_open[stage]) return;
    hipEvent_t e = prof_event();
    if (e && hipEventRecord(e, s) == hipSuccess) g_prof_recs.push_back({stage, g_prof_open[stage], e});
    g_prof_open[stage] = nullptr;
}

void prof_quiet(bool on) { g_prof_quiet = on; }

void prof_enable(bool on) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = on;
}

hipError_t prof_collect(double *ms, int64_t *calls) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (int i = 0; i < VRS_NUM_STAGES; ++i) {
        ms[i] = 0.0;
        calls[i] = 0;
    }
    hipError_t err = hipSuccess;
    for (auto &r : g_prof_recs) {
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess) err = e;
        ms[r.stage] += t;
        calls[r.stage] += 1;
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
    }
    g_prof_recs.clear();
    return err;
}

int planner_num_tiles() { return kNumTiles; }
const TileCfg &planner_tile(int id) { return kTiles[id]; }

int kprime_rule(int k, vrs_dtype store, int kmult) {
    int kp;
    if (kmult > 0)
        kp = k * kmult;
    else if (store == VRS_F32)
        kp = std::max(2 * k, k + 32);
    else
        kp = std::max(4 * k, k + 32);
    return std::min(std::max(kp, k), 1024);
}

size_t plan_workspace(const vrs_table_s *t, int B, int kmax, const vrs_opts *opts) {
    size_t m = 0;
    for (int tile = 0; tile < kNumTiles; ++tile)
        if (tile_ok(t, B, kmax, opts, tile))
            m = std::max(m, make_plan(t, B, kmax, opts, tile, VRS_STRATEGY_GATHER).total);
    return m;
}

bool planner_tile_ok(const vrs_table_s *t, int B, int kmax, const vrs_opts *opts, int tile) {
    return tile_ok(t, B, kmax, opts, tile);
}

void plan_features(const vrs_table_s *t, int B, double sel, int k, float f[6]) {
    f[0] = (float)log((double)t->n);
    f[1] = (float)log((double)t->d);
    f[2] = (float)log((double)B);
    f[3] = (float)log(std::max(sel, 1e-6));
    f[4] = (float)log((double)k);
    f[5] = (float)t->store;
}

// The arms offered to the learned chooser for a call.
static void chooser_arms(const vrs_table_s *t, int B, int k, int metric, bool batched, double est_sel,
                         const vrs_opts *opts, bool *allowed) {
    const int want_s = opts ? opts->strategy : VRS_STRATEGY_AUTO;
    const int want_t = opts ? opts->tile : -1;
    // A streaming tile re-reads the table once per query tile; when an MFMA
    // tile exists, arms that would re-read it 8 or more times are not
    // offered to the network (it has not seen every such shape).
    bool any_mfma = false;
    for (int tile = 0; tile < kNumTiles; ++tile)
        if (kTiles[tile].kind == 1 && tile_ok(t, B, k, opts, tile, metric)) any_mfma = true;
    // When the predicate keeps (almost) every row, the gathered scan can
    // skip nothing and still pays the selection pass and the id reads: only
    // masked arms are offered (the network has seen few such workloads and
    // can misjudge the small margin).
    const bool dense = est_sel >= 0.9;
    for (int sidx = 0; sidx < 2; ++sidx)
        for (int tile = 0; tile < kNumTiles; ++tile) {
            const int st = sidx + 1;
            bool ok = tile_ok(t, B, k, opts, tile, metric);
            if (want_s != VRS_STRATEGY_AUTO && st != want_s) ok = false;
            if (want_s == VRS_STRATEGY_AUTO && dense && st == VRS_STRATEGY_GATHER) ok = false;
            if (batched && st != VRS_STRATEGY_MASK) ok = false;
            if (want_t >= 0 && tile != want_t) ok = false;
            if (want_t < 0 && any_mfma && kTiles[tile].kind == 0 && (B + kTiles[tile].qt - 1) / kTiles[tile].qt >= 8)
                ok = false;
            allowed[sidx * kNumTiles + tile] = ok;
        }
}

double plan_predict_ms(const vrs_table_s *t, int B, const PredDev &p, int k, int metric) {
    if (!chooser_ready() || B > kChooserMaxB) return -1.0;
    const double est_sel = estimate_selectivity(t, p);
    float feats[6];
    plan_features(t, B, est_sel, k, feats);
    bool allowed[2 * kNumTiles];
    chooser_arms(t, B, k, metric, false, est_sel, nullptr, allowed);
    float y = 0.0f;
    if (chooser_pick_value(feats, allowed, 2 * kNumTiles, &y) < 0) return -1.0;
    return std::exp((double)y);
}

void plan_decide(const vrs_table_s *t, int B, const PredDev &p, bool batched, int k, int metric,
                 const vrs_opts *opts, float feats[6], int *strategy_out, int *tile_out) {
    const double est_sel = batched ? 1.0 : estimate_selectivity(t, p);
    plan_features(t, B, est_sel, k, feats);
    const int want_s = opts ? opts->strategy : VRS_STRATEGY_AUTO;
    const int want_t = opts ? opts->tile : -1;
    // The network is trained on batches of 1 to kChooserMaxB queries; larger
    // ones (e.g. a join's batches of R rows) take the heuristic rather than an
    // extrapolation.
    const bool learned = (!opts || opts->chooser == VRS_CHOOSER_LEARNED) && chooser_ready() && B <= kChooserMaxB;
    if (learned && (want_s == VRS_STRATEGY_AUTO || want_t < 0)) {
        bool allowed[2 * kNumTiles];
        chooser_arms(t, B, k, metric, batched, est_sel, opts, allowed);
        const int arm = chooser_pick(feats, allowed, 2 * kNumTiles);
        if (arm >= 0) {
            *strategy_out = arm / kNumTiles + 1;
            *tile_out = arm % kNumTiles;
            return;
        }
    }
    int tile = want_t >= 0 ? want_t : default_tile(t, B, k, opts, metric);
    if (!tile_ok(t, B, k, opts, tile, metric)) tile = default_tile(t, B, k, opts, metric);
    int strategy = want_s;
    if (batched) strategy = VRS_STRATEGY_MASK;  // per-query predicates are checked per row
    if (strategy == VRS_STRATEGY_AUTO) {
        // selectivity-threshold heuristic
        strategy = est_sel < 0.5 ? VRS_STRATEGY_GATHER : VRS_STRATEGY_MASK;
        if (p.nterms == 0) strategy = VRS_STRATEGY_MASK;
    }
    *strategy_out = strategy;
    *tile_out = tile;
}

hipError_t run_scan(const vrs_table_s *t, const float *q, int B, const PredDev &p,
                    const vrs_pred *preds, const int32_t *ks, int k, vrs_metric metric,
                    int64_t *out_idx, float *out_dist, void *ws, const vrs_opts *opts,
                    hipStream_t s) {
    const bool batched = preds != nullptr;
    float feats[6];
    int strategy, tile;
    plan_decide(t, B, p, batched, k, metric, opts, feats, &strategy, &tile);
    const double est_sel = batched ? 1.0 : estimate_selectivity(t, p);
    const int64_t est_rows =
        strategy == VRS_STRATEGY_GATHER ? (int64_t)(est_sel * (double)t->n * 1.25) + 4096 : t->n;
    Plan P = make_plan(t, B, k, opts, tile, strategy, est_rows);
    // the caller's workspace holds plan_workspace() bytes: a plan larger than
    // that is refused rather than run past the end of the buffer
    if (P.total > plan_workspace(t, B, k, opts)) return hipErrorInvalidValue;
    char *w = (char *)ws;
    float *qp = (float *)(w + P.o_qp);
    double *qnorm = (double *)(w + P.o_qnorm);
    float *qn2 = (float *)(w + P.o_qn2);
    uint16_t *qhl = t->store == VRS_F32 ? nullptr : (uint16_t *)(w + P.o_qhl);
    uint64_t *gthr = (uint64_t *)(w + P.o_gthr);
    int32_t *fail_count = (int32_t *)(w + P.o_failcnt);
    prof_begin(0, s);
    // (a streaming scan's per-chunk best keys start empty: they bound the lists)
    uint64_t *heads = P.mfma ? nullptr : (uint64_t *)(w + P.o_heads);
    hipError_t e = launch_prep_queries(q, B, t->d, t->dp, qp, qnorm, qn2, qhl, gthr, fail_count, heads,
                                       heads ? P.n_chunks : 0, s);
    if (e != hipSuccess) return e;
    PredDev *pdev = (PredDev *)(w + P.o_preds);
    int32_t *kc = (int32_t *)(w + P.o_kc), *kps = (int32_t *)(w + P.o_kps);
    if (batched) {
        e = launch_prep_batched(preds, ks, B, k, t->n_attr, opts ? opts->kprime_mult : 0,
                                t->store == VRS_F32, pdev, kc, kps, s);
        if (e != hipSuccess) return e;
    }
    prof_end(0, s);
    const bool gather = strategy == VRS_STRATEGY_GATHER;
    int32_t *sel = (int32_t *)(w + P.o_sel);
    int64_t *selcnt = (int64_t *)(w + P.o_selcnt);
    if (gather) {
        prof_begin(1, s);
        e = launch_select(t->attr, t->n, t->attr_stride, p, (uint32_t *)(w + P.o_bitmap),
                          (uint32_t *)(w + P.o_blk), sel, selcnt, s);
        if (e != hipSuccess) return e;
        prof_end(1, s);
    }
    ScreenArgs sa{};
    sa.rows = t->rows;
    sa.scale = t->scale;
    sa.n = t->n;
    sa.dp = t->dp;
    sa.store = t->store;
    sa.attr = t->attr;
    sa.an = t->attr_stride;
    sa.n_attr = t->n_attr;
    sa.pred = p;
    sa.preds = batched ? pdev : nullptr;
    sa.sel_ids = sel;
    sa.sel_count = selcnt;
    sa.gather = gather;
    // qualifying fraction of the rows a chunk visits (per-query predicates:
    // not known here, taken low so the first pass samples enough rows)
    sa.prefix_sel = gather ? 1.0f : (batched ? 0.01f : (float)std::max(est_sel, 1e-3));
    sa.qp = qp;
    sa.qn2 = qn2;
    sa.qhl = qhl;
    sa.norm2 = t->norm2;
    sa.cbuf = (uint64_t *)(w + P.o_cbuf);
    sa.gthr = gthr;
    sa.B = B;
    sa.metric = metric;
    sa.K = P.K;
    sa.Kp = P.Kp;
    sa.CB = P.CB;
    sa.n_chunks = P.n_chunks;
    sa.shared_rows = P.n_qtiles > 1;
    sa.partials = (uint64_t *)(w + P.o_part);
    sa.heads = heads;
    sa.heads_bound = heads != nullptr;
    sa.fills = P.mfma ? (int32_t *)(w + P.o_fills) : nullptr;
    FinishArgs fa{};
    fa.rows = t->rows;
    fa.scale = t->scale;
    fa.n = t->n;
    fa.d = t->d;
    fa.dp = t->dp;
    fa.store = t->store;
    fa.attr = t->attr;
    fa.an = t->attr_stride;
    fa.pred = p;
    fa.preds = batched ? pdev : nullptr;
    fa.q = q;
    fa.qnorm = qnorm;
    fa.B = B;
    fa.metric = metric;
    fa.k = k;
    fa.ks = batched ? kc : nullptr;
    fa.kmax = k;
    fa.kprime = P.kprime;
    fa.kps = batched ? kps : nullptr;
    fa.K = P.K;
    fa.n_chunks = P.n_chunks;
    fa.partials = sa.partials;
    fa.heads = sa.heads;
    fa.fills = sa.fills;
    // with a dense predicate the chunk lists are full and one head per list
    // bounds the merge well; with a selective one a chunk's rows come from
    // one neighbourhood and several heads per list are needed, unless the
    // lists hold few keys each (at most 128 qualifying rows per chunk
    // expected: gathered rows spread over the streaming kernel's many chunks)
    const double keys_per_list = std::exp((double)feats[3]) * (double)t->n / std::max(1, P.n_chunks);
    fa.merge_one_head = feats[3] >= (float)std::log(0.05) || keys_per_list <= 128.0;
    fa.merge_mid = (uint64_t *)(w + P.o_mid);
    fa.merged = (uint64_t *)(w + P.o_merged);
    fa.rr_dist = (double *)(w + P.o_rrdist);
    // Screening error bound, FP32 accumulation in any order (both sides of the
    // certificate also carry the FP64 sum's own error):
    //   VALU L2SQ: sum of dp non-negative rounded terms -> relative gamma_{dp+3};
    //   MFMA L2SQ: |q|^2 + |x|^2 - 2 q.x with every product possibly rounded
    //              -> absolute gamma_{dp+6} * (|q| + max|x|)^2;
    //   IP:        |error| <= gamma_{dp+3} * |q| * max|x|.
    // The VALU kernels use IEEE fused multiply-adds rounded to nearest (unit
    // roundoff u = 2^-24).  For the matrix instructions the internal rounding
    // of the accumulation is not relied on: the model assumes only that every
    // operation is faithful (error below one ulp of its result), i.e. unit
    // roundoff 2^-23; the measured ratio error / bound is reported by the
    // err_ratio diagnostic.
    const double u32 = ldexp(1.0, -24), u64 = ldexp(1.0, -53);
    const double um = P.mfma ? ldexp(1.0, -23) : u32;
    const double g = (gamma_n(t->dp + 3, u32) + gamma_n(t->dp + 3, u64)) * 1.001;
    const double g6 = (gamma_n(t->dp + 6, um) + gamma_n(t->dp + 3, u64)) * 1.001;
    //   bf16 MFMA IP (hi/lo query split, FP8 scale applied to the sum):
    //              gamma_{dp+2} (1 + 2^-7) + 2^-16 + 3u, times |q| max|x|.
    fa.rel = (metric == VRS_L2SQ && !P.mfma) ? g : 0.0;
    fa.abs_ip = metric == VRS_IP ? g6 : 0.0;
    fa.abs_l2 = (metric == VRS_L2SQ && P.mfma) ? g6 : 0.0;
    if (P.mfma && t->store != VRS_F32)
        fa.abs_ip = (gamma_n(t->dp + 2, um) * (1.0 + ldexp(1.0, -7)) + ldexp(1.0, -16) +
                     3.0 * um + gamma_n(t->dp + 2, u64)) * 1.001;
    fa.max_norm = t->max_norm;
    fa.fail_list = (int32_t *)(w + P.o_fail);
    fa.fail_count = fail_count;
    fa.out_idx = out_idx;
    fa.out_dist = out_dist;
    fa.n_valid = opts ? opts->n_valid : nullptr;
    fa.certified = opts ? opts->certified : nullptr;
    fa.err_ratio = opts ? opts->err_ratio : nullptr;
    fa.fb_rows_per_chunk = P.fb_rows_per_chunk;
    fa.fb_chunks = P.fb_chunks;
    fa.fb_slots = B;
    fa.fb_partials = (uint64_t *)(w + P.o_fb);
    // MFMA kernels keep one bound per query and row chunk, so every chunk
    // pays for its own list fills.  With long chunks the scan runs in two
    // passes: a short prefix of every chunk, a merge of those lists whose
    // K-th key bounds the result (K keys are at or below it), then every
    // chunk in full with fresh lists that admit only keys up to that bound.
    auto screen = [&]() -> hipError_t {
        prof_begin(2, s);
        hipError_t r;
        if (!P.mfma)
            r = launch_screen_stream(sa, P.qt, s);
        else if (t->store == VRS_F32)
            r = launch_screen_mfma(sa, P.qt, s);
        else
            r = launch_screen_mfma_bf16(sa, s);
        prof_end(2, s);
        return r;
    };
    if (P.two_pass) {
        sa.pass = 1;
        if ((e = screen()) != hipSuccess) return e;
        prof_begin(3, s);
        if ((e = launch_merge(fa, s)) != hipSuccess) return e;
        if ((e = launch_set_bound(fa, gthr, nullptr, s)) != hipSuccess) return e;
        prof_end(3, s);
        sa.pass = 2;
    }
    if ((e = screen()) != hipSuccess) return e;

    prof_begin(3, s);
    e = launch_merge(fa, s);
    if (e != hipSuccess) return e;
    prof_end(3, s);
    prof_begin(4, s);
    e = launch_rerank(fa, s);
    if (e != hipSuccess) return e;
    prof_end(4, s);
    prof_begin(5, s);
    e = launch_fallback(fa, s);
    prof_end(5, s);
    return e;
}

// ------------------------------------------------------------- chooser
namespace {
std::mutex g_ch_mu;
bool g_ch_ready = false;
std::vector<float> g_ch_p, g_ch_mean, g_ch_std;
}  // namespace

bool chooser_set(const float *params, const float *mean, const float *stdv) {
    for (int i = 0; i < VRS_MLP_PARAMS; ++i)
        if (!std::isfinite(params[i])) return false;
    for (int i = 0; i < VRS_MLP_IN; ++i)
        if (!std::isfinite(mean[i]) || !std::isfinite(stdv[i]) || !(stdv[i] > 0.0f)) return false;
    std::lock_guard<std::mutex> g(g_ch_mu);
    g_ch_p.assign(params, params + VRS_MLP_PARAMS);
    g_ch_mean.assign(mean, mean + VRS_MLP_IN);
    g_ch_std.assign(stdv, stdv + VRS_MLP_IN);
    g_ch_ready = true;
    return true;
}

void chooser_clear() {
    std::lock_guard<std::mutex> g(g_ch_mu);
    g_ch_ready = false;
}

bool chooser_load(const char *path, std::string *err) {
    if (!path) {
        *err = "path is NULL";
        return false;
    }
    FILE *f = fopen(path, "rb");
    if (!f) {
        *err = std::string("cannot open chooser weights: ") + path;
        return false;
    }
    char magic[8];
    int32_t ver = 0, np = 0;
    std::vector<float> buf(VRS_MLP_PARAMS + 2 * VRS_MLP_IN);
    bool good = fread(magic, 1, 8, f) == 8 && memcmp(magic, "VRSCHOOS", 8) == 0 &&
                fread(&ver, 4, 1, f) == 1 && ver == 1 && fread(&np, 4, 1, f) == 1 &&
                np == VRS_MLP_PARAMS && fread(buf.data(), 4, buf.size(), f) == buf.size();
    fclose(f);
    if (!good) {
        *err = std::string("corrupt chooser weights file: ") + path;
        return false;
    }
    if (!chooser_set(buf.data(), buf.data() + VRS_MLP_PARAMS, buf.data() + VRS_MLP_PARAMS + VRS_MLP_IN)) {
        *err = std::string("chooser weights are not finite: ") + path;
        return false;
    }
    return true;
}

bool chooser_ready() {
    std::lock_guard<std::mutex> g(g_ch_mu);
    return g_ch_ready;
}

// Host inference of the chooser network (same layer formula as the kernels).
// The network's forward pass on the host: fmaf per multiply-add (the same
// correctly rounded operation as the GPU kernel's), compiled twice: with the
// FMA instruction set when the CPU has it, else through the library call.
__attribute__((always_inline)) static inline void mlp_host(const float *p, const float *mean, const float *stdv,
                                                           const float feats[6], float *y) {
    const int NI = VRS_MLP_IN, NH = VRS_MLP_HIDDEN, NO = VRS_MLP_OUT;
    const float *W1 = p, *b1 = W1 + NI * NH, *W2 = b1 + NH, *b2 = W2 + NH * NH, *W3 = b2 + NH,
                *b3 = W3 + NH * NO;
    float x[VRS_MLP_IN], h1[VRS_MLP_HIDDEN], h2[VRS_MLP_HIDDEN];
    for (int i = 0; i < NI; ++i) x[i] = (feats[i] - mean[i]) / stdv[i];
    for (int j = 0; j < NH; ++j) {
        float a = b1[j];
        for (int i = 0; i < NI; ++i) a = fmaf(x[i], W1[i * NH + j], a);
        h1[j] = a > 0.0f ? a : 0.0f;
    }
    for (int j = 0; j < NH; ++j) {
        float a = b2[j];
        for (int i = 0; i < NH; ++i) a = fmaf(h1[i], W2[i * NH + j], a);
        h2[j] = a > 0.0f ? a : 0.0f;
    }
    for (int j = 0; j < NO; ++j) {
        float a = b3[j];
        for (int i = 0; i < NH; ++i) a = fmaf(h2[i], W3[i * NO + j], a);
        y[j] = a;
    }
}
__attribute__((target("fma"))) static void mlp_host_fma(const float *p, const float *mean, const float *stdv,
                                                        const float feats[6], float *y) {
    mlp_host(p, mean, stdv, feats, y);
}
static void mlp_host_any(const float *p, const float *mean, const float *stdv, const float feats[6], float *y) {
    mlp_host(p, mean, stdv, feats, y);
}
static const bool g_host_fma = __builtin_cpu_supports("fma");

int chooser_pick(const float feats[6], const bool *allowed, int n_arms) {
    float y = 0.0f;
    return chooser_pick_value(feats, allowed, n_arms, &y);
}

int chooser_pick_value(const float feats[6], const bool *allowed, int n_arms, float *value) {
    std::lock_guard<std::mutex> g(g_ch_mu);
    if (!g_ch_ready) return -1;
    const int NO = VRS_MLP_OUT;
    float y[VRS_MLP_OUT];
    if (g_host_fma)
        mlp_host_fma(g_ch_p.data(), g_ch_mean.data(), g_ch_std.data(), feats, y);
    else
        mlp_host_any(g_ch_p.data(), g_ch_mean.data(), g_ch_std.data(), feats, y);
    int best = -1;
    for (int j = 0; j < std::min(n_arms, NO); ++j)
        if (allowed[j] && (best < 0 || y[j] < y[best])) best = j;
    if (best >= 0) *value = y[best];
    return best;
}

}  // namespace vrs
