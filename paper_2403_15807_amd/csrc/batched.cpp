// batched.cpp -- host side of the batched uneven form: workspace layout,
// the launch sequence (no host synchronisation, no memset: capturable into
// a HIP graph), the configuration table and its autotuner.
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "planner.h"

namespace vrs {

namespace {

// cap_frac, rounds, seg_rows
const BatchCfg kCfgs[] = {
    {0.0, 4, 4096},          // every query dense
    {0.0, 8, 4096},
    {1.0 / 1024, 4, 4096},
    {1.0 / 256, 4, 4096},
    {1.0 / 100, 4, 4096},
    {1.0 / 100, 8, 4096},
    {1.0 / 32, 4, 4096},
    {1.0 / 32, 8, 8192},
};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);
constexpr int kDefaultCfg = 4;
int dense_qm(const vrs_table_s *t) { return t->store == VRS_F32 ? 64 : screen_mfma_bf16_qm(); }
constexpr int NC_CAP = 512;       // most row chunks per dense query
constexpr int SEG_MAX = 32;       // most work items per sparse query
constexpr int SPARSE_WG_PER_CU = 4;
constexpr int NUM_CU = 256;

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
double gamma_n(double n, double u) { return n * u / (1.0 - n * u); }

struct BPlan {
    int kprime, K, Kp, CB;
    int occ, dense_grid, sparse_grid, items_target;
    int64_t rows_cap;
    int nsub;
    int64_t dense_lists, lists;
    int fb_chunks, fb_rows_per_chunk;
    bool two_pass;  // dense side in two passes (prefix of every chunk, merged bound, all rows)
    size_t o_qp, o_qnorm, o_qn2, o_qhl, o_gthr, o_ctl, o_pred_o, o_pred_p, o_qr, o_cands, o_kc_o, o_kps_o, o_kc_p,
        o_kps_p, o_cand, o_tot, o_perm, o_spoff, o_spcnt, o_segpre, o_listoff, o_nlists,
        o_pool, o_part, o_cbuf, o_merged, o_rrdist, o_fail, o_failcnt, o_fb, total;
};

BPlan make_bplan(const vrs_table_s *t, int B, int kmax, const vrs_opts *opts, int cfg) {
    const BatchCfg &c = kCfgs[cfg];
    BPlan P{};
    const int kmult = opts ? opts->kprime_mult : 0;
    P.kprime = kprime_rule(kmax, t->store, kmult);
    P.K = P.kprime + 1;
    P.Kp = next_pow2(P.K);
    P.CB = mfma_cb(P.Kp);
    P.occ = t->store == VRS_F32 ? screen_mfma_occupancy(P.Kp, P.CB, 64) : 1;
    P.dense_grid = NUM_CU * P.occ;
    P.sparse_grid = NUM_CU * SPARSE_WG_PER_CU;
    P.items_target = c.rounds * P.dense_grid;
    P.rows_cap = (int64_t)floor(c.cap_frac * (double)t->n);
    const int passes = opts ? opts->passes : 0;
    P.two_pass = passes == 2 || (passes != 1 && t->n >= ((int64_t)1 << 20));
    P.nsub = (int)((t->n + BSUB_ROWS - 1) / BSUB_ROWS);
    const int qm = dense_qm(t);
    const int64_t ntiles = (B + qm - 1) / qm;
    P.dense_lists = std::min<int64_t>((int64_t)B * NC_CAP,
                                      (int64_t)qm * std::max<int64_t>(P.items_target, 8 * ntiles));
    P.lists = P.dense_lists + (P.rows_cap > 0 ? (int64_t)B * SEG_MAX : 0);
    const size_t fb_cap = (size_t)256 << 20;
    const int64_t want = std::max<int64_t>(1, (t->n + 65535) / 65536);
    const int64_t cap = std::max<int64_t>(1, (int64_t)(fb_cap / ((size_t)B * kmax * 16)));
    P.fb_chunks = (int)std::min(want, cap);
    P.fb_rows_per_chunk = (int)((t->n + P.fb_chunks - 1) / P.fb_chunks);
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
    P.o_ctl = take(BC_WORDS * 4);
    P.o_pred_o = take((size_t)B * sizeof(PredDev));
    P.o_pred_p = take((size_t)B * sizeof(PredDev));
    P.o_qr = take((size_t)B * sizeof(QRange));
    P.o_cands = take((size_t)B * sizeof(QRange));
    P.o_kc_o = take((size_t)B * 4);
    P.o_kps_o = take((size_t)B * 4);
    P.o_kc_p = take((size_t)B * 4);
    P.o_kps_p = take((size_t)B * 4);
    P.o_cand = take((size_t)B);
    P.o_tot = take((size_t)B * 4);
    P.o_perm = take((size_t)B * 4);
    P.o_spoff = take((size_t)B * 8);
    P.o_spcnt = take((size_t)B * 4);
    P.o_segpre = take((size_t)(B + 1) * 4);
    P.o_listoff = take((size_t)B * 8);
    P.o_nlists = take((size_t)B * 4);
    P.o_pool = take((size_t)B * P.rows_cap * 4);
    P.o_part = take((size_t)P.lists * P.K * 8);
    P.o_cbuf = take((size_t)P.dense_lists * P.CB * 8);
    P.o_merged = take((size_t)B * P.K * 8);
    P.o_rrdist = take((size_t)B * P.K * 8);
    P.o_fail = take((size_t)B * 4);
    P.o_failcnt = take(8);
    P.o_fb = take((size_t)B * P.fb_chunks * kmax * 16);
    P.total = o;
    return P;
}

std::mutex g_tune_mu;
std::map<std::tuple<const void *, int64_t, int, int, int, int>, int> g_tuned;

auto tune_key(const vrs_table_s *t, int B, int kmax, int metric, const vrs_opts *opts) {
    return std::make_tuple((const void *)t->rows, t->n, B, kmax, metric, opts ? opts->kprime_mult : 0);
}

}  // namespace

int batched_num_cfgs() { return kNumCfgs; }
const BatchCfg &batched_cfg(int i) { return kCfgs[i]; }

bool batched_native(const vrs_table_s *t, int kmax, int metric, const vrs_opts *opts) {
    const int kmult = opts ? opts->kprime_mult : 0;
    const int Kp = next_pow2(kprime_rule(kmax, t->store, kmult) + 1);
    // (the persistent FP32 kernel keeps whole rows of at most 256 coordinates)
    if (t->store == VRS_F32) return t->dp <= 256 && screen_mfma_supported(t->dp, t->store, Kp, mfma_cb(Kp));
    return screen_mfma_bf16_supported(t->dp, t->store, metric, Kp, mfma_cb(Kp));
}

size_t batched_workspace(const vrs_table_s *t, int B, int kmax, int metric, const vrs_opts *opts) {
    if (!batched_native(t, kmax, metric, opts)) return 0;
    size_t m = 0;
    for (int c = 0; c < kNumCfgs; ++c) m = std::max(m, make_bplan(t, B, kmax, opts, c).total);
    return m;
}

int batched_tuned(const vrs_table_s *t, int B, int kmax, int metric, const vrs_opts *opts) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tuned.find(tune_key(t, B, kmax, metric, opts));
    return it == g_tuned.end() ? -1 : it->second;
}

int batched_pick(const vrs_table_s *t, int B, int kmax, int metric, const vrs_opts *opts) {
    if (opts && opts->tile >= 0) return opts->tile;
    const int c = batched_tuned(t, B, kmax, metric, opts);
    return c >= 0 ? c : kDefaultCfg;
}

hipError_t run_batched(const vrs_table_s *t, const float *q, int B, const vrs_pred *preds,
                       const int32_t *ks, int kmax, vrs_metric metric, int64_t *out_idx,
                       float *out_dist, void *ws, const vrs_opts *opts, int cfg, hipStream_t s) {
    const BPlan P = make_bplan(t, B, kmax, opts, cfg);
    char *w = (char *)ws;
    int32_t *ctl = (int32_t *)(w + P.o_ctl);
    BatchArgs ba{};
    ba.preds = preds;
    ba.ks = ks;
    ba.B = B;
    ba.kmax = kmax;
    ba.n_attr = t->n_attr;
    ba.kmult = opts ? opts->kprime_mult : 0;
    ba.f32_rule = t->store == VRS_F32;
    // every query's list holds up to P.kprime + 1 keys (sized for k_max):
    // under the default rule a query with a small k reranks at least
    // min(128, P.kprime) of them, which keeps its certificate clear of the
    // near-ties of dense clusters at little cost
    ba.kfloor = std::min(128, P.kprime);
    ba.attr = t->attr;
    ba.n = t->n;
    ba.an = t->attr_stride;
    ba.dstats = t->dstats;
    ba.rows_cap = t->n_attr > 0 && t->dstats ? P.rows_cap : 0;
    ba.seg_rows = kCfgs[cfg].seg_rows;
    ba.seg_max = SEG_MAX;
    ba.items_target = P.items_target;
    ba.nc_cap = NC_CAP;
    ba.qm = dense_qm(t);
    ba.nsub = P.nsub;
    ba.pred_o = (PredDev *)(w + P.o_pred_o);
    ba.qr = (QRange *)(w + P.o_qr);
    ba.cands = (QRange *)(w + P.o_cands);
    ba.kc_o = (int32_t *)(w + P.o_kc_o);
    ba.kps_o = (int32_t *)(w + P.o_kps_o);
    ba.cand = (uint8_t *)(w + P.o_cand);
    ba.tot = (int32_t *)(w + P.o_tot);
    ba.perm = (int32_t *)(w + P.o_perm);
    ba.sp_off = (int64_t *)(w + P.o_spoff);
    ba.sp_cnt = (int32_t *)(w + P.o_spcnt);
    ba.seg_pre = (int32_t *)(w + P.o_segpre);
    ba.list_off = (int64_t *)(w + P.o_listoff);
    ba.nlists = (int32_t *)(w + P.o_nlists);
    ba.pool = (int32_t *)(w + P.o_pool);
    ba.ctl = ctl;

    float *qp = (float *)(w + P.o_qp);
    double *qnorm = (double *)(w + P.o_qnorm);
    float *qn2 = (float *)(w + P.o_qn2);
    uint16_t *qhl = t->store == VRS_F32 ? nullptr : (uint16_t *)(w + P.o_qhl);
    uint64_t *gthr = (uint64_t *)(w + P.o_gthr);
    int32_t *fail_count = (int32_t *)(w + P.o_failcnt);
    PredDev *pred_p = (PredDev *)(w + P.o_pred_p);
    int32_t *kc_p = (int32_t *)(w + P.o_kc_p), *kps_p = (int32_t *)(w + P.o_kps_p);

    // predicate passes: selection vectors of the candidates, split, order
    prof_begin(1, s);
    hipError_t e = launch_batch_classify(ba, s);
    if (e != hipSuccess) return e;
    prof_end(1, s);
    prof_begin(0, s);
    e = launch_prep_permuted(q, ba.perm, B, t->d, t->dp, ba.pred_o, ba.kc_o, ba.kps_o, qp, qnorm, qn2,
                             qhl, gthr, fail_count, pred_p, kc_p, kps_p, s);
    if (e != hipSuccess) return e;
    prof_end(0, s);

    ScreenArgs sa{};
    sa.rows = t->rows;
    sa.scale = t->scale;
    sa.n = t->n;
    sa.dp = t->dp;
    sa.store = t->store;
    sa.attr = t->attr;
    sa.an = t->attr_stride;
    sa.n_attr = t->n_attr;
    sa.preds = pred_p;
    sa.qp = qp;
    sa.qn2 = qn2;
    sa.qhl = qhl;
    sa.norm2 = t->norm2;
    sa.B = B;
    sa.metric = metric;
    sa.K = P.K;
    sa.Kp = P.Kp;
    sa.CB = P.CB;
    sa.n_chunks = 0;  // set on the device
    sa.shared_rows = 1;
    sa.partials = (uint64_t *)(w + P.o_part);
    sa.cbuf = (uint64_t *)(w + P.o_cbuf);
    sa.gthr = gthr;
    sa.bctl = ctl;
    sa.sp_off = ba.sp_off;
    sa.sp_cnt = ba.sp_cnt;
    sa.seg_pre = ba.seg_pre;
    sa.sp_pool = ba.pool;
    sa.kps = kps_p;
    FinishArgs fa{};
    fa.rows = t->rows;
    fa.scale = t->scale;
    fa.n = t->n;
    fa.d = t->d;
    fa.dp = t->dp;
    fa.store = t->store;
    fa.attr = t->attr;
    fa.an = t->attr_stride;
    fa.preds = pred_p;
    fa.q = q;
    fa.qnorm = qnorm;
    fa.B = B;
    fa.metric = metric;
    fa.k = kmax;
    fa.ks = kc_p;
    fa.kmax = kmax;
    fa.kprime = P.kprime;
    fa.kps = kps_p;
    fa.K = P.K;
    fa.n_chunks = std::max(NC_CAP, SEG_MAX);  // most lists of one query
    fa.partials = sa.partials;
    fa.list_off = ba.list_off;
    fa.nlists = ba.nlists;
    fa.perm = ba.perm;
    fa.merge_mid = nullptr;
    fa.merged = (uint64_t *)(w + P.o_merged);
    fa.rr_dist = (double *)(w + P.o_rrdist);
    // Screening error: the larger of the two kernels' models (the sparse
    // kernel is the VALU form with IEEE round-to-nearest, unit roundoff
    // 2^-24; the dense one the MFMA form, whose internal rounding is only
    // assumed faithful, unit roundoff 2^-23).
    const double u32 = ldexp(1.0, -24), u64 = ldexp(1.0, -53), um = ldexp(1.0, -23);
    const double g = (gamma_n(t->dp + 3, u32) + gamma_n(t->dp + 3, u64)) * 1.001;
    const double g6 = (gamma_n(t->dp + 6, um) + gamma_n(t->dp + 3, u64)) * 1.001;
    const double gb = (gamma_n(t->dp + 2, um) * (1.0 + ldexp(1.0, -7)) + ldexp(1.0, -16) + 3.0 * um +
                       gamma_n(t->dp + 2, u64)) * 1.001;
    fa.rel = metric == VRS_L2SQ ? g : 0.0;
    fa.abs_l2 = metric == VRS_L2SQ ? g6 : 0.0;
    fa.abs_ip = metric == VRS_IP ? (t->store == VRS_F32 ? g6 : std::max(g6, gb)) : 0.0;
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
    // Dense side in two passes (as in the single-predicate scan): a prefix of
    // every chunk, a merge of the dense positions' lists whose (k'+1)-th key
    // then bounds each dense query, every chunk in full with fresh lists.
    auto dense = [&]() -> hipError_t {
        return t->store == VRS_F32 ? launch_screen_mfma_persistent(sa, 64, P.dense_grid, s)
                                   : launch_screen_mfma_bf16_persistent(sa, P.dense_grid, s);
    };
    prof_begin(2, s);
    if (P.two_pass) {
        sa.pass = 1;
        // a dense query keeps more than cap_frac of the rows (at least 1/1024)
        sa.prefix_sel = (float)std::max(kCfgs[cfg].cap_frac, 1.0 / 1024);
        if ((e = dense()) != hipSuccess) return e;
        prof_end(2, s);
        prof_begin(3, s);
        fa.merge_limit = ctl + BC_NDENSE;
        if ((e = launch_merge(fa, s)) != hipSuccess) return e;
        // the bound, and fresh work queues for the second pass
        if ((e = launch_set_bound(fa, gthr, ctl + BC_QDENSE, s)) != hipSuccess) return e;
        fa.merge_limit = nullptr;
        prof_end(3, s);
        prof_begin(2, s);
        sa.pass = 2;
    }
    if ((e = dense()) != hipSuccess) return e;
    if (ba.rows_cap > 0) {
        e = launch_screen_sparse(sa, P.sparse_grid, s);
        if (e != hipSuccess) return e;
    }
    prof_end(2, s);

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

hipError_t batched_tune(const vrs_table_s *t, const float *q, int B, const vrs_pred *preds,
                        const int32_t *ks, int kmax, vrs_metric metric, int64_t *out_idx,
                        float *out_dist, void *ws, const vrs_opts *opts, hipStream_t s, int *best,
                        float *ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int bi = -1;
    float bt = 0.0f;
    for (int c = 0; c < kNumCfgs && e == hipSuccess; ++c) {
        // one untimed run, then the best of two timed runs
        e = run_batched(t, q, B, preds, ks, kmax, metric, out_idx, out_dist, ws, opts, c, s);
        float tc = -1.0f;
        for (int r = 0; r < 2 && e == hipSuccess; ++r) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess)
                e = run_batched(t, q, B, preds, ks, kmax, metric, out_idx, out_dist, ws, opts, c, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float x = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&x, e0, e1);
            if (e == hipSuccess && (tc < 0.0f || x < tc)) tc = x;
        }
        if (ms) ms[c] = tc;
        if (e == hipSuccess && (bi < 0 || tc < bt)) {
            bi = c;
            bt = tc;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tuned[tune_key(t, B, kmax, metric, opts)] = bi;
    }
    // leave the outputs as the chosen configuration computes them
    e = run_batched(t, q, B, preds, ks, kmax, metric, out_idx, out_dist, ws, opts, bi, s);
    *best = bi;
    return e;
}

}  // namespace vrs
