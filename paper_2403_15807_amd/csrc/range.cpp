// range.cpp -- host side of the threshold selection (vrs_scan_range):
// workspace layout, strategy (mask or gather, eq. 3), screening error model
// and the launch sequence of k_range.hip.
#include <math.h>

#include <algorithm>

#include "internal.h"
#include "planner.h"

namespace vrs {

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
double gamma_n(double n, double u) { return n * u / (1.0 - n * u); }

struct RangePlan {
    int64_t words, nblk, nblk_sel;
    int32_t cap_c;
    size_t o_qp, o_qnorm, o_qn2, o_gthr, o_failcnt, o_tf, o_cnt, o_ovf, o_ovfcnt, o_cand, o_bitmap,
        o_blk, o_selbm, o_selblk, o_sel, o_selcnt, total;
};

RangePlan range_plan(const vrs_table_s *t, int B, int cap) {
    RangePlan P{};
    P.words = ((t->n + 31) / 32 + 1) / 2 * 2;
    P.nblk = (t->n + RANGE_BLOCK_ROWS - 1) / RANGE_BLOCK_ROWS;
    P.nblk_sel = (t->n + SEL_BLOCK_ROWS - 1) / SEL_BLOCK_ROWS;
    // candidate slots per query: at least 64K (and 4 per output slot), at
    // most every row (then no query can overflow)
    P.cap_c = (int32_t)std::min<int64_t>(t->n, std::max<int64_t>(65536, 4 * (int64_t)cap));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += a256(bytes);
        return r;
    };
    P.o_qp = take((size_t)B * t->dp * 4);
    P.o_qnorm = take((size_t)B * 8);
    P.o_qn2 = take((size_t)B * 4);
    P.o_gthr = take((size_t)B * 8);
    P.o_failcnt = take(8);
    P.o_tf = take((size_t)B * 4);
    P.o_cnt = take((size_t)B * 4);
    P.o_ovf = take((size_t)B * 4);
    P.o_ovfcnt = take(8);
    P.o_cand = take((size_t)B * P.cap_c * 4);
    P.o_bitmap = take((size_t)B * P.words * 4);
    P.o_blk = take((size_t)B * P.nblk * 4);
    P.o_selbm = take((size_t)(t->n + 31) / 32 * 4);
    P.o_selblk = take((size_t)P.nblk_sel * 4);
    P.o_sel = take((size_t)t->n * 4);
    P.o_selcnt = take(8);
    P.total = o;
    return P;
}

}  // namespace

size_t range_workspace(const vrs_table_s *t, int B, int cap) { return range_plan(t, B, cap).total; }

hipError_t run_range(const vrs_table_s *t, const float *q, int B, const PredDev &p, vrs_metric metric,
                     const double *thr, int cap, int64_t *out_idx, float *out_dist, int64_t *out_count,
                     void *ws, const vrs_opts *opts, hipStream_t s) {
    const RangePlan P = range_plan(t, B, cap);
    char *w = (char *)ws;
    // strategy: the caller's, else gather below half of the rows (estimate)
    int strategy = opts ? opts->strategy : VRS_STRATEGY_AUTO;
    if (strategy == VRS_STRATEGY_AUTO)
        strategy = estimate_selectivity(t, p) < 0.5 ? VRS_STRATEGY_GATHER : VRS_STRATEGY_MASK;
    const bool gather = strategy == VRS_STRATEGY_GATHER;
    RangeArgs a{};
    a.rows = t->rows;
    a.scale = t->scale;
    a.n = t->n;
    a.d = t->d;
    a.dp = t->dp;
    a.store = t->store;
    a.attr = t->attr;
    a.an = t->attr_stride;
    a.pred = p;
    a.sel_ids = (int32_t *)(w + P.o_sel);
    a.sel_count = (int64_t *)(w + P.o_selcnt);
    a.gather = gather;
    a.q = q;
    a.qp = (float *)(w + P.o_qp);
    a.qnorm = (double *)(w + P.o_qnorm);
    a.B = B;
    a.metric = metric;
    a.thr = thr;
    a.tf = (float *)(w + P.o_tf);
    // Screening error of the VALU kernel (IEEE fused multiply-adds rounded to
    // nearest, any order of the partial sums), with the FP64 sum's own error:
    //   L2SQ: relative gamma_{dp+3};  IP: absolute gamma_{dp+6} |q| max|x|.
    const double u32 = ldexp(1.0, -24), u64 = ldexp(1.0, -53);
    a.rel = metric == VRS_L2SQ ? (gamma_n(t->dp + 3, u32) + gamma_n(t->dp + 3, u64)) * 1.001 : 0.0;
    a.abs_ip = metric == VRS_IP ? (gamma_n(t->dp + 6, u32) + gamma_n(t->dp + 3, u64)) * 1.001 : 0.0;
    a.abs_l2 = 0.0;
    a.max_norm = t->max_norm;
    const int qt = B >= 8 ? 8 : (B >= 4 ? 4 : (B >= 2 ? 2 : 1));
    const int qg = (B + qt - 1) / qt;
    const int64_t rows = gather ? std::max<int64_t>(1, (int64_t)(estimate_selectivity(t, p) * t->n)) : t->n;
    // (at most 1024 workgroups per query group: 2048 ran as one full round
    // of resident workgroups and a partial second one, 2 % slower)
    a.n_chunks = (int)std::max<int64_t>(1, std::min<int64_t>((rows + 1023) / 1024, 1024 / qg));
    a.cap_c = P.cap_c;
    a.cnt = (uint32_t *)(w + P.o_cnt);
    a.cand = (int32_t *)(w + P.o_cand);
    a.ovf_list = (int32_t *)(w + P.o_ovf);
    a.ovf_count = (int32_t *)(w + P.o_ovfcnt);
    a.fb_chunks = (int)std::max<int64_t>(1, std::min<int64_t>((t->n + 16383) / 16384, 4096));
    a.bitmap = (uint32_t *)(w + P.o_bitmap);
    a.words = P.words;
    a.blkcnt = (uint32_t *)(w + P.o_blk);
    a.nblk = (int32_t)P.nblk;
    a.cap = cap;
    a.out_idx = out_idx;
    a.out_dist = out_dist;
    a.out_count = out_count;

    hipError_t e;
    prof_begin(0, s);
    if ((e = launch_prep_queries(q, B, t->d, t->dp, (float *)a.qp, (double *)a.qnorm, (float *)(w + P.o_qn2),
                                 nullptr, (uint64_t *)(w + P.o_gthr), (int32_t *)(w + P.o_failcnt), nullptr,
                                 0, s)) != hipSuccess)
        return e;
    if ((e = launch_range(a, qt, 0, s)) != hipSuccess) return e;
    prof_end(0, s);
    if (gather) {
        prof_begin(1, s);
        if ((e = launch_select(t->attr, t->n, t->attr_stride, p, (uint32_t *)(w + P.o_selbm),
                               (uint32_t *)(w + P.o_selblk), (int32_t *)a.sel_ids, (int64_t *)a.sel_count,
                               s)) != hipSuccess)
            return e;
        prof_end(1, s);
    }
    prof_begin(2, s);
    if ((e = launch_range(a, qt, 1, s)) != hipSuccess) return e;
    prof_end(2, s);
    prof_begin(3, s);
    if ((e = launch_range(a, qt, 2, s)) != hipSuccess) return e;
    prof_end(3, s);
    prof_begin(4, s);
    if ((e = launch_range(a, qt, 3, s)) != hipSuccess) return e;
    prof_end(4, s);
    return hipSuccess;
}

}  // namespace vrs
