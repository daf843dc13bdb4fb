// api.cpp -- the C ABI of include/vrs.h: argument validation, table
// ownership, the access-path planner, workspace carving and the launch
// sequence of a scan.  Host code only; kernels live in k_*.hip.
//
// A scan of B queries runs, all asynchronously on the caller's stream:
//   prep      -> pad queries, FP64 query norms, reset the fallback counter
//   [select]  -> gather strategy only: predicate -> selection vector
//   screen    -> per (query tile, row chunk): K smallest FP32 screening keys
//   merge     -> per query: K smallest keys over all chunks
//   rerank    -> per query: FP64 distances of the k' survivors, (dist, id)
//                order, certificate against the (k'+1)-th screening key
//   fallback  -> exact FP64 scan for the queries whose certificate failed
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>

#include "internal.h"
#include "planner.h"

using namespace vrs;

namespace {

thread_local std::string g_err;

vrs_status fail(vrs_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
vrs_status fail(vrs_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

vrs_status ok() {
    g_err.clear();
    return VRS_OK;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(VRS_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));             \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Host-side fold of an ABI predicate into inclusive int32 ranges.
vrs_status fold_pred(const vrs_pred *p, int n_attr, PredDev *out) {
    PredDev o{};
    o.nterms = 0;
    for (int t = 0; t < 4; ++t) {
        o.col[t] = 0;
        o.lo[t] = 0;
        o.hi[t] = -1;
    }
    if (!p) {
        *out = o;
        return VRS_OK;
    }
    if (p->nterms < 0 || p->nterms > VRS_MAX_TERMS)
        return fail(VRS_E_ARG, "pred.nterms=%d outside [0,%d]", p->nterms, VRS_MAX_TERMS);
    bool empty = false;
    for (int t = 0; t < p->nterms; ++t) {
        const vrs_range &r = p->term[t];
        if (r.col < 0 || r.col >= n_attr)
            return fail(VRS_E_ARG, "pred.term[%d].col=%d outside [0,%d)", t, r.col, n_attr);
        int64_t lo = r.lo, hi = r.hi;
        if (hi <= lo || hi <= (int64_t)INT32_MIN || lo > (int64_t)INT32_MAX) {
            empty = true;
            continue;
        }
        o.col[t] = r.col;
        o.lo[t] = (int32_t)std::max<int64_t>(lo, INT32_MIN);
        o.hi[t] = (int32_t)std::min<int64_t>(hi - 1, INT32_MAX);
    }
    o.nterms = empty ? -1 : p->nterms;
    *out = o;
    return VRS_OK;
}

}  // namespace

namespace vrs {

// Status and message of a failed call, for entry points in other files.
vrs_status set_error(vrs_status st, const char *msg) { return fail(st, "%s", msg); }

int elem_bytes(vrs_dtype t) { return t == VRS_F32 ? 4 : (t == VRS_BF16 ? 2 : 1); }

// Rows are zero-padded so that a row is a whole number of 128-byte blocks.
int pad_dim(int d, vrs_dtype t) {
    int per = 128 / elem_bytes(t);
    return (d + per - 1) / per * per;
}

// Estimated fraction of rows satisfying `p` from the per-column histograms,
// assuming independent columns.
double estimate_selectivity(const vrs_table_s *t, const PredDev &p) {
    if (p.nterms < 0) return 0.0;
    double sel = 1.0;
    for (int k = 0; k < p.nterms; ++k) {
        int c = p.col[k];
        const int64_t lo = t->amin[c], span = (int64_t)t->amax[c] - lo + 1;
        double hit = 0.0, tot = 0.0;
        for (int b = 0; b < HIST_BINS; ++b) {
            // values v with floor((v - lo) * BINS / span) == b
            int64_t v0 = lo + (b * span + HIST_BINS - 1) / HIST_BINS;
            int64_t v1 = lo + ((b + 1) * span + HIST_BINS - 1) / HIST_BINS;  // exclusive
            double cntb = t->hist[c][b];
            tot += cntb;
            if (v1 <= v0 || cntb == 0) continue;
            int64_t a = std::max<int64_t>(v0, p.lo[k]), z = std::min<int64_t>(v1 - 1, p.hi[k]);
            if (z >= a) hit += cntb * (double)(z - a + 1) / (double)(v1 - v0);
        }
        sel *= tot > 0 ? hit / tot : 0.0;
    }
    return sel;
}

}  // namespace vrs

// ====================================================================== API
extern "C" {

const char *vrs_last_error(void) { return g_err.c_str(); }

vrs_status vrs_build_table(const float *vec, int64_t n, int32_t d, const int32_t *attr,
                           int32_t n_attr, vrs_dtype store, int32_t normalize, void *stream,
                           vrs_table *out) {
    if (!out) return fail(VRS_E_ARG, "out is NULL");
    *out = nullptr;
    if (!vec) return fail(VRS_E_ARG, "vec is NULL");
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(VRS_E_ARG, "n=%lld outside [1, 2^31)", (long long)n);
    if (d < 1 || d > 4096) return fail(VRS_E_ARG, "d=%d outside [1, 4096]", d);
    if (n_attr < 0 || n_attr > 64) return fail(VRS_E_ARG, "n_attr=%d outside [0, 64]", n_attr);
    if (n_attr > 0 && !attr) return fail(VRS_E_ARG, "attr is NULL with n_attr=%d", n_attr);
    if (store != VRS_F32 && store != VRS_BF16 && store != VRS_FP8E4M3)
        return fail(VRS_E_ARG, "unknown storage dtype %d", (int)store);
    hipStream_t s = (hipStream_t)stream;
    auto *t = new vrs_table_s();
    t->n = n;
    t->d = d;
    t->dp = pad_dim(d, store);
    t->n_attr = n_attr;
    t->attr_stride = n;
    t->store = store;
    HIP_TRY(hipGetDevice(&t->device));
    auto cleanup = [&]() { vrs_destroy_table(t); };
    size_t rows_bytes = (size_t)n * t->dp * elem_bytes(store);
    void *scratch = nullptr;
    size_t hist_words = (size_t)std::max(n_attr, 1) * HIST_BINS;
    size_t scratch_bytes = 16 + 16 + 2 * 4 * 64 + hist_words * 4;
    if (hipMalloc(&t->rows, rows_bytes) != hipSuccess ||
        hipMalloc((void **)&t->norm2, (size_t)n * 4) != hipSuccess ||
        (store == VRS_FP8E4M3 && hipMalloc((void **)&t->scale, (size_t)n * 4) != hipSuccess) ||
        (n_attr > 0 && hipMalloc((void **)&t->attr, (size_t)n * n_attr * 4) != hipSuccess) ||
        hipMalloc(&scratch, scratch_bytes) != hipSuccess) {
        (void)hipGetLastError();
        if (scratch) (void)hipFree(scratch);
        cleanup();
        return fail(VRS_E_NOMEM, "device allocation of %zu bytes failed", rows_bytes);
    }
    unsigned long long *mx = (unsigned long long *)scratch;
    int *bad = (int *)((char *)scratch + 16);
    int32_t *amin = (int32_t *)((char *)scratch + 32);
    int32_t *amax = amin + 64;
    uint32_t *hist = (uint32_t *)(amax + 64);
    hipError_t e = hipMemsetAsync(scratch, 0, 32, s);
    if (e == hipSuccess && n_attr > 0)
        e = hipMemcpyAsync(t->attr, attr, (size_t)n * n_attr * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = launch_build_rows(vec, n, d, t->dp, store, normalize, t->rows, t->scale, t->norm2, mx,
                              bad, s);
    if (e == hipSuccess) e = launch_attr_stats(t->attr, n, n_attr, amin, amax, hist, s);
    unsigned long long mxh = 0;
    int badh = 0;
    std::vector<int32_t> hmin(std::max(n_attr, 1)), hmax(std::max(n_attr, 1));
    std::vector<uint32_t> hh(hist_words);
    if (e == hipSuccess) e = hipMemcpyAsync(&mxh, mx, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&badh, bad, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && n_attr > 0) {
        e = hipMemcpyAsync(hmin.data(), amin, 4 * n_attr, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(hmax.data(), amax, 4 * n_attr, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(hh.data(), hist, hist_words * 4, hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the build's one host sync
    // the column statistics stay on the device for estimates made inside
    // batched launches
    t->stats_alloc = scratch;
    t->dstats = (char *)scratch + 32;
    if (e != hipSuccess) {
        cleanup();
        return fail(VRS_E_HIP, "table build failed: %s", hipGetErrorString(e));
    }
    if (badh) {
        cleanup();
        return fail(VRS_E_NONFINITE, "the table holds a non-finite value (or overflows the storage type)");
    }
    double mxd;
    memcpy(&mxd, &mxh, 8);
    t->max_norm = mxd;
    for (int c = 0; c < n_attr; ++c) {
        t->amin.push_back(hmin[c]);
        t->amax.push_back(hmax[c]);
        t->hist.emplace_back(hh.begin() + (size_t)c * HIST_BINS, hh.begin() + (size_t)(c + 1) * HIST_BINS);
    }
    *out = t;
    return ok();
}

vrs_status vrs_destroy_table(vrs_table t) {
    if (!t) return fail(VRS_E_ARG, "table is NULL");
    if (!t->owner) {
        delete t;
        return ok();
    }
    if (t->rows) (void)hipFree(t->rows);
    if (t->scale) (void)hipFree(t->scale);
    if (t->norm2) (void)hipFree(t->norm2);
    if (t->attr) (void)hipFree(t->attr);
    if (t->stats_alloc) (void)hipFree(t->stats_alloc);
    delete t;
    return ok();
}

vrs_status vrs_table_info(vrs_table t, int64_t *n, int32_t *d, int32_t *n_attr, vrs_dtype *store,
                          double *max_row_norm) {
    if (!t) return fail(VRS_E_ARG, "table is NULL");
    if (n) *n = t->n;
    if (d) *d = t->d;
    if (n_attr) *n_attr = t->n_attr;
    if (store) *store = t->store;
    if (max_row_norm) *max_row_norm = t->max_norm;
    return ok();
}

vrs_status vrs_table_export(vrs_table t, void *rows_out, float *scale_out, void *stream) {
    if (!t) return fail(VRS_E_ARG, "table is NULL");
    if (!rows_out) return fail(VRS_E_ARG, "rows_out is NULL");
    if (t->store == VRS_FP8E4M3 && !scale_out) return fail(VRS_E_ARG, "scale_out is NULL for an FP8 table");
    hipStream_t s = (hipStream_t)stream;
    const size_t eb = elem_bytes(t->store);
    HIP_TRY(hipMemcpy2DAsync(rows_out, t->d * eb, t->rows, t->dp * eb, t->d * eb, t->n,
                             hipMemcpyDeviceToDevice, s));
    if (t->store == VRS_FP8E4M3)
        HIP_TRY(hipMemcpyAsync(scale_out, t->scale, t->n * 4, hipMemcpyDeviceToDevice, s));
    return ok();
}

vrs_status vrs_select_workspace_bytes(vrs_table t, size_t *bytes) {
    if (!t || !bytes) return fail(VRS_E_ARG, "NULL argument");
    int64_t nblk = (t->n + SEL_BLOCK_ROWS - 1) / SEL_BLOCK_ROWS;
    *bytes = align256((t->n + 31) / 32 * 4) + align256(nblk * 4);
    return ok();
}

vrs_status vrs_select(vrs_table t, const vrs_pred *pred, int32_t *ids_out, int64_t *count_out,
                      void *ws, size_t ws_bytes, void *stream) {
    if (!t) return fail(VRS_E_ARG, "table is NULL");
    if (!ids_out || !count_out) return fail(VRS_E_ARG, "output is NULL");
    size_t need;
    vrs_select_workspace_bytes(t, &need);
    if (!ws || ws_bytes < need) return fail(VRS_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    PredDev p;
    vrs_status st = fold_pred(pred, t->n_attr, &p);
    if (st != VRS_OK) return st;
    uint32_t *bitmap = (uint32_t *)ws;
    uint32_t *blk = (uint32_t *)((char *)ws + align256((t->n + 31) / 32 * 4));
    HIP_TRY(launch_select(t->attr, t->n, t->attr_stride, p, bitmap, blk, ids_out, count_out,
                          (hipStream_t)stream));
    return ok();
}

int32_t vrs_num_tiles(void) { return planner_num_tiles(); }

vrs_status vrs_profile(int32_t enable) {
    prof_enable(enable != 0);
    return ok();
}

vrs_status vrs_stage_times(double *ms, int64_t *calls) {
    if (!ms || !calls) return fail(VRS_E_ARG, "NULL output");
    hipError_t e = prof_collect(ms, calls);
    if (e != hipSuccess) return fail(VRS_E_HIP, "stage timing failed: %s", hipGetErrorString(e));
    return ok();
}

vrs_status vrs_chooser_load(const char *path) {
    std::string err;
    if (!chooser_load(path, &err)) return fail(VRS_E_ARG, "%s", err.c_str());
    return ok();
}

vrs_status vrs_chooser_set(const float *params, const float *feat_mean, const float *feat_std) {
    if (!params || !feat_mean || !feat_std) return fail(VRS_E_ARG, "NULL argument");
    if (!chooser_set(params, feat_mean, feat_std))
        return fail(VRS_E_ARG, "chooser weights must be finite and std > 0");
    return ok();
}

vrs_status vrs_chooser_pick(const float *feats, const uint8_t *allowed, int32_t *arm) {
    if (!feats || !allowed || !arm) return fail(VRS_E_ARG, "NULL argument");
    const int n = 2 * planner_num_tiles();
    bool al[64];
    for (int i = 0; i < n; ++i) al[i] = allowed[i] != 0;
    *arm = chooser_pick(feats, al, n);
    return ok();
}

vrs_status vrs_chooser_clear(void) {
    chooser_clear();
    return ok();
}

vrs_status vrs_plan(vrs_table t, int32_t B, const vrs_pred *pred, int32_t k, vrs_metric metric,
                    const vrs_opts *opts, float *features, int32_t *strategy, int32_t *tile) {
    if (!t) return fail(VRS_E_ARG, "table is NULL");
    if (B < 1 || B > VRS_MAX_BATCH || k < 1 || k > 256) return fail(VRS_E_ARG, "bad B or k");
    PredDev p;
    vrs_status st = fold_pred(pred, t->n_attr, &p);
    if (st != VRS_OK) return st;
    float f[6];
    int s_, t_;
    plan_decide(t, B, p, false, k, metric, opts, f, &s_, &t_);
    if (features)
        for (int i = 0; i < 6; ++i) features[i] = f[i];
    if (strategy) *strategy = s_;
    if (tile) *tile = t_;
    return ok();
}

vrs_status vrs_table_view(vrs_table t, int64_t n, vrs_table *out) {
    if (!t || !out) return fail(VRS_E_ARG, "NULL argument");
    if (n < 1 || n > t->n) return fail(VRS_E_ARG, "view rows %lld outside [1, %lld]", (long long)n, (long long)t->n);
    auto *v = new vrs_table_s(*t);
    v->n = n;
    v->owner = false;
    *out = v;
    return ok();
}

vrs_status vrs_mlp_forward(const float *params, const float *x, int32_t nb, float *y, float *act,
                           void *stream) {
    if (!params || !x || !y || nb < 1) return fail(VRS_E_ARG, "bad MLP forward arguments");
    HIP_TRY(launch_mlp_forward(params, x, nb, y, act, (hipStream_t)stream));
    return ok();
}

vrs_status vrs_mlp_backward(const float *params, const float *x, const float *y,
                            const float *act, const float *target, const uint8_t *mask,
                            int32_t nb, int32_t count, float *sig, float *sqerr, float *grad,
                            float *loss, void *stream) {
    if (!params || !x || !y || !act || !target || !mask || !sig || !sqerr || !grad || nb < 1 || count < 1)
        return fail(VRS_E_ARG, "bad MLP backward arguments");
    HIP_TRY(launch_mlp_backward(params, x, y, act, target, mask, nb, 1.0f / (float)count, sig,
                                sqerr, grad, loss, (hipStream_t)stream));
    return ok();
}

vrs_status vrs_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t step,
                        float lr, float beta1, float beta2, float eps, void *stream) {
    if (!params || !grad || !m || !v || step < 1) return fail(VRS_E_ARG, "bad Adam arguments");
    HIP_TRY(launch_mlp_adam(params, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream));
    return ok();
}

vrs_status vrs_scan_workspace_bytes(vrs_table t, int32_t B, int32_t k_max, const vrs_opts *opts,
                                    size_t *bytes) {
    if (!t || !bytes) return fail(VRS_E_ARG, "NULL argument");
    if (B < 1 || B > VRS_MAX_BATCH) return fail(VRS_E_ARG, "B=%d outside [1, %d]", B, VRS_MAX_BATCH);
    if (k_max < 1 || k_max > 256) return fail(VRS_E_ARG, "k=%d outside [1, 256]", k_max);
    *bytes = plan_workspace(t, B, k_max, opts);
    return ok();
}

static vrs_status scan_common(vrs_table t, const float *q, int32_t B, const vrs_pred *pred,
                              const vrs_pred *preds, const int32_t *ks, int32_t k,
                              vrs_metric metric, int64_t *out_idx, float *out_dist, void *ws,
                              size_t ws_bytes, const vrs_opts *opts, void *stream) {
    if (!t) return fail(VRS_E_ARG, "table is NULL");
    if (!q) return fail(VRS_E_ARG, "queries are NULL");
    if (!out_idx || !out_dist) return fail(VRS_E_ARG, "outputs are NULL");
    if (B < 1 || B > VRS_MAX_BATCH) return fail(VRS_E_ARG, "B=%d outside [1, %d]", B, VRS_MAX_BATCH);
    if (k < 1 || k > 256) return fail(VRS_E_ARG, "k=%d outside [1, 256]", k);
    if (metric != VRS_L2SQ && metric != VRS_IP) return fail(VRS_E_ARG, "unknown metric %d", (int)metric);
    if (metric == VRS_L2SQ && t->store != VRS_F32)
        return fail(VRS_E_UNSUPPORTED, "L2SQ needs a float32 table (bfloat16/FP8 tables support IP)");
    if (opts && (opts->strategy < 0 || opts->strategy > 2))
        return fail(VRS_E_ARG, "opts.strategy=%d outside [0, 2]", opts->strategy);
    if (opts && (opts->tile < -1 || opts->tile >= planner_num_tiles()))
        return fail(VRS_E_ARG, "opts.tile=%d outside [-1, %d)", opts->tile, planner_num_tiles());
    if (opts && (opts->kprime_mult < 0 || opts->kprime_mult > 64))
        return fail(VRS_E_ARG, "opts.kprime_mult=%d outside [0, 64]", opts->kprime_mult);
    if (preds && !ks) return fail(VRS_E_ARG, "ks is NULL");
    PredDev p;
    if (!preds) {
        vrs_status st = fold_pred(pred, t->n_attr, &p);
        if (st != VRS_OK) return st;
    } else {
        fold_pred(nullptr, t->n_attr, &p);
    }
    size_t need = plan_workspace(t, B, k, opts);
    if (!ws || ws_bytes < need)
        return fail(VRS_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    if (((uintptr_t)ws & 255) != 0) return fail(VRS_E_WORKSPACE, "workspace not 256-byte aligned");
    hipError_t e = run_scan(t, q, B, p, preds, ks, k, metric, out_idx, out_dist, ws, opts,
                            (hipStream_t)stream);
    if (e != hipSuccess) return fail(VRS_E_HIP, "scan launch failed: %s", hipGetErrorString(e));
    return ok();
}

vrs_status vrs_scan_topk(vrs_table t, const float *q, int32_t B, const vrs_pred *pred, int32_t k,
                         vrs_metric metric, int64_t *out_idx, float *out_dist, void *ws,
                         size_t ws_bytes, const vrs_opts *opts, void *stream) {
    return scan_common(t, q, B, pred, nullptr, nullptr, k, metric, out_idx, out_dist, ws, ws_bytes,
                       opts, stream);
}

vrs_status vrs_range_workspace_bytes(vrs_table t, int32_t B, int32_t cap, size_t *bytes) {
    if (!t || !bytes) return fail(VRS_E_ARG, "NULL argument");
    if (B < 1 || B > VRS_MAX_BATCH) return fail(VRS_E_ARG, "B=%d outside [1, %d]", B, VRS_MAX_BATCH);
    if (cap < 1) return fail(VRS_E_ARG, "cap=%d < 1", cap);
    *bytes = range_workspace(t, B, cap);
    return ok();
}

vrs_status vrs_scan_range(vrs_table t, const float *q, int32_t B, const vrs_pred *pred,
                          vrs_metric metric, const double *thr, int32_t cap, int64_t *out_idx,
                          float *out_dist, int64_t *out_count, void *ws, size_t ws_bytes,
                          const vrs_opts *opts, void *stream) {
    if (!t) return fail(VRS_E_ARG, "table is NULL");
    if (!q || !thr) return fail(VRS_E_ARG, "queries or thresholds are NULL");
    if (!out_idx || !out_dist || !out_count) return fail(VRS_E_ARG, "outputs are NULL");
    if (B < 1 || B > VRS_MAX_BATCH) return fail(VRS_E_ARG, "B=%d outside [1, %d]", B, VRS_MAX_BATCH);
    if (cap < 1) return fail(VRS_E_ARG, "cap=%d < 1", cap);
    if (metric != VRS_L2SQ && metric != VRS_IP) return fail(VRS_E_ARG, "unknown metric %d", (int)metric);
    if (metric == VRS_L2SQ && t->store != VRS_F32)
        return fail(VRS_E_UNSUPPORTED, "L2SQ needs a float32 table (bfloat16/FP8 tables support IP)");
    if (opts && (opts->strategy < 0 || opts->strategy > 2))
        return fail(VRS_E_ARG, "opts.strategy=%d outside [0, 2]", opts->strategy);
    PredDev p;
    vrs_status st = fold_pred(pred, t->n_attr, &p);
    if (st != VRS_OK) return st;
    const size_t need = range_workspace(t, B, cap);
    if (!ws || ws_bytes < need) return fail(VRS_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    if (((uintptr_t)ws & 255) != 0) return fail(VRS_E_WORKSPACE, "workspace not 256-byte aligned");
    hipError_t e = run_range(t, q, B, p, metric, thr, cap, out_idx, out_dist, out_count, ws, opts,
                             (hipStream_t)stream);
    if (e != hipSuccess) return fail(VRS_E_HIP, "range launch failed: %s", hipGetErrorString(e));
    return ok();
}

vrs_status vrs_join_workspace_bytes(vrs_table R, vrs_table S, int32_t k, const vrs_opts *opts,
                                    size_t *bytes) {
    if (!R || !S || !bytes) return fail(VRS_E_ARG, "NULL argument");
    if (k < 1 || k > 256) return fail(VRS_E_ARG, "k=%d outside [1, 256]", k);
    if (R->d != S->d) return fail(VRS_E_ARG, "R has d=%d, S has d=%d", R->d, S->d);
    *bytes = join_workspace(R, S, k, opts);
    return ok();
}

vrs_status vrs_join_topk(vrs_table R, vrs_table S, const vrs_pred *pred, int32_t k, vrs_metric metric,
                         int64_t *out_idx, float *out_dist, void *ws, size_t ws_bytes,
                         const vrs_opts *opts, void *stream) {
    if (!R || !S) return fail(VRS_E_ARG, "table is NULL");
    if (!out_idx || !out_dist) return fail(VRS_E_ARG, "outputs are NULL");
    if (R->d != S->d) return fail(VRS_E_ARG, "R has d=%d, S has d=%d", R->d, S->d);
    if (k < 1 || k > 256) return fail(VRS_E_ARG, "k=%d outside [1, 256]", k);
    if (metric != VRS_L2SQ && metric != VRS_IP) return fail(VRS_E_ARG, "unknown metric %d", (int)metric);
    if (metric == VRS_L2SQ && S->store != VRS_F32)
        return fail(VRS_E_UNSUPPORTED, "L2SQ needs a float32 table S (bfloat16/FP8 tables support IP)");
    if (opts && (opts->strategy < 0 || opts->strategy > 2))
        return fail(VRS_E_ARG, "opts.strategy=%d outside [0, 2]", opts->strategy);
    if (opts && (opts->tile < -1 || opts->tile >= planner_num_tiles()))
        return fail(VRS_E_ARG, "opts.tile=%d outside [-1, %d)", opts->tile, planner_num_tiles());
    if (opts && (opts->kprime_mult < 0 || opts->kprime_mult > 64))
        return fail(VRS_E_ARG, "opts.kprime_mult=%d outside [0, 64]", opts->kprime_mult);
    PredDev p;
    vrs_status st = fold_pred(pred, S->n_attr, &p);
    if (st != VRS_OK) return st;
    const size_t need = join_workspace(R, S, k, opts);
    if (!ws || ws_bytes < need) return fail(VRS_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    if (((uintptr_t)ws & 255) != 0) return fail(VRS_E_WORKSPACE, "workspace not 256-byte aligned");
    hipError_t e = run_join(R, S, p, k, metric, out_idx, out_dist, ws, opts, (hipStream_t)stream);
    if (e != hipSuccess) return fail(VRS_E_HIP, "join launch failed: %s", hipGetErrorString(e));
    return ok();
}

vrs_status vrs_index_build(vrs_table t, int32_t nlist, int32_t iters, void *stream, vrs_index *out) {
    if (!t || !out) return fail(VRS_E_ARG, "NULL argument");
    if (nlist < 1 || nlist > 16384 || nlist > t->n)
        return fail(VRS_E_ARG, "nlist=%d outside [1, min(16384, n)]", nlist);
    if (iters < 0 || iters > 100) return fail(VRS_E_ARG, "iters=%d outside [0, 100]", iters);
    std::string err;
    vrs_index_s *ix = nullptr;
    hipError_t e = index_build(t, nlist, iters, (hipStream_t)stream, &ix, &err);
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? VRS_E_NOMEM : VRS_E_HIP, "index build: %s", err.c_str());
    *out = ix;
    return ok();
}

vrs_status vrs_index_destroy(vrs_index ix) {
    if (!ix) return fail(VRS_E_ARG, "index is NULL");
    index_free(ix);
    return ok();
}

vrs_status vrs_index_info(vrs_index ix, int32_t *nlist, int64_t *max_list) {
    if (!ix) return fail(VRS_E_ARG, "index is NULL");
    if (nlist) *nlist = ix->nlist;
    if (max_list) *max_list = ix->max_list;
    return ok();
}

vrs_status vrs_index_export(vrs_index ix, float *centroids, int64_t *list_off, int32_t *list_ids,
                            void *stream) {
    if (!ix) return fail(VRS_E_ARG, "index is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (centroids)
        HIP_TRY(hipMemcpyAsync(centroids, ix->cent, (size_t)ix->nlist * ix->d * 4, hipMemcpyDeviceToDevice, s));
    if (list_off)
        HIP_TRY(hipMemcpyAsync(list_off, ix->list_off, (size_t)(ix->nlist + 1) * 8, hipMemcpyDeviceToDevice, s));
    if (list_ids)
        HIP_TRY(hipMemcpyAsync(list_ids, ix->ids, (size_t)ix->table->n * 4, hipMemcpyDeviceToDevice, s));
    return ok();
}

vrs_status vrs_plan_access(vrs_index ix, int32_t B, const vrs_pred *pred, int32_t k, int32_t nprobe,
                           int64_t cap_c, double *scan_ms, double *probe_ms, int32_t *use_probe) {
    if (!ix) return fail(VRS_E_ARG, "index is NULL");
    if (B < 1 || B > VRS_MAX_BATCH) return fail(VRS_E_ARG, "B=%d outside [1, %d]", B, VRS_MAX_BATCH);
    if (k < 1 || k > 256) return fail(VRS_E_ARG, "k=%d outside [1, 256]", k);
    if (nprobe < 1 || nprobe > std::min(256, ix->nlist))
        return fail(VRS_E_ARG, "nprobe=%d outside [1, min(256, nlist)]", nprobe);
    PredDev p;
    vrs_status st = fold_pred(pred, ix->table->n_attr, &p);
    if (st != VRS_OK) return st;
    double sc = 0.0, pr = 0.0;
    access_costs(ix, B, p, k, nprobe, std::max<int64_t>(cap_c, 1), &sc, &pr);
    if (scan_ms) *scan_ms = sc;
    if (probe_ms) *probe_ms = pr;
    if (use_probe) *use_probe = pr < sc;
    return ok();
}

vrs_status vrs_probe_workspace_bytes(vrs_index ix, int32_t B, int32_t k, int32_t nprobe, int64_t cap_c,
                                     size_t *bytes) {
    if (!ix || !bytes) return fail(VRS_E_ARG, "NULL argument");
    if (B < 1 || B > VRS_MAX_BATCH) return fail(VRS_E_ARG, "B=%d outside [1, %d]", B, VRS_MAX_BATCH);
    if (k < 1 || k > 256) return fail(VRS_E_ARG, "k=%d outside [1, 256]", k);
    if (nprobe < 1 || nprobe > std::min(256, ix->nlist))
        return fail(VRS_E_ARG, "nprobe=%d outside [1, min(256, nlist)]", nprobe);
    if (cap_c < 1) return fail(VRS_E_ARG, "cap_c=%lld < 1", (long long)cap_c);
    *bytes = probe_workspace(ix, B, k, nprobe, cap_c);
    return ok();
}

vrs_status vrs_probe_topk(vrs_index ix, const float *q, int32_t B, const vrs_pred *pred, int32_t k,
                          vrs_metric metric, int32_t nprobe, int64_t min_cand, int64_t cap_c,
                          int64_t *out_idx, float *out_dist, int32_t *out_taken, void *ws,
                          size_t ws_bytes, void *stream) {
    if (!ix) return fail(VRS_E_ARG, "index is NULL");
    if (!q) return fail(VRS_E_ARG, "queries are NULL");
    if (!out_idx || !out_dist) return fail(VRS_E_ARG, "outputs are NULL");
    size_t need = 0;
    vrs_status st = vrs_probe_workspace_bytes(ix, B, k, nprobe, cap_c, &need);
    if (st != VRS_OK) return st;
    if (min_cand < 1) return fail(VRS_E_ARG, "min_cand=%lld < 1", (long long)min_cand);
    if (metric != VRS_L2SQ && metric != VRS_IP) return fail(VRS_E_ARG, "unknown metric %d", (int)metric);
    if (metric == VRS_L2SQ && ix->table->store != VRS_F32)
        return fail(VRS_E_UNSUPPORTED, "L2SQ needs a float32 table (bfloat16/FP8 tables support IP)");
    PredDev p;
    st = fold_pred(pred, ix->table->n_attr, &p);
    if (st != VRS_OK) return st;
    if (!ws || ws_bytes < need) return fail(VRS_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    if (((uintptr_t)ws & 255) != 0) return fail(VRS_E_WORKSPACE, "workspace not 256-byte aligned");
    hipError_t e = run_probe(ix, q, B, p, k, metric, nprobe, min_cand, cap_c, out_idx, out_dist, out_taken, ws,
                             (hipStream_t)stream);
    if (e != hipSuccess) return fail(VRS_E_HIP, "probe launch failed: %s", hipGetErrorString(e));
    return ok();
}

static size_t batched_bytes(vrs_table t, int32_t B, int32_t k_max, vrs_metric metric,
                            const vrs_opts *opts) {
    if (batched_native(t, k_max, metric, opts)) return batched_workspace(t, B, k_max, metric, opts);
    vrs_opts o = opts ? *opts : vrs_opts{};
    o.tile = -1;
    return plan_workspace(t, B, k_max, &o);
}

// Argument checks of the batched entry points (everything a launch needs).
static vrs_status batched_check(vrs_table t, const float *q, int32_t B, const vrs_pred *preds,
                                const int32_t *ks, int32_t k_max, vrs_metric metric,
                                int64_t *out_idx, float *out_dist, void *ws, size_t ws_bytes,
                                const vrs_opts *opts) {
    if (!t) return fail(VRS_E_ARG, "table is NULL");
    if (!q || !preds || !ks) return fail(VRS_E_ARG, "queries, preds or ks is NULL");
    if (!out_idx || !out_dist) return fail(VRS_E_ARG, "outputs are NULL");
    if (B < 1 || B > VRS_MAX_BATCH) return fail(VRS_E_ARG, "B=%d outside [1, %d]", B, VRS_MAX_BATCH);
    if (k_max < 1 || k_max > 256) return fail(VRS_E_ARG, "k_max=%d outside [1, 256]", k_max);
    if (metric != VRS_L2SQ && metric != VRS_IP) return fail(VRS_E_ARG, "unknown metric %d", (int)metric);
    if (metric == VRS_L2SQ && t->store != VRS_F32)
        return fail(VRS_E_UNSUPPORTED, "L2SQ needs a float32 table (bfloat16/FP8 tables support IP)");
    if (opts && (opts->kprime_mult < 0 || opts->kprime_mult > 64))
        return fail(VRS_E_ARG, "opts.kprime_mult=%d outside [0, 64]", opts->kprime_mult);
    if (opts && (opts->tile < -1 || opts->tile >= batched_num_cfgs()))
        return fail(VRS_E_ARG, "opts.tile=%d outside [-1, %d)", opts->tile, batched_num_cfgs());
    const size_t need = batched_bytes(t, B, k_max, metric, opts);
    if (!ws || ws_bytes < need) return fail(VRS_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, need);
    if (((uintptr_t)ws & 255) != 0) return fail(VRS_E_WORKSPACE, "workspace not 256-byte aligned");
    return VRS_OK;
}

static hipError_t batched_run(vrs_table t, const float *q, int32_t B, const vrs_pred *preds,
                              const int32_t *ks, int32_t k_max, vrs_metric metric, int64_t *out_idx,
                              float *out_dist, void *ws, const vrs_opts *opts, int cfg,
                              hipStream_t s) {
    if (batched_native(t, k_max, metric, opts))
        return run_batched(t, q, B, preds, ks, k_max, metric, out_idx, out_dist, ws, opts, cfg, s);
    // no persistent dense kernel for this row width: the per-pair masked
    // screening of the single-predicate path, with per-query predicates
    vrs_opts o = opts ? *opts : vrs_opts{};
    o.tile = -1;
    o.strategy = VRS_STRATEGY_MASK;
    PredDev p;
    fold_pred(nullptr, t->n_attr, &p);
    return run_scan(t, q, B, p, preds, ks, k_max, metric, out_idx, out_dist, ws, &o, s);
}

vrs_status vrs_scan_topk_batched(vrs_table t, const float *q, int32_t B, const vrs_pred *preds,
                                 const int32_t *ks, int32_t k_max, vrs_metric metric,
                                 int64_t *out_idx, float *out_dist, void *ws, size_t ws_bytes,
                                 const vrs_opts *opts, void *stream) {
    vrs_status st = batched_check(t, q, B, preds, ks, k_max, metric, out_idx, out_dist, ws, ws_bytes, opts);
    if (st != VRS_OK) return st;
    const int cfg = batched_pick(t, B, k_max, metric, opts);
    hipError_t e = batched_run(t, q, B, preds, ks, k_max, metric, out_idx, out_dist, ws, opts, cfg,
                               (hipStream_t)stream);
    if (e != hipSuccess) return fail(VRS_E_HIP, "batched scan launch failed: %s", hipGetErrorString(e));
    return ok();
}

vrs_status vrs_batched_workspace_bytes(vrs_table t, int32_t B, int32_t k_max, vrs_metric metric,
                                       const vrs_opts *opts, size_t *bytes) {
    if (!t || !bytes) return fail(VRS_E_ARG, "NULL argument");
    if (B < 1 || B > VRS_MAX_BATCH) return fail(VRS_E_ARG, "B=%d outside [1, %d]", B, VRS_MAX_BATCH);
    if (k_max < 1 || k_max > 256) return fail(VRS_E_ARG, "k_max=%d outside [1, 256]", k_max);
    if (metric != VRS_L2SQ && metric != VRS_IP) return fail(VRS_E_ARG, "unknown metric %d", (int)metric);
    *bytes = batched_bytes(t, B, k_max, metric, opts);
    return ok();
}

int32_t vrs_batched_num_configs(void) { return batched_num_cfgs(); }

vrs_status vrs_batched_tune(vrs_table t, const float *q, int32_t B, const vrs_pred *preds,
                            const int32_t *ks, int32_t k_max, vrs_metric metric, int64_t *out_idx,
                            float *out_dist, void *ws, size_t ws_bytes, const vrs_opts *opts,
                            void *stream, int32_t *best, float *ms) {
    if (!best) return fail(VRS_E_ARG, "best is NULL");
    vrs_status st = batched_check(t, q, B, preds, ks, k_max, metric, out_idx, out_dist, ws, ws_bytes, opts);
    if (st != VRS_OK) return st;
    if (!batched_native(t, k_max, metric, opts))
        return fail(VRS_E_UNSUPPORTED, "no batched configurations for this table (float32 rows wider than 256)");
    int b = -1;
    hipError_t e = batched_tune(t, q, B, preds, ks, k_max, metric, out_idx, out_dist, ws, opts,
                                (hipStream_t)stream, &b, ms);
    if (e != hipSuccess) return fail(VRS_E_HIP, "batched autotuning failed: %s", hipGetErrorString(e));
    *best = b;
    return ok();
}

}  // extern "C"

struct vrs_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int cfg = -1;
    int device = 0;
};

extern "C" {

vrs_status vrs_batched_graph_create(vrs_table t, const float *q, int32_t B, const vrs_pred *preds,
                                    const int32_t *ks, int32_t k_max, vrs_metric metric,
                                    int64_t *out_idx, float *out_dist, void *ws, size_t ws_bytes,
                                    const vrs_opts *opts, void *stream, vrs_graph *out) {
    if (!out) return fail(VRS_E_ARG, "out is NULL");
    *out = nullptr;
    vrs_status st = batched_check(t, q, B, preds, ks, k_max, metric, out_idx, out_dist, ws, ws_bytes, opts);
    if (st != VRS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const bool native = batched_native(t, k_max, metric, opts);
    int cfg = batched_pick(t, B, k_max, metric, opts);
    hipError_t e = hipSuccess;
    if (native && !(opts && opts->tile >= 0) && batched_tuned(t, B, k_max, metric, opts) < 0) {
        // autotune this shape first
        int b = -1;
        e = batched_tune(t, q, B, preds, ks, k_max, metric, out_idx, out_dist, ws, opts, s, &b, nullptr);
        cfg = b;
    } else {
        // one eager run: kernel attributes are set outside the capture
        e = batched_run(t, q, B, preds, ks, k_max, metric, out_idx, out_dist, ws, opts, cfg, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(VRS_E_HIP, "batched graph warm-up failed: %s", hipGetErrorString(e));
    auto *g = new vrs_graph_s();
    g->cfg = cfg;
    HIP_TRY(hipGetDevice(&g->device));
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) {
        prof_quiet(true);
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t er = batched_run(t, q, B, preds, ks, k_max, metric, out_idx, out_dist, ws, opts, cfg, cs);
            e = hipStreamEndCapture(cs, &g->graph);
            if (er != hipSuccess) e = er;
        }
        prof_quiet(false);
        (void)hipStreamDestroy(cs);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return fail(VRS_E_HIP, "batched graph capture failed: %s", hipGetErrorString(e));
    }
    *out = g;
    return ok();
}

vrs_status vrs_scan_graph_create(vrs_table t, const float *q, int32_t B, const vrs_pred *pred, int32_t k,
                                 vrs_metric metric, int64_t *out_idx, float *out_dist, void *ws,
                                 size_t ws_bytes, const vrs_opts *opts, void *stream, vrs_graph *out) {
    if (!out) return fail(VRS_E_ARG, "out is NULL");
    *out = nullptr;
    // one eager run: checks the arguments, sets kernel attributes outside the
    // capture, and leaves this call's results in the outputs
    vrs_status st = scan_common(t, q, B, pred, nullptr, nullptr, k, metric, out_idx, out_dist, ws, ws_bytes,
                                opts, stream);
    if (st != VRS_OK) return st;
    PredDev p;
    st = fold_pred(pred, t->n_attr, &p);
    if (st != VRS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(VRS_E_HIP, "scan graph warm-up failed: %s", hipGetErrorString(e));
    auto *g = new vrs_graph_s();
    g->cfg = -1;
    HIP_TRY(hipGetDevice(&g->device));
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) {
        prof_quiet(true);
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t er = run_scan(t, q, B, p, nullptr, nullptr, k, metric, out_idx, out_dist, ws, opts, cs);
            e = hipStreamEndCapture(cs, &g->graph);
            if (er != hipSuccess) e = er;
        }
        prof_quiet(false);
        (void)hipStreamDestroy(cs);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return fail(VRS_E_HIP, "scan graph capture failed: %s", hipGetErrorString(e));
    }
    *out = g;
    return ok();
}

vrs_status vrs_graph_launch(vrs_graph g, void *stream) {
    if (!g) return fail(VRS_E_ARG, "graph is NULL");
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return ok();
}

int32_t vrs_graph_config(vrs_graph g) { return g ? g->cfg : -1; }

vrs_status vrs_graph_destroy(vrs_graph g) {
    if (!g) return fail(VRS_E_ARG, "graph is NULL");
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return ok();
}

}  // extern "C"
