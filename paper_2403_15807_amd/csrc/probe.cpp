// probe.cpp -- host side of the probe-based access path: the partition index
// (vrs_index_build: k-means on the stored vectors, squared L2; every
// assignment is the exact nearest centroid, a vector join against the
// centroid table) and the filtered probe (vrs_probe_topk: the queries'
// nearest centroids by an exact scan of the centroid table, then the
// walk, exact scoring and merge kernels of k_probe.hip).
#include <algorithm>
#include <vector>

#include "internal.h"
#include "planner.h"


namespace vrs {

namespace {
size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// Probe time model (ms): fixed, per query, per GB of predicate columns
// visited, per GB of qualifying rows (see access_costs).
constexpr double PROBE_FIT[4] = {0.175, 2.75e-3, 1.48, 0.438};

struct ProbePlan {
    int gc, gs, srows;  // counting / scoring workgroups per query, rows per scoring step
    bool two_level;     // partial lists merged in groups of PROBE_FAN first
    size_t o_ckeys, o_cidx, o_pre, o_cnt, o_state, o_part, o_part2, total;
};

// Launch shape of the probe: small batches split a query's rows over many
// workgroups in short steps (latency), large ones use fewer, longer steps.
ProbePlan probe_plan(const vrs_index_s *ix, int B, int k, int nprobe, int64_t cap_c) {
    (void)nprobe;
    ProbePlan P{};
    const int walk = std::min(ix->nlist, PROBE_MAX_WALK);
    // rows one query may visit: the first partition, or partitions within cap_c
    const int64_t vis = std::max<int64_t>(std::min<int64_t>(cap_c, ix->table->n), ix->max_list);
    P.srows = B <= 16 ? 256 * 2 : 256 * 16;
    const int64_t nst = std::max<int64_t>(1, (vis + P.srows - 1) / P.srows);
    P.gc = std::max(1, std::min(256, 8192 / B));
    P.gs = (int)std::max<int64_t>(1, std::min<int64_t>({nst, 4096 / B, PROBE_MAX_GS}));
    P.two_level = P.gs > 2 * PROBE_FAN;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += a256(bytes);
        return r;
    };
    P.o_ckeys = take(ix->nlist <= PROBE_SORT_MAX ? (size_t)B * next_pow2(ix->nlist) * 16 : 0);
    P.o_cidx = take((size_t)B * walk * 8);
    P.o_pre = take((size_t)B * (walk + 1) * 8);
    P.o_cnt = take((size_t)B * walk * 4);
    P.o_state = take((size_t)B * 4 * 8);
    P.o_part = take((size_t)B * P.gs * k * 16);
    P.o_part2 = P.two_level ? take((size_t)B * ((P.gs + PROBE_FAN - 1) / PROBE_FAN) * k * 16) : 0;
    P.total = o;
    return P;
}

template <typename T>
hipError_t dalloc(T **p, size_t count) {
    return hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
}
}  // namespace

size_t probe_workspace(const vrs_index_s *ix, int B, int k, int nprobe, int64_t cap_c) {
    return probe_plan(ix, B, k, nprobe, cap_c).total;
}

void index_free(vrs_index_s *ix) {
    if (!ix) return;
    if (ix->cent_tab) vrs_destroy_table(ix->cent_tab);
    (void)hipFree(ix->cent);
    (void)hipFree(ix->list_off);
    (void)hipFree(ix->ids);
    (void)hipFree(ix->rows_p);
    (void)hipFree(ix->scale_p);
    (void)hipFree(ix->attr_p);
    delete ix;
}

// k-means: centroids start at the rows floor(i n / nlist); each iteration
// assigns every row to its exact nearest centroid (a join of the table
// against the centroid table, k = 1) and moves every centroid to its
// partition's mean.  The final lists come from the final centroids.
hipError_t index_build(const vrs_table_s *t, int nlist, int iters, hipStream_t s, vrs_index_s **out,
                       std::string *err) {
    vrs_index_s *ix = new vrs_index_s();
    ix->table = t;
    ix->nlist = nlist;
    ix->d = t->d;
    const int64_t n = t->n;
    const int nblk = (int)((n + PROBE_LIST_BLOCK - 1) / PROBE_LIST_BLOCK);
    float *x32 = nullptr, *jdist = nullptr;
    int64_t *assign = nullptr, *size = nullptr;
    uint32_t *cnt = nullptr;
    void *jws = nullptr;
    size_t jws_bytes = 0;
    hipError_t e = hipSuccess;
    auto fail = [&](const char *what) {
        *err = std::string(what) + ": " + hipGetErrorString(e);
        (void)hipStreamSynchronize(s);
        (void)hipFree(x32);
        (void)hipFree(jdist);
        (void)hipFree(assign);
        (void)hipFree(size);
        (void)hipFree(cnt);
        (void)hipFree(jws);
        index_free(ix);
        return e;
    };
    if ((e = dalloc(&x32, (size_t)n * t->d)) != hipSuccess) return fail("allocation");
    if ((e = dalloc(&jdist, (size_t)n)) != hipSuccess) return fail("allocation");
    if ((e = dalloc(&assign, (size_t)n)) != hipSuccess) return fail("allocation");
    if ((e = dalloc(&size, (size_t)nlist)) != hipSuccess) return fail("allocation");
    if ((e = dalloc(&cnt, (size_t)nblk * nlist)) != hipSuccess) return fail("allocation");
    if ((e = dalloc(&ix->cent, (size_t)nlist * t->d)) != hipSuccess) return fail("allocation");
    if ((e = dalloc(&ix->list_off, (size_t)nlist + 1)) != hipSuccess) return fail("allocation");
    if ((e = dalloc(&ix->ids, (size_t)n)) != hipSuccess) return fail("allocation");
    if ((e = launch_rows_to_f32(t, 0, n, x32, s)) != hipSuccess) return fail("decode");
    if ((e = launch_centroid_init(x32, n, nlist, t->d, ix->cent, s)) != hipSuccess) return fail("init");
    for (int it = 0; it <= iters; ++it) {
        vrs_table_s *ct = nullptr;
        vrs_status st = vrs_build_table(ix->cent, nlist, t->d, nullptr, 0, VRS_F32, 0, s, &ct);
        if (st != VRS_OK) {
            e = hipErrorUnknown;
            return fail("centroid table");
        }
        const size_t need = join_workspace(t, ct, 1, nullptr);
        if (need > jws_bytes) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(jws);
            jws = nullptr;
            if ((e = hipMalloc(&jws, need)) != hipSuccess) {
                vrs_destroy_table(ct);
                return fail("allocation");
            }
            jws_bytes = need;
        }
        PredDev none{};
        none.nterms = 0;
        e = run_join(t, ct, none, 1, VRS_L2SQ, assign, jdist, jws, nullptr, s);
        if (e == hipSuccess) e = launch_index_lists(assign, n, nlist, cnt, size, ix->list_off, ix->ids, s);
        if (e == hipSuccess && it < iters) e = launch_centroid_mean(x32, nlist, t->d, ix->list_off, ix->ids, ix->cent, s);
        if (e != hipSuccess) {
            vrs_destroy_table(ct);
            return fail("iteration");
        }
        if (it < iters) {
            (void)hipStreamSynchronize(s);  // the centroid table is rebuilt from the new centroids
            vrs_destroy_table(ct);
        } else {
            ix->cent_tab = ct;        // the final centroids: the coarse scan's table
        }
    }
    // the partition-ordered copies the probe reads
    const int64_t row_bytes = (int64_t)t->dp * elem_bytes(t->store);
    if ((e = hipMalloc(&ix->rows_p, std::max<size_t>((size_t)n * row_bytes, 16))) != hipSuccess)
        return fail("allocation");
    if (t->scale && (e = dalloc(&ix->scale_p, (size_t)n)) != hipSuccess) return fail("allocation");
    if ((e = dalloc(&ix->attr_p, (size_t)std::max(1, t->n_attr) * n)) != hipSuccess) return fail("allocation");
    if ((e = launch_list_gather(ix->ids, n, t->rows, row_bytes, t->scale, t->attr, t->n_attr, t->attr_stride,
                                ix->rows_p, ix->scale_p, ix->attr_p, s)) != hipSuccess)
        return fail("list copies");
    std::vector<int64_t> off(nlist + 1);
    e = hipMemcpyAsync(off.data(), ix->list_off, (nlist + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail("list sizes");
    for (int c = 0; c < nlist; ++c) {
        const int64_t sz = off[c + 1] - off[c];
        ix->max_list = std::max(ix->max_list, sz);
        ix->size_biased += (double)sz * (double)sz / (double)n;
    }
    (void)hipFree(x32);
    (void)hipFree(jdist);
    (void)hipFree(assign);
    (void)hipFree(size);
    (void)hipFree(cnt);
    (void)hipFree(jws);
    *out = ix;
    return hipSuccess;
}

hipError_t run_probe(const vrs_index_s *ix, const float *q, int B, const PredDev &p, int k, vrs_metric metric,
                     int nprobe, int64_t min_cand, int64_t cap_c, int64_t *out_idx, float *out_dist,
                     int32_t *out_taken, void *ws, hipStream_t s) {
    const vrs_table_s *t = ix->table;
    const ProbePlan P = probe_plan(ix, B, k, nprobe, cap_c);
    char *w = (char *)ws;
    int64_t *cidx = (int64_t *)(w + P.o_cidx);
    ProbeArgs a{};
    a.rows = ix->rows_p;
    a.scale = ix->scale_p;
    a.d = t->d;
    a.dp = t->dp;
    a.store = t->store;
    a.metric = metric;
    a.attr = ix->attr_p;
    a.an = t->n;
    a.pred = p;
    a.q = q;
    a.B = B;
    a.k = k;
    a.cent_rows = ix->cent_tab->rows;
    a.cdp = ix->cent_tab->dp;
    a.nlist = ix->nlist;
    a.ckeys = ix->nlist <= PROBE_SORT_MAX ? (void *)(w + P.o_ckeys) : nullptr;
    a.coarse_out = cidx;
    a.coarse = cidx;
    a.walk = std::min(ix->nlist, PROBE_MAX_WALK);
    a.nprobe = nprobe;
    a.min_cand = min_cand;
    a.cap_c = cap_c;
    a.list_off = ix->list_off;
    a.ids = ix->ids;
    a.pre = (int64_t *)(w + P.o_pre);
    a.cnt = (uint32_t *)(w + P.o_cnt);
    a.state = (int64_t *)(w + P.o_state);
    a.gc = P.gc;
    a.gs = P.gs;
    a.srows = P.srows;
    a.taken = out_taken;
    a.part = (uint64_t *)(w + P.o_part);
    a.part2 = P.two_level ? (uint64_t *)(w + P.o_part2) : nullptr;
    a.out_idx = out_idx;
    a.out_dist = out_dist;
    prof_begin(4, s);
    hipError_t e = launch_probe(a, s);
    prof_end(4, s);
    return e;
}

// Scan-vs-probe estimates (ms).  The scan: the learned chooser's predicted
// time of the arm it would pick, when a network is installed (it is trained
// on measured scan timings); otherwise a bytes-moved model (the predicate
// columns and either every row or the qualifying ones, read once for the
// batch, plus 2 B s N d flops).  The probe: the rows a query's walk visits,
// from the size-biased mean partition size L (the partition of a random row
// holds sum(size^2) / n rows on average, and queries fall where the rows
// are):
//   V = min(cap_c, walk L, max(nprobe L, k / s)),
// then a linear model of the batch's bytes: the predicate columns of the
// visited rows (read by the counting and the scoring passes) and the
// qualifying rows.  Its coefficients are fitted to measured probe times of a
// 10M x 128 float32 index with 1024 partitions at B = 1, 16 and 256.
void access_costs(const vrs_index_s *ix, int B, const PredDev &p, int k, int nprobe, int64_t cap_c,
                  double *scan_ms, double *probe_ms) {
    const vrs_table_s *t = ix->table;
    const double s = std::max(estimate_selectivity(t, p), 1e-9);
    const double n = (double)t->n, terms = std::max(0, p.nterms);
    const double row = (double)t->dp * elem_bytes(t->store);
    const double learned = plan_predict_ms(t, B, p, k, VRS_L2SQ);
    if (learned > 0.0) {
        *scan_ms = learned;
    } else {
        const double hbm = 5.0e12, mfma = 60e12, fixed_scan = 80e-6;
        const double mask = n * (row + 4.0 * terms), gather = 4.0 * terms * n + s * n * (row + 4.0);
        *scan_ms = 1e3 * (fixed_scan + std::min(mask, gather) / hbm + 2.0 * B * s * n * t->d / mfma);
    }
    const double L = std::max(1.0, ix->size_biased);
    const double walk = std::min(ix->nlist, PROBE_MAX_WALK);
    const double V = std::min({(double)cap_c, walk * L, std::max(nprobe * L, k / s)});
    const double attr_gb = B * V * 4.0 * std::max(1.0, terms) / 1e9;
    const double rows_gb = B * V * s * (row + 4.0) / 1e9;
    *probe_ms = PROBE_FIT[0] + PROBE_FIT[1] * B + PROBE_FIT[2] * attr_gb + PROBE_FIT[3] * rows_gb;
}

}  // namespace vrs
