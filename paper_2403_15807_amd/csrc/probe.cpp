// probe.cpp -- host side of the probe-based access path: the partition index
// (vrs_index_build: k-means on the stored vectors, squared L2; every
// assignment is the exact nearest centroid, a vector join against the
// centroid table) and the filtered probe (vrs_probe_topk: the queries'
// nearest centroids by an exact scan of the centroid table, then the
// collection, exact scoring and merge kernels of k_probe.hip).
#include <algorithm>
#include <vector>

#include "internal.h"
#include "planner.h"


namespace vrs {

namespace {
size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct ProbePlan {
    int64_t cand_cap;
    int nchunk;
    size_t o_scan, o_cidx, o_cdist, o_cand, o_ncand, o_part, total;
};

ProbePlan probe_plan(const vrs_index_s *ix, int B, int k, int nprobe, int64_t cap_c) {
    ProbePlan P{};
    P.cand_cap = std::max<int64_t>(std::min<int64_t>(cap_c, ix->table->n), ix->max_list);
    P.nchunk = (int)((P.cand_cap + PROBE_CHUNK - 1) / PROBE_CHUNK);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += a256(bytes);
        return r;
    };
    P.o_scan = take(plan_workspace(ix->cent_tab, B, nprobe, nullptr));
    P.o_cidx = take((size_t)B * nprobe * 8);
    P.o_cdist = take((size_t)B * nprobe * 4);
    P.o_cand = take((size_t)B * P.cand_cap * 4);
    P.o_ncand = take((size_t)B * 4);
    P.o_part = take((size_t)B * P.nchunk * k * 16);
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
    std::vector<int64_t> off(nlist + 1);
    e = hipMemcpyAsync(off.data(), ix->list_off, (nlist + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail("list sizes");
    for (int c = 0; c < nlist; ++c) ix->max_list = std::max(ix->max_list, off[c + 1] - off[c]);
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
    PredDev none{};
    none.nterms = 0;
    prof_begin(2, s);
    hipError_t e = run_scan(ix->cent_tab, q, B, none, nullptr, nullptr, nprobe, VRS_L2SQ, cidx,
                            (float *)(w + P.o_cdist), w + P.o_scan, nullptr, s);
    prof_end(2, s);
    if (e != hipSuccess) return e;
    ProbeArgs a{};
    a.rows = t->rows;
    a.scale = t->scale;
    a.d = t->d;
    a.dp = t->dp;
    a.store = t->store;
    a.metric = metric;
    a.attr = t->attr;
    a.an = t->attr_stride;
    a.pred = p;
    a.q = q;
    a.B = B;
    a.k = k;
    a.coarse = cidx;
    a.nprobe = nprobe;
    a.min_cand = min_cand;
    a.cap_c = cap_c;
    a.list_off = ix->list_off;
    a.ids = ix->ids;
    a.cand = (int32_t *)(w + P.o_cand);
    a.cand_cap = P.cand_cap;
    a.ncand = (int32_t *)(w + P.o_ncand);
    a.taken = out_taken;
    a.nchunk = P.nchunk;
    a.part = (uint64_t *)(w + P.o_part);
    a.out_idx = out_idx;
    a.out_dist = out_dist;
    prof_begin(4, s);
    e = launch_probe(a, s);
    prof_end(4, s);
    return e;
}

// Scan-vs-probe cost model (bytes moved at the HBM rate plus a fixed launch
// cost per call, and the batch's MFMA work for the scan), from the
// estimated selectivity s of the predicate:
//   scan:  min(mask: every row and its predicate columns once,
//              gather: the predicate columns, then the s N qualifying rows
//              and their ids), the table read once for the whole batch,
//              plus 2 B s N d flops;
//   probe: per query, the partitions visited until k rows qualify, at least
//          one and at most nprobe (average partition n / nlist), capped at
//          cap_c rows: their ids and predicate columns, and the qualifying
//          rows among them; plus the coarse scan of the centroids.
void access_costs(const vrs_index_s *ix, int B, const PredDev &p, int k, int nprobe, int64_t cap_c,
                  double *scan_ms, double *probe_ms) {
    const vrs_table_s *t = ix->table;
    const double s = std::max(estimate_selectivity(t, p), 1e-9);
    const double n = (double)t->n, terms = std::max(0, p.nterms);
    const double row = (double)t->dp * elem_bytes(t->store);
    const double hbm = 5.0e12, mfma = 60e12, fixed_scan = 80e-6, fixed_probe = 60e-6;
    const double mask = n * (row + 4.0 * terms), gather = 4.0 * terms * n + s * n * (row + 4.0);
    *scan_ms = 1e3 * (fixed_scan + std::min(mask, gather) / hbm + 2.0 * B * s * n * t->d / mfma);
    const double L = n / ix->nlist;
    const double visited = std::min((double)cap_c, std::min(nprobe * L, std::max(L, k / s)));
    const double per_q = visited * (4.0 + 4.0 * terms) + s * visited * row;
    *probe_ms = 1e3 * (fixed_probe + (B * per_q + (double)ix->nlist * row) / hbm);
}

}  // namespace vrs
