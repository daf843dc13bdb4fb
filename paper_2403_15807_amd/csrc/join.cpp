// join.cpp -- host side of the vector join (vrs_join_topk): every row of R,
// as its stored vector, is a query against the rows of S.  R is taken in
// batches of up to JOIN_BATCH rows; each batch is decoded to float32 into
// the workspace and scanned as one batch of the filtered top-k scan (the
// N:N tensor form of Section 3.1, with the planner's choice of strategy and
// kernel per batch).
#include <algorithm>

#include "internal.h"
#include "planner.h"

namespace vrs {

namespace {
constexpr int64_t JOIN_BATCH = 8192;
size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

size_t join_workspace(const vrs_table_s *R, const vrs_table_s *S, int k, const vrs_opts *opts) {
    const int64_t jb = std::min(R->n, JOIN_BATCH), last = R->n % jb;
    size_t scan = plan_workspace(S, (int)jb, k, opts);
    if (last) scan = std::max(scan, plan_workspace(S, (int)last, k, opts));
    return a256((size_t)jb * R->d * 4) + scan;
}

hipError_t run_join(const vrs_table_s *R, const vrs_table_s *S, const PredDev &p, int k,
                    vrs_metric metric, int64_t *out_idx, float *out_dist, void *ws,
                    const vrs_opts *opts, hipStream_t s) {
    const int64_t jb = std::min(R->n, JOIN_BATCH);
    float *qbuf = (float *)ws;
    void *scan_ws = (char *)ws + a256((size_t)jb * R->d * 4);
    for (int64_t i0 = 0; i0 < R->n; i0 += jb) {
        const int b = (int)std::min(jb, R->n - i0);
        hipError_t e = launch_rows_to_f32(R, i0, b, qbuf, s);
        if (e != hipSuccess) return e;
        // per-query outputs of this batch start at row i0
        vrs_opts o = opts ? *opts : vrs_opts{};
        o.tile = opts ? opts->tile : -1;
        if (o.n_valid) o.n_valid += i0;
        if (o.certified) o.certified += i0;
        if (o.err_ratio) o.err_ratio += i0;
        e = run_scan(S, qbuf, b, p, nullptr, nullptr, k, metric, out_idx + i0 * k, out_dist + i0 * k, scan_ws,
                     &o, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace vrs
