// internal.h -- host-side structures shared by the library's translation
// units (table object, launch parameters, kernel launchers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/vrs.h"
#include "common.h"

struct vrs_table_s {
    int64_t n = 0;
    int32_t d = 0, dp = 0;      // logical and padded dimension
    int32_t n_attr = 0;
    vrs_dtype store = VRS_F32;
    int device = 0;
    void *rows = nullptr;       // [n][dp] float / uint16 / uint8
    float *scale = nullptr;     // [n] FP8 row scales
    float *norm2 = nullptr;     // [n] ||x_i||^2 of the stored row (float32)
    int32_t *attr = nullptr;    // [n_attr][attr_stride]
    int64_t attr_stride = 0;    // column stride of attr (the parent's n for a view)
    bool owner = true;          // false for a view (vrs_table_view)
    double max_norm = 0.0;      // max_i ||x_i|| of stored rows (rounded up)
    // per-column equi-width histograms for selectivity estimates (host copy,
    // and a device copy for estimates made inside a batched launch)
    std::vector<int32_t> amin, amax;
    std::vector<std::vector<uint32_t>> hist;
    void *dstats = nullptr;     // device: amin[64] | amax[64] | hist[n_attr][HIST_BINS]
    void *stats_alloc = nullptr;  // the allocation holding dstats (owner only)
};

// A partition index over a table's vector column (probe.cpp).
struct vrs_index_s {
    const vrs_table_s *table = nullptr;  // the indexed table (the caller keeps it alive)
    vrs_table_s *cent_tab = nullptr;     // centroids as a float32 table (coarse scans)
    float *cent = nullptr;               // [nlist][d]
    int64_t *list_off = nullptr;         // [nlist + 1]
    int32_t *ids = nullptr;              // [n] rows of every partition, ascending
    // The table's stored rows, FP8 scales and predicate columns copied into
    // the same partition order (position m holds row ids[m]), so that a
    // probe reads a partition's data contiguously.
    void *rows_p = nullptr;              // [n][dp] as stored
    float *scale_p = nullptr;            // [n] (FP8 tables)
    int32_t *attr_p = nullptr;           // [n_attr][n]
    int32_t nlist = 0, d = 0;
    int64_t max_list = 0;                // largest partition
    double size_biased = 0.0;            // mean size of a row's partition: sum of size^2 / n
};

namespace vrs {

constexpr int HIST_BINS = 256;

// Raise a kernel's dynamic LDS limit to `bytes` (once per kernel and size, so
// launches made while a stream is being captured set nothing).
void ensure_dyn_lds(const void *kernel, size_t bytes);

int elem_bytes(vrs_dtype t);
// Record a failed call's status and message for vrs_last_error().
vrs_status set_error(vrs_status st, const char *msg);
int pad_dim(int d, vrs_dtype t);

// ---- build kernels (k_build.hip)
hipError_t launch_build_rows(const float *vec, int64_t n, int32_t d, int32_t dp, vrs_dtype store,
                             int normalize, void *rows, float *scale, float *norm2,
                             unsigned long long *max_norm_bits, int *bad_flag, hipStream_t s);
hipError_t launch_attr_stats(const int32_t *attr, int64_t n, int32_t n_attr, int32_t *amin,
                             int32_t *amax, uint32_t *hist, hipStream_t s);
// Rows [i0, i0 + count) as float32 vectors [count][d] (FP8: scale * code,
// rounded to float32).
hipError_t launch_rows_to_f32(const vrs_table_s *t, int64_t i0, int64_t count, float *out, hipStream_t s);

// ---- predicate pass (k_select.hip)
constexpr int SEL_BLOCK_ROWS = 8192;
hipError_t launch_select(const int32_t *attr, int64_t n, int64_t an, const PredDev &p,
                         uint32_t *bitmap, uint32_t *blkcnt, int32_t *ids, int64_t *count,
                         hipStream_t s);

// ---- query preparation (k_finish.hip)
// heads (or null): [B][n_heads] keys set to KEY_INF (see ScreenArgs::heads_bound)
hipError_t launch_prep_queries(const float *q, int32_t B, int32_t d, int32_t dp, float *qp,
                               double *qnorm, float *qn2, uint16_t *qhl, uint64_t *gthr,
                               int32_t *fail_count, uint64_t *heads, int32_t n_heads, hipStream_t s);
int screen_mfma_occupancy(int Kp, int CB, int qm);
hipError_t launch_prep_batched(const vrs_pred *preds, const int32_t *ks, int32_t B, int32_t kmax,
                               int32_t n_attr, int kmult, int f32_rule, PredDev *out,
                               int32_t *kc, int32_t *kps, hipStream_t s);
// Query preparation of the batched uneven form, by position: queries in the
// order of `perm`, with their folded predicates and k, k' gathered alongside.
hipError_t launch_prep_permuted(const float *q, const int32_t *perm, int32_t B, int32_t d,
                                int32_t dp, const PredDev *pred_o, const int32_t *kc_o,
                                const int32_t *kps_o, float *qp, double *qnorm, float *qn2,
                                uint16_t *qhl, uint64_t *gthr, int32_t *fail_count,
                                PredDev *pred_p, int32_t *kc_p, int32_t *kps_p, hipStream_t s);

// ---- screening (k_stream.hip): per-(query, chunk) sorted lists of the K
// smallest screening keys.
struct ScreenArgs {
    const void *rows;
    const float *scale;
    int64_t n;
    int32_t dp;
    vrs_dtype store;
    const int32_t *attr;
    int64_t an;                    // attribute column stride
    int32_t n_attr;
    PredDev pred;                  // shared predicate (batch form: preds != null)
    const PredDev *preds;          // [B] per-query predicates or null
    const int32_t *sel_ids;        // gather: qualifying rows
    const int64_t *sel_count;
    int gather;
    const float *qp;               // [B][dp]
    const float *qn2;              // [B] ||q||^2 (float32 of the FP64 sum)
    const uint16_t *qhl;           // [B][2][dp] bfloat16 hi/lo split of the queries
    const float *norm2;            // [n] ||x_i||^2 of stored rows
    int32_t B;
    int metric;
    int32_t K, Kp, CB;
    int32_t n_chunks;
    int32_t shared_rows;           // rows are read by several query tiles: keep them cacheable
    uint64_t *partials;            // [B][n_chunks][K]
    uint64_t *heads;               // [B][n_chunks] first key of each list, or null
    // heads were set to KEY_INF before the launch: a one-query streaming
    // workgroup then publishes its best key there at every flush and bounds
    // its list by the K-th smallest published key
    int32_t heads_bound;
    // [B][n_chunks] keys each list holds (MFMA kernels), or null: the list
    // entries past them are then left unwritten instead of set to KEY_INF
    int32_t *fills;
    uint64_t *cbuf;                // [B][n_chunks][CB] candidate buffers (MFMA kernels)
    uint64_t *gthr;                // [B] smallest K-th key published by any chunk
    // Two-pass screening (MFMA kernels): pass 1 covers the first tiles of
    // every chunk (a sample whose merged K-th key bounds the result), pass 2
    // all of every chunk again with fresh lists, admitting keys below that
    // bound; pass 0 = one pass over everything.  prefix_sel: the fraction of
    // the visited rows expected to qualify (1 with a selection vector).
    int32_t pass;
    float prefix_sel;
    // batched uneven form only (null otherwise): control words written on the
    // device (dense query count, row chunks per dense query, work queues) and
    // the sparse queries' id lists; see BatchCtl.
    int32_t *bctl;
    const int64_t *sp_off;         // [B] by position: first id of the query's list in sp_pool
    const int32_t *sp_cnt;         // [B] by position: ids in the list
    const int32_t *seg_pre;        // [B + 1] segments of the sparse positions, prefix sums
    const int32_t *sp_pool;
    const int32_t *kps;            // [B] by position: per-query k'
};

// Rows [c0, c1) of a chunk (one of nchunks) that this screening pass covers
// (tiles of br rows).  The first pass screens a prefix of every chunk sized
// so that the K-th smallest key of all prefixes leaves about 64 keys per
// list for the second pass (a sample of K * rows / 64 / nchunks rows) and
// holds 2K qualifying rows, between one tile and an eighth of the chunk.
__device__ __forceinline__ void pass_range(const ScreenArgs &a, int64_t &c0, int64_t &c1, int br,
                                           int64_t total, int nchunks) {
    if (a.pass != 1 || c1 <= c0) return;
    const int64_t nt = (c1 - c0 + br - 1) / br;
    const double per_list = (double)a.K * (double)total / (64.0 * nchunks * (double)nchunks);
    const double qual = 2.0 * a.K / ((double)nchunks * fmax((double)a.prefix_sel, 1e-3));
    int64_t tp = (int64_t)ceil(fmax(per_list, qual) / br);
    tp = max((int64_t)1, min(tp, nt / 8));
    c1 = min(c1, c0 + tp * br);
}

// Control words of a batched launch (int32, in the workspace).
enum BatchCtl {
    BC_NDENSE = 0,   // queries screened by the dense MFMA kernel (positions [0, n_dense))
    BC_NSPARSE = 1,  // queries screened by the sparse gather kernel
    BC_NC = 2,       // row chunks (lists) per dense query
    BC_QDENSE = 3,   // 8 work-queue counters of the dense kernel, one per XCD
    BC_QSPARSE = 11, // work-queue counter of the sparse kernel
    BC_NCAND = 12,   // sparse candidates (entries of BatchArgs::cands)
    BC_WORDS = 16
};

// A query's predicate as unsigned range tests on the first two attribute
// columns (the batched predicate passes keep those columns in registers):
// row i qualifies iff (uint32)(A[0][i] - lo0) <= span0 and likewise for
// column 1.  kind 1 = a term on another column (evaluated from the folded
// predicate), kind 2 = selects no row.
struct QRange {
    int32_t b;
    int32_t kind;
    int32_t lo0, lo1;
    uint32_t span0, span1;
};
hipError_t launch_screen_stream(const ScreenArgs &a, int qt, hipStream_t s);
size_t screen_stream_lds(int qt, int Kp, int CB, int dp);
hipError_t launch_screen_mfma(const ScreenArgs &a, int qm, hipStream_t s);
size_t screen_mfma_lds(int dp, int qm);
hipError_t launch_screen_mfma_bf16(const ScreenArgs &a, hipStream_t s);
size_t screen_mfma_bf16_lds(int kc);  // kc = coordinates per chunk (64 or 128)
int screen_mfma_bf16_qm();                              // queries per workgroup
size_t screen_mfma_bf16_qfrag_bytes(int B, int dp);     // fragment-ordered query copy
bool screen_mfma_bf16_supported(int dp, vrs_dtype store, int metric, int Kp, int CB);
bool screen_mfma_supported(int dp, vrs_dtype store, int Kp, int CB);
// persistent forms for the batched uneven launch (queue-driven, one grid)
hipError_t launch_screen_mfma_persistent(const ScreenArgs &a, int qm, int grid, hipStream_t s);
hipError_t launch_screen_mfma_bf16_persistent(const ScreenArgs &a, int grid, hipStream_t s);

// Fold a caller's predicate (int64 half-open bounds) into inclusive int32
// ranges: a term on a column outside [0, n_attr), a term count outside
// [0, VRS_MAX_TERMS] or an empty range selects nothing (nterms = -1).
__device__ inline PredDev fold_pred_dev(const vrs_pred &p, int n_attr) {
    PredDev o;
    o.nterms = 0;
    for (int t = 0; t < 4; ++t) {
        o.col[t] = 0;
        o.lo[t] = 0;
        o.hi[t] = -1;
    }
    bool empty = p.nterms < 0 || p.nterms > VRS_MAX_TERMS;
    if (!empty) {
        for (int t = 0; t < p.nterms; ++t) {
            const vrs_range &r = p.term[t];
            const int64_t lo = r.lo, hi = r.hi;
            if (r.col < 0 || r.col >= n_attr || hi <= lo || hi <= (int64_t)INT32_MIN ||
                lo > (int64_t)INT32_MAX) {
                empty = true;
                break;
            }
            o.col[t] = r.col;
            o.lo[t] = (int32_t)(lo < (int64_t)INT32_MIN ? (int64_t)INT32_MIN : lo);
            o.hi[t] = (int32_t)(hi - 1 > (int64_t)INT32_MAX ? (int64_t)INT32_MAX : hi - 1);
        }
        o.nterms = p.nterms;
    }
    if (empty) o.nterms = -1;
    return o;
}

// Range form of a folded predicate (see QRange).
__device__ inline QRange range_form(int b, const PredDev &o) {
    QRange r;
    r.b = b;
    r.kind = 0;
    int32_t lo[2] = {INT32_MIN, INT32_MIN}, hi[2] = {INT32_MAX, INT32_MAX};
    bool none = o.nterms < 0;
    for (int t = 0; t < 4; ++t) {
        if (t >= o.nterms) break;
        const int c = o.col[t];
        if (c > 1) {
            r.kind = 1;
        } else {
            lo[c] = max(lo[c], o.lo[t]);
            hi[c] = min(hi[c], o.hi[t]);
        }
    }
    if (lo[0] > hi[0] || lo[1] > hi[1]) none = true;
    r.lo0 = lo[0];
    r.lo1 = lo[1];
    r.span0 = (uint32_t)hi[0] - (uint32_t)lo[0];
    r.span1 = (uint32_t)hi[1] - (uint32_t)lo[1];
    if (none) r.kind = 2;
    return r;
}

// k' of one query (the host rule of the planner).  kfloor: the batched
// form's lists are sized for k_max, so a query with a smaller k keeps (and
// reranks) at least kfloor of them under the default rule.
__device__ inline int kprime_dev(int k, int kmult, int f32_rule, int kfloor = 0) {
    int kp = kmult > 0 ? k * kmult : max(f32_rule ? max(2 * k, k + 32) : max(4 * k, k + 32), kfloor);
    return min(max(kp, k), 1024);
}

// ---- batched uneven form (k_batched.hip)
constexpr int BSUB_ROWS = 1024;    // rows per wave in the batched predicate passes
struct BatchArgs {
    const vrs_pred *preds;         // [B] caller's predicates
    const int32_t *ks;             // [B] caller's k
    int32_t B, kmax, n_attr, kmult, f32_rule;
    int32_t kfloor;                // k' floor of the default rule (see kprime_dev)
    const int32_t *attr;
    int64_t n, an;
    const void *dstats;            // device column statistics (table)
    int64_t rows_cap;              // a query is sparse when it qualifies at most this many rows
    int32_t seg_rows;              // target rows per sparse work item
    int32_t seg_max;               // at most this many segments per sparse query
    int32_t items_target;          // dense work items wanted (sets the row chunks per query)
    int32_t nc_cap;                // most row chunks per dense query
    int32_t qm;                    // queries per dense work item
    int32_t nsub;                  // 1024-row sub-blocks
    PredDev *pred_o;               // [B] folded predicates, by query
    QRange *qr;                    // [B] range form, by query
    QRange *cands;                 // [B] range form of the sparse candidates (any order)
    int32_t *kc_o, *kps_o;         // [B] clamped k and k', by query
    uint8_t *cand;                 // [B] sparse candidate by the estimate
    int32_t *tot;                  // [B] qualifying rows (-1: not a candidate)
    int32_t *perm;                 // [B] position -> query
    int64_t *sp_off;               // [B] by position
    int32_t *sp_cnt;               // [B] by position
    int32_t *seg_pre;              // [B + 1]
    int64_t *list_off;             // [B] by position: first list in the partials
    int32_t *nlists;               // [B] by position: lists in the partials
    int32_t *pool;                 // [B][rows_cap] sparse id lists, one region per query
    int32_t *ctl;                  // BatchCtl words
};
hipError_t launch_batch_classify(const BatchArgs &b, hipStream_t s);
hipError_t launch_screen_sparse(const ScreenArgs &a, int grid, hipStream_t s);
size_t screen_sparse_lds(int K, int dp);

// ---- merge, rerank, fallback (k_finish.hip)
struct FinishArgs {
    const void *rows;
    const float *scale;
    int64_t n;
    int32_t d, dp;
    vrs_dtype store;
    const int32_t *attr;
    int64_t an;                    // attribute column stride
    PredDev pred;
    const PredDev *preds;
    const float *q;                // original queries [B][d]
    const double *qnorm;           // [B]
    int32_t B;
    int metric;
    int32_t k;                     // shared k (ks == null)
    const int32_t *ks;             // [B] per-query k or null
    int32_t kmax;                  // output row stride
    int32_t kprime;                // shared k' (kps == null)
    const int32_t *kps;            // [B] per-query k' or null
    int32_t K;                     // list length = max k' + 1
    int32_t n_chunks;
    const uint64_t *partials;
    const uint64_t *heads;         // [B][n_chunks] first key of each list, or null
    const int32_t *fills;          // [B][n_chunks] keys each list holds (entries past them unread), or null
    const int64_t *list_off;       // batched uneven form: [B] first list of each position
    const int32_t *nlists;         // and its list count (null: n_chunks lists per query)
    const int32_t *perm;           // position -> query index (null: identity)
    uint64_t *merge_mid;           // [B][ceil(n_chunks/2048)][K] (two-level merge)
    uint64_t *merged;              // [B][K]
    const int32_t *merge_limit;    // positions >= *merge_limit get an empty merged list (or null)
    int32_t merge_one_head;        // the merge's bound starts from one head per list (dense predicates)
    double *rr_dist;               // [B][K] exact distances of the candidates
    double rel, abs_ip, abs_l2, max_norm;  // screening error model
    int32_t *fail_list;            // [B]
    int32_t *fail_count;           // [1]
    int64_t *out_idx;
    float *out_dist;
    int32_t *n_valid;
    uint8_t *certified;
    // [B] out or null: largest |screening distance - exact distance| / bound
    // over the query's reranked keys (the k' survivors and the (k'+1)-th key)
    float *err_ratio;
    // exact fallback
    int32_t fb_rows_per_chunk, fb_chunks, fb_slots;
    uint64_t *fb_partials;         // [fb_slots][fb_chunks][kmax][2]
};
hipError_t launch_merge(const FinishArgs &a, hipStream_t s);
// gthr[b] = merged[b][Kb-1] + 1 with Kb = the query's k'+1: the Kb-th
// smallest key of the merged lists bounds the Kb-th key of every superset of
// their rows, and a pass that admits keys below gthr then keeps that key too.
// zero8 (or null): 8 counters cleared on the way.
hipError_t launch_set_bound(const FinishArgs &a, uint64_t *gthr, int32_t *zero8, hipStream_t s);
hipError_t launch_rerank(const FinishArgs &a, hipStream_t s);
hipError_t launch_fallback(const FinishArgs &a, hipStream_t s);

// ---- threshold selection (k_range.hip): for each query, the qualifying
// rows whose exact FP64 distance is below its threshold, ascending by id.
constexpr int RANGE_BLOCK_ROWS = 8192;   // rows per block of the output compaction
struct RangeArgs {
    const void *rows;
    const float *scale;
    int64_t n;
    int32_t d, dp;
    vrs_dtype store;
    const int32_t *attr;
    int64_t an;                    // attribute column stride
    PredDev pred;
    const int32_t *sel_ids;        // gather: qualifying rows, ascending
    const int64_t *sel_count;
    int gather;
    const float *q;                // original queries [B][d]
    const float *qp;               // [B][dp] padded
    const double *qnorm;           // [B] FP64 query norms (rounded up)
    int32_t B;
    int metric;
    const double *thr;             // [B] thresholds (caller's)
    float *tf;                     // [B] screening admission bound (>= thr + error bound)
    double rel, abs_ip, abs_l2, max_norm;  // screening error model
    int32_t n_chunks;              // row chunks of the screening grid
    int32_t cap_c;                 // candidate slots per query
    uint32_t *cnt;                 // [B] candidates found (may exceed cap_c)
    int32_t *cand;                 // [B][cap_c] candidate rows
    int32_t *ovf_list;             // [B] queries whose candidates overflowed
    int32_t *ovf_count;            // [1]
    int32_t fb_chunks;             // row chunks of the exact pass for overflowed queries
    uint32_t *bitmap;              // [B][words] selected rows
    int64_t words;                 // 32-bit words per query bitmap (a multiple of 2)
    uint32_t *blkcnt;              // [B][nblk] selected rows per block of RANGE_BLOCK_ROWS
    int32_t nblk;
    int32_t cap;                   // output slots per query
    int64_t *out_idx;              // [B][cap]
    float *out_dist;               // [B][cap]
    int64_t *out_count;            // [B]
};
// Steps of a call, in order on one stream: 0 prep (admission bounds, empty
// bitmaps), 1 screening (qt queries per workgroup: 1, 2, 4 or 8), 2 exact
// distances of the candidates (and of every row for overflowed queries),
// 3 output (compaction, exact distances of the written ids, padding).
hipError_t launch_range(const RangeArgs &a, int qt, int step, hipStream_t s);

// ---- probe path (k_probe.hip): partition index build and filtered probe
constexpr int PROBE_LIST_BLOCK = 4096;  // rows placed by one thread
constexpr int PROBE_MAX_WALK = 256;     // partitions ordered per query
constexpr int PROBE_SORT_MAX = 4096;    // centroids sorted at once by the coarse scan
constexpr int PROBE_COUNT_R = 8;        // rows per thread in one counting step
constexpr int PROBE_FAN = 16;           // partial lists merged by one workgroup
constexpr int PROBE_MAX_GS = 512;       // scoring workgroups per query at most
struct ProbeArgs {
    const void *rows;              // partition-ordered rows [n][dp]
    const float *scale;            // partition-ordered FP8 scales, or null
    int32_t d, dp;
    vrs_dtype store;
    int metric;
    const int32_t *attr;           // partition-ordered predicate columns [n_attr][an]
    int64_t an;
    PredDev pred;
    const float *q;                // [B][d]
    int32_t B, k;
    const void *cent_rows;         // centroid table rows [nlist][cdp] float32
    int32_t cdp, nlist;
    void *ckeys;                   // [B][next_pow2(nlist)] (distance, centroid) keys of the
                                   // coarse scan (nlist <= PROBE_SORT_MAX), or null
    int64_t *coarse_out;           // [B][walk] partitions in centroid order (-1 pads)
    const int64_t *coarse;         // (the same array, read by the walk)
    int32_t walk;                  // partitions ordered per query: min(nlist, 256)
    int32_t nprobe;                // partitions always visited
    int64_t min_cand, cap_c;       // stopping rules of the walk
    const int64_t *list_off;       // [nlist + 1]
    const int32_t *ids;            // rows of every partition, ascending
    int64_t *pre;                  // [B][walk + 1] rows in the first i partitions of the walk
    uint32_t *cnt;                 // [B][walk] qualifying rows of every counted partition
    int64_t *state;                // [B][4] open, walk position, qualifying rows so far, limit
    int32_t w0, w1;                // walk positions counted by this round
    int32_t gc, gs;                // counting / scoring workgroups per query
    int32_t srows;                 // rows per scoring step (256 per thread-row)
    int32_t *taken;                // [B] partitions visited, or null
    uint64_t *part;                // [B][gs][k][2] exact keys of every scoring workgroup
    uint64_t *part2;               // [B][ceil(gs / PROBE_FAN)][k][2] merged groups, or null
    int64_t *out_idx;              // [B][k]
    float *out_dist;               // [B][k]
};
// assign [n] partition of every row -> partition offsets [nlist + 1] and the
// rows of every partition ascending; cnt: [ceil(n / PROBE_LIST_BLOCK)][nlist]
// scratch, size: [nlist] scratch.
hipError_t launch_index_lists(const int64_t *assign, int64_t n, int nlist, uint32_t *cnt, int64_t *size,
                              int64_t *off, int32_t *ids, hipStream_t s);
hipError_t launch_centroid_init(const float *x32, int64_t n, int nlist, int d, float *cent, hipStream_t s);
// Copies of the rows (row_bytes each, a multiple of 16), FP8 scales (or
// null) and n_attr predicate columns (stride an) in the order of ids [n].
hipError_t launch_list_gather(const int32_t *ids, int64_t n, const void *rows, int64_t row_bytes,
                              const float *scale, const int32_t *attr, int n_attr, int64_t an, void *rows_p,
                              float *scale_p, int32_t *attr_p, hipStream_t s);
hipError_t launch_centroid_mean(const float *x32, int nlist, int d, const int64_t *off, const int32_t *ids,
                                float *cent, hipStream_t s);
hipError_t launch_probe(const ProbeArgs &a, hipStream_t s);

// ---- chooser network (k_mlp.hip)
hipError_t launch_mlp_forward(const float *p, const float *x, int nb, float *y, float *act,
                              hipStream_t s);
hipError_t launch_mlp_backward(const float *p, const float *x, const float *y, const float *act,
                               const float *t, const uint8_t *mask, int nb, float inv_count,
                               float *sig, float *sqerr, float *grad, float *loss, hipStream_t s);
hipError_t launch_mlp_adam(float *p, const float *g, float *m, float *v, int step, float lr,
                           float b1, float b2, float eps, hipStream_t s);

}  // namespace vrs
