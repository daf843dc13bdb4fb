/*
 * vrs.h -- filtered exact top-k vector search on one MI355X (gfx950).
 *
 * The library implements the exhaustive scan access path for mixed
 * vector-relational search of Sanca & Ailamaki, "Efficient Data Access Paths
 * for Mixed Vector-Relational Search" (Section 3): for a table R holding a
 * vector column and int32 relational columns, a query vector v, a relational
 * predicate theta and a similarity predicate eps, it returns
 *
 *     sigma_{eps,v,theta}(R) = sigma_eps(v x sigma_theta(R))       (eq. 3)
 *
 * where eps keeps the k qualifying rows nearest to v, ordered by (distance,
 * row id) ascending.  The result is exact (a scan, unlike an index, is exact:
 * Table 1): ids are those of the FP64 definition of the distance and the
 * returned distances are that FP64 value rounded to float32.
 *
 * Conventions shared by every entry point:
 *   - Pointers are DEVICE pointers unless the comment says "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Scan calls are asynchronous on `stream`, never synchronise and never
 *     allocate device memory: the caller owns queries, outputs and the
 *     workspace; the library owns only the table built by vrs_build_table.
 *   - Every argument and shape error is detected on the host before anything
 *     is enqueued; then nothing is launched, outputs are untouched and
 *     vrs_last_error() says why.  No C++ exception crosses this interface.
 *   - Inputs are never modified.
 */
#ifndef VRS_H
#define VRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vrs_table_s *vrs_table; /* opaque, library-owned */
typedef struct vrs_index_s *vrs_index; /* opaque, library-owned */

typedef enum {
    VRS_OK = 0,
    VRS_E_ARG = 1,         /* bad argument or shape */
    VRS_E_NONFINITE = 2,   /* the table holds a NaN/inf (or overflows bfloat16) */
    VRS_E_NOMEM = 3,       /* device allocation failed (vrs_build_table only) */
    VRS_E_UNSUPPORTED = 4, /* valid but not implemented combination */
    VRS_E_HIP = 5,         /* a HIP runtime call failed */
    VRS_E_WORKSPACE = 6    /* workspace missing or smaller than required */
} vrs_status;

/* Distance between query q and stored row x (smaller = nearer):
 *   VRS_L2SQ: sum_j (q_j - x_j)^2            (squared Euclidean)
 *   VRS_IP:   -sum_j q_j x_j                 (negated inner product)
 * IP on a table built with normalize=1 ranks rows by cosine similarity to q
 * (the tensor formulation on normalised matrices, Section 3.1). */
typedef enum { VRS_L2SQ = 0, VRS_IP = 1 } vrs_metric;

/* Storage type of the vector column.  BF16 rounds to nearest-even; FP8 is OCP
 * e4m3fn (max 448, saturating, round to nearest-even) with one float32 scale
 * per row, scale_i = max_j |x_ij| / 448 (1 for an all-zero row) and stored
 * value scale_i * e4m3(x_ij / scale_i).  BF16 and FP8 tables support IP only. */
typedef enum { VRS_F32 = 0, VRS_BF16 = 1, VRS_FP8E4M3 = 2 } vrs_dtype;

/* One range term of a relational predicate: lo <= A[col][i] < hi, with int64
 * bounds so that full and empty ranges over int32 columns are expressible. */
typedef struct {
    int32_t col;
    int32_t _pad;
    int64_t lo, hi;
} vrs_range;

#define VRS_MAX_TERMS 4

/* Largest query batch B of one call (queries are a grid dimension of the
 * merge and rerank launches); larger batches are VRS_E_ARG. */
#define VRS_MAX_BATCH 65535

/* A conjunction of nterms range terms; nterms == 0 selects every row. */
typedef struct {
    int32_t nterms;
    int32_t _pad;
    vrs_range term[VRS_MAX_TERMS];
} vrs_pred;

enum { VRS_STRATEGY_AUTO = 0, VRS_STRATEGY_MASK = 1, VRS_STRATEGY_GATHER = 2 };
enum { VRS_CHOOSER_LEARNED = 0, VRS_CHOOSER_HEURISTIC = 1 };

/* Optional knobs (pass NULL for defaults).  None of them changes results.
 *   strategy:    AUTO, MASK (compute-then-mask: every row tile is scanned and
 *                non-qualifying rows are masked out, eq. 3 middle form) or
 *                GATHER (predicate first into a selection vector, then only
 *                qualifying rows are compared, eq. 3 right form).
 *   tile:        kernel configuration id (vrs_num_tiles()), -1 = auto.
 *   chooser:     LEARNED (MLP, if weights are loaded) or HEURISTIC.
 *   kprime_mult: screening survivors per query k' = kprime_mult * k when > 0;
 *                0 = default (max(2k, k+32) for FP32 tables, max(4k, k+32)
 *                for bfloat16 / FP8 tables), at most 1024.
 *   n_valid:     [B] int32 out: min(k_b, |sigma_theta(R)|), or NULL.
 *   certified:   [B] uint8 out: 1 if the screened candidates provably held the
 *                exact top-k, 0 if the exact FP64 fallback pass ran; or NULL.
 *   passes:      MFMA screening in one pass (1) or in two (2: a prefix of
 *                every row chunk, a merge whose K-th key then bounds every
 *                chunk, the rest of every chunk); 0 = two when a chunk holds
 *                at least 2048 rows.  Results do not depend on it; streaming
 *                tiles always use one pass.
 *   err_ratio:   [B] float out, or NULL: a diagnostic of the certificate's
 *                screening error model.  For query b, the largest
 *                |screening distance - exact distance| / E over its reranked
 *                keys (the k' survivors and the (k'+1)-th key, whose exact
 *                distance is then computed as well), where E is the bound the
 *                certificate uses for that distance.  Values below 1 mean the
 *                model held on every key seen. */
typedef struct {
    int32_t strategy;
    int32_t tile;
    int32_t chooser;
    int32_t kprime_mult;
    int32_t *n_valid;
    uint8_t *certified;
    int32_t passes;
    int32_t _pad;
    float *err_ratio;
} vrs_opts;

/* Build a table (the column store of Section 3) from float32 rows.
 *   vec:       [n][d] float32 row-major (device).
 *   attr:      [n_attr][n] int32 column-major (device), may be NULL if n_attr == 0.
 *   store:     storage dtype; normalize = 1 divides every row by its FP64 L2
 *              norm first (rounded to float32; all-zero rows unchanged).
 *   out:       host pointer receiving the handle.
 * 1 <= d <= 4096, 1 <= n < 2^31, 0 <= n_attr <= 64.  Synchronises `stream`
 * once to check that every stored value is finite (VRS_E_NONFINITE if not). */
vrs_status vrs_build_table(const float *vec, int64_t n, int32_t d, const int32_t *attr,
                           int32_t n_attr, vrs_dtype store, int32_t normalize, void *stream,
                           vrs_table *out);

/* Free a table (waits for nothing: the caller must not have scans in flight). */
vrs_status vrs_destroy_table(vrs_table t);

/* Table shape: any out pointer (host) may be NULL. */
vrs_status vrs_table_info(vrs_table t, int64_t *n, int32_t *d, int32_t *n_attr,
                          vrs_dtype *store, double *max_row_norm);

/* Copy the stored vector column out, unpadded, to device buffers:
 * rows_out [n][d] of float32 / uint16 (bfloat16 bits) / uint8 (e4m3 codes);
 * scale_out [n] float32 for FP8 tables (NULL otherwise). */
vrs_status vrs_table_export(vrs_table t, void *rows_out, float *scale_out, void *stream);

/* Bytes of workspace that a scan of B queries with k <= k_max needs under
 * `opts` (host pointers; opts may be NULL). */
vrs_status vrs_scan_workspace_bytes(vrs_table t, int32_t B, int32_t k_max, const vrs_opts *opts,
                                    size_t *bytes);

/* The relational selection sigma_theta(R) alone (eq. 3, inner part):
 * ascending qualifying row ids into ids_out [n] int32 and their number into
 * count_out [1] int64.  Uses ws of vrs_select_workspace_bytes(). */
vrs_status vrs_select_workspace_bytes(vrs_table t, size_t *bytes);
vrs_status vrs_select(vrs_table t, const vrs_pred *pred /* host */, int32_t *ids_out,
                      int64_t *count_out, void *ws, size_t ws_bytes, void *stream);

/* Filtered exact top-k for B queries sharing one predicate: the query of
 * Section 3, eq. 3 (the k rows of sigma_theta(R) nearest to q, by the exact
 * distance of the definition, ties by row id), computed by screening in FP32
 * (the strategy, mask or gather, of Section 3.2; the tensor formulation of
 * Section 3.1 for batches), an FP64 rerank of the k' survivors and a
 * certificate, with an exact fallback for an uncertified query.
 *   q:        [B][d] float32 (device), finite.
 *   pred:     host pointer, one conjunction for the whole batch.
 *   1 <= k <= 256.
 *   out_idx:  [B][k] int64 row ids, ascending by (distance, id); -1 pads.
 *   out_dist: [B][k] float32 distances (FP64 value rounded); +inf pads.
 *   ws:       >= vrs_scan_workspace_bytes(t, B, k, opts) bytes, 256-aligned. */
vrs_status vrs_scan_topk(vrs_table t, const float *q, int32_t B, const vrs_pred *pred, int32_t k,
                         vrs_metric metric, int64_t *out_idx, float *out_dist, void *ws,
                         size_t ws_bytes, const vrs_opts *opts, void *stream);

/* vrs_scan_topk without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * vrs_scan_topk; the workspace is a static device array of
 * VRS_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.  A call whose scan needs more workspace than that
 * (vrs_scan_workspace_bytes) returns VRS_E_WORKSPACE and launches nothing;
 * nothing is allocated.  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (two streams, two threads) race, so the caller
 * serialises them. */
#define VRS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
vrs_status vrs_scan_topk_noalloc(vrs_table t, const float *q, int32_t B, const vrs_pred *pred,
                                 int32_t k, vrs_metric metric, int64_t *out_idx, float *out_dist,
                                 const vrs_opts *opts, void *stream);

/* Threshold selection: for each query b, every row i that satisfies the
 * relational predicate and whose exact FP64 distance (the distance of this
 * header) is below thr[b], ascending by row id.  This is the selection with
 * a query vector and a similarity predicate of Section 3 (eq. 1), with the
 * relational predicate pushed down as in eq. 3; the paper's evaluation uses
 * a cosine-similarity threshold (Section 5, "Dataset"): on a table built
 * with normalize=1 and a unit-norm query, cosine similarity > t is
 * VRS_IP distance < -t.
 *   q:         [B][d] float32 (device), finite.
 *   pred:      host pointer, one conjunction for the whole batch.
 *   thr:       [B] float64 (device); +inf selects every qualifying row,
 *              -inf and NaN select none.
 *   cap:       result slots per query (>= 1).
 *   out_idx:   [B][cap] int64: the first min(count, cap) selected row ids,
 *              ascending, then -1.
 *   out_dist:  [B][cap] float32: their exact distances rounded to float32,
 *              then +inf.
 *   out_count: [B] int64: the number of selected rows (may exceed cap; then
 *              out_idx holds the cap lowest ids).
 *   ws:        >= vrs_range_workspace_bytes(t, B, cap) bytes, 256-aligned.
 *   opts:      may be NULL; only opts->strategy is used (AUTO, MASK or
 *              GATHER; results do not depend on it).
 * The FP32 screening admits every row whose screening distance is below
 * thr[b] plus a bound on its error; every admitted row is then decided by
 * its exact FP64 distance, so the set is exact.  A query with more admitted
 * rows than its candidate slots is decided by an exact pass over every
 * qualifying row. */
vrs_status vrs_range_workspace_bytes(vrs_table t, int32_t B, int32_t cap, size_t *bytes);
vrs_status vrs_scan_range(vrs_table t, const float *q, int32_t B, const vrs_pred *pred,
                          vrs_metric metric, const double *thr, int32_t cap, int64_t *out_idx,
                          float *out_dist, int64_t *out_count, void *ws, size_t ws_bytes,
                          const vrs_opts *opts, void *stream);

/* Vector join: for every row r of R, taken as its stored vector (float32
 * and bfloat16 values exactly, an FP8 value scale * code rounded to the
 * nearest float32), the exact top-k rows of S satisfying pred, as
 * vrs_scan_topk returns them for that query.  This is the N:N strategy of
 * Section 3.1 with a whole relation as the query batch (the paper names
 * joins as the large-batch use of the tensor form, Section 5.2).  R and S
 * may be the same table (then every row finds itself at distance 0 when
 * L2SQ is used and no lower-id duplicate exists).
 *   pred:     host pointer, a conjunction over S's attributes.
 *   out_idx:  [R.n][k] int64, out_dist: [R.n][k] float32 (device).
 *   ws:       >= vrs_join_workspace_bytes(R, S, k, opts) bytes, 256-aligned.
 *   opts:     as for vrs_scan_topk; n_valid, certified and err_ratio, when
 *             given, hold R.n entries.
 * R.d must equal S.d; L2SQ needs a float32 table S. */
vrs_status vrs_join_workspace_bytes(vrs_table R, vrs_table S, int32_t k, const vrs_opts *opts,
                                    size_t *bytes);
vrs_status vrs_join_topk(vrs_table R, vrs_table S, const vrs_pred *pred, int32_t k, vrs_metric metric,
                         int64_t *out_idx, float *out_dist, void *ws, size_t ws_bytes,
                         const vrs_opts *opts, void *stream);

/* Probe-based access path (Section 4): a partition index over a table's
 * vector column and its filtered probe with pre-filtering (Section 4.1: the
 * relational predicate decides which rows may enter the result, not which
 * partitions are visited).  The result is approximate: the exact top-k of
 * the rows the probe collects.  (The paper's index is HNSW; this one is
 * k-means partitions, which turn a probe into a few short scans.)
 *
 * vrs_index_build: k-means with nlist partitions (1 <= nlist <= min(16384,
 * n)) and iters Lloyd iterations (0..100) on the stored vectors, squared
 * L2: the initial centroids are the stored rows floor(i n / nlist); every
 * assignment is the row's exact nearest centroid (by FP64 distance, then
 * centroid id); a centroid moves to its partition's mean (an FP64 running
 * sum over the partition's rows in ascending order, divided by the count,
 * rounded to float32; an empty partition keeps its centroid).  The index
 * keeps its own copy of the stored rows (and FP8 scales) and of the
 * predicate columns in partition order, so that a probe reads every
 * partition contiguously: about the table's size again in device memory.
 * The table must outlive the index.  Allocates and synchronises `stream`. */
vrs_status vrs_index_build(vrs_table t, int32_t nlist, int32_t iters, void *stream, vrs_index *out);
vrs_status vrs_index_destroy(vrs_index ix);
/* nlist and the largest partition (host pointers, may be NULL). */
vrs_status vrs_index_info(vrs_index ix, int32_t *nlist, int64_t *max_list);
/* Device copies: centroids [nlist][d] float32, partition offsets [nlist+1]
 * int64, the rows of every partition ascending [n] int32 (any may be NULL). */
vrs_status vrs_index_export(vrs_index ix, float *centroids, int64_t *list_off, int32_t *list_ids,
                            void *stream);
/* Scan or probe (the access-path choice of Section 5.3): estimated times
 * (ms, host pointers, may be NULL) of the exact scan and of the probe for B
 * queries with this predicate (selectivity s from the table's column
 * histograms) and k.  The scan: the installed chooser network's predicted
 * time of the arm it would pick, else a bytes-moved model (the predicate
 * columns and either every row or the qualifying ones, once for the batch).
 * The probe: per query the rows its walk visits (at least nprobe
 * partitions of the size-biased mean partition size, more until k rows
 * qualify, at most cap_c rows), then a linear time model of the predicate
 * columns and qualifying rows the batch reads, fitted to measured probes.
 * use_probe = 1 when the probe is estimated faster.  The probe's results are
 * approximate: a caller that needs the exact answer scans. */
vrs_status vrs_plan_access(vrs_index ix, int32_t B, const vrs_pred *pred, int32_t k, int32_t nprobe,
                           int64_t cap_c, double *scan_ms, double *probe_ms, int32_t *use_probe);
/* Filtered probe of B queries sharing one predicate.  Each query walks the
 * partitions in the order of their centroids' distance to it (exact,
 * squared L2, ties by centroid id; at most min(nlist, 256) partitions); a
 * visited partition contributes its rows that satisfy the predicate.  The
 * first nprobe partitions (1 <= nprobe <= min(256, nlist)) are visited;
 * past them the walk continues only while fewer than min_cand rows
 * qualified (with pre-filtering a selective predicate makes the probe visit
 * more of the index).  A partition that would take the rows visited past
 * cap_c ends the walk (the first partition is always visited).  The result
 * is the exact top-k of the collected rows by (FP64 distance, id), padded
 * with (-1, +inf); out_taken [B] (or NULL) receives the number of
 * partitions visited.  ws >= vrs_probe_workspace_bytes(...). */
vrs_status vrs_probe_workspace_bytes(vrs_index ix, int32_t B, int32_t k, int32_t nprobe, int64_t cap_c,
                                     size_t *bytes);
vrs_status vrs_probe_topk(vrs_index ix, const float *q, int32_t B, const vrs_pred *pred, int32_t k,
                          vrs_metric metric, int32_t nprobe, int64_t min_cand, int64_t cap_c,
                          int64_t *out_idx, float *out_dist, int32_t *out_taken, void *ws,
                          size_t ws_bytes, void *stream);

/* Filtered exact top-k for B queries, each with its own predicate and k:
 * the selection of Section 3 (brute-force search with a relational
 * predicate) per query.  The paper's batched (tensor) form stages one shared
 * filter before the batch (Sections 3.1-3.2); here every query may differ.
 *   preds:    [B] vrs_pred (device).  A malformed predicate (column outside
 *             the table, more than VRS_MAX_TERMS terms, empty range) selects
 *             no row; it is not an error, since it is only seen on the device.
 *   ks:       [B] int32 (device), clamped into [1, k_max]; 1 <= k_max <= 256.
 *   out_idx/out_dist: [B][k_max]; row b holds k_b results then padding.
 *   ws:       >= vrs_batched_workspace_bytes(t, B, k_max, metric, opts).
 *   opts->tile: batched configuration in [0, vrs_batched_num_configs()), or
 *             -1 for the one vrs_batched_tune() chose for this (table, B,
 *             k_max, metric), else a default.  opts->strategy and
 *             opts->chooser are ignored.
 * Each query is screened either densely (MFMA kernel shared by 64 queries,
 * predicate checked per pair) or, when it qualifies few rows, through its own
 * selection vector (gather kernel); the split is made on the device.  One
 * launch sequence, no host synchronisation and no memset, so it can be
 * captured into a HIP graph (vrs_batched_graph_create). */
vrs_status vrs_scan_topk_batched(vrs_table t, const float *q, int32_t B, const vrs_pred *preds,
                                 const int32_t *ks, int32_t k_max, vrs_metric metric,
                                 int64_t *out_idx, float *out_dist, void *ws, size_t ws_bytes,
                                 const vrs_opts *opts, void *stream);

/* Workspace of vrs_scan_topk_batched (host pointers; opts may be NULL). */
vrs_status vrs_batched_workspace_bytes(vrs_table t, int32_t B, int32_t k_max, vrs_metric metric,
                                       const vrs_opts *opts, size_t *bytes);

/* Number of batched configurations (sparse-query row cap, dense work per
 * workgroup round, rows per sparse work item). */
int32_t vrs_batched_num_configs(void);

/* Autotuner: runs vrs_scan_topk_batched once per configuration on these
 * inputs, times each (best of two runs, HIP events on `stream`; this call
 * synchronizes), remembers the fastest for (t, B, k_max, metric, k' rule) and
 * leaves its results in the outputs.  best: host int32; ms: host
 * float[vrs_batched_num_configs()] or NULL.  Every configuration returns the
 * same results. */
vrs_status vrs_batched_tune(vrs_table t, const float *q, int32_t B, const vrs_pred *preds,
                            const int32_t *ks, int32_t k_max, vrs_metric metric, int64_t *out_idx,
                            float *out_dist, void *ws, size_t ws_bytes, const vrs_opts *opts,
                            void *stream, int32_t *best, float *ms);

/* HIP-graph form of vrs_scan_topk_batched: the whole launch sequence for
 * these buffers (queries, predicates, ks, outputs, workspace, opts->n_valid
 * and opts->certified pointers) captured once and replayed by
 * vrs_graph_launch; the caller rewrites the buffers' contents between
 * launches.  With opts->tile == -1 the configuration is autotuned first
 * (as vrs_batched_tune) unless already known.  Creation runs the sequence
 * once eagerly (its results land in the outputs) and synchronizes `stream`.
 * The buffers must stay allocated while the graph exists. */
typedef struct vrs_graph_s *vrs_graph;
vrs_status vrs_batched_graph_create(vrs_table t, const float *q, int32_t B, const vrs_pred *preds,
                                    const int32_t *ks, int32_t k_max, vrs_metric metric,
                                    int64_t *out_idx, float *out_dist, void *ws, size_t ws_bytes,
                                    const vrs_opts *opts, void *stream, vrs_graph *out);
/* The launch sequence of vrs_scan_topk (Section 3, eq. 3; arguments as
 * there) for these buffers (queries, outputs, workspace and the opts
 * pointers) and this predicate, k and opts, with the access path the planner
 * picks now, captured once into a graph that vrs_graph_launch replays: one
 * launch instead of one per kernel, for callers that repeat a call (a
 * serving loop over new query vectors written into q).  The caller may
 * rewrite the buffers' contents between replays, not their addresses; the
 * table must not change.  Creation runs the call once eagerly (its results
 * land in the outputs) and synchronizes `stream`.  The buffers and the table
 * must stay allocated while the graph exists.  vrs_graph_config returns -1. */
vrs_status vrs_scan_graph_create(vrs_table t, const float *q, int32_t B, const vrs_pred *pred, int32_t k,
                                 vrs_metric metric, int64_t *out_idx, float *out_dist, void *ws,
                                 size_t ws_bytes, const vrs_opts *opts, void *stream, vrs_graph *out);
/* Enqueue one replay on `stream` (asynchronous). */
vrs_status vrs_graph_launch(vrs_graph g, void *stream);
/* The configuration a graph was captured with. */
int32_t vrs_graph_config(vrs_graph g);
vrs_status vrs_graph_destroy(vrs_graph g);

/* Number of kernel configurations ("tiles") the planner chooses from.  An
 * access path ("arm") is strategy x tile: arm = (strategy - 1) * tiles + tile
 * with strategy MASK = 1, GATHER = 2. */
int32_t vrs_num_tiles(void);

/* ---- Learned access-path chooser (workload-driven access path selection,
 * Sections 3.2 and 5: the best scan strategy depends on selectivity,
 * dimensionality and the number of concurrent queries).
 *
 * A 6 -> 64 -> 64 -> 16 perceptron with ReLU (FP32) maps standardised
 * features (ln n, ln d, ln B, ln estimated selectivity, ln k, storage dtype)
 * to a predicted ln(milliseconds) per arm; the planner takes the arm with the
 * smallest prediction among the valid ones.  It never changes results (every
 * arm returns the same exact top-k).  Parameter block (floats, in order):
 * W1[6][64], b1[64], W2[64][64], b2[64], W3[64][16], b3[16]; a layer computes
 * out[j] = b[j] + sum_i in[i] * W[i][j]. */
#define VRS_MLP_IN 6
#define VRS_MLP_HIDDEN 64
#define VRS_MLP_OUT 16
#define VRS_MLP_PARAMS 5648

/* Forward pass of nb samples: x [nb][6] -> y [nb][16]; act [nb][128] keeps the
 * hidden activations for a backward pass (NULL when none follows). */
vrs_status vrs_mlp_forward(const float *params, const float *x, int32_t nb, float *y, float *act,
                           void *stream);

/* Gradient of the masked mean squared error sum(mask (y - target)^2) / count,
 * count = number of set mask entries (> 0): writes grad [VRS_MLP_PARAMS] and,
 * if loss != NULL, loss [1].  Scratch: sig [nb][144], sqerr [nb] floats. */
vrs_status vrs_mlp_backward(const float *params, const float *x, const float *y,
                            const float *act, const float *target, const uint8_t *mask,
                            int32_t nb, int32_t count, float *sig, float *sqerr, float *grad,
                            float *loss, void *stream);

/* One Adam step (Kingma & Ba) on all parameters; step counts from 1. */
vrs_status vrs_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t step,
                        float lr, float beta1, float beta2, float eps, void *stream);

/* Install chooser weights from host memory: params [VRS_MLP_PARAMS], feature
 * mean and standard deviation [6] each.  vrs_chooser_clear() returns the
 * planner to the selectivity-threshold heuristic. */
vrs_status vrs_chooser_set(const float *params, const float *feat_mean, const float *feat_std);
vrs_status vrs_chooser_clear(void);

/* The installed network's pick among the allowed arms (host inference, the
 * same computation the planner runs per call): feats [6] as vrs_plan returns
 * them, allowed [2 * vrs_num_tiles()] uint8 (arm = (strategy - 1) *
 * vrs_num_tiles() + tile), *arm (host) = the allowed arm with the lowest
 * predicted time, or -1 when no network is installed or nothing is allowed. */
vrs_status vrs_chooser_pick(const float *feats, const uint8_t *allowed, int32_t *arm);

/* Load chooser weights from a file written by the training tool (magic
 * "VRSCHOOS", version 1, then the params, mean and std as little-endian
 * float32).  On a missing or corrupt file the chooser stays on the heuristic
 * and the call returns VRS_E_ARG. */
vrs_status vrs_chooser_load(const char *path);

/* The planner's decision for a call without running it (host only): raw
 * features [6] (host, may be NULL), and the strategy / tile AUTO would use
 * under opts->chooser. */
vrs_status vrs_plan(vrs_table t, int32_t B, const vrs_pred *pred, int32_t k, vrs_metric metric,
                    const vrs_opts *opts, float *features, int32_t *strategy, int32_t *tile);

/* A non-owning view of the first n rows of a table (same storage; destroy
 * the view before its parent).  Used to time scans at many table sizes. */
vrs_status vrs_table_view(vrs_table t, int64_t n, vrs_table *out);

/* Stage timing for measurement tools.  While enabled, every scan records a
 * pair of HIP events around each of its stages on the scan's own stream:
 *   0 prep, 1 select (gather only), 2 screen, 3 merge, 4 rerank, 5 fallback.
 * vrs_stage_times() waits for the recorded events, adds each stage's elapsed
 * milliseconds and launch count into ms[VRS_NUM_STAGES] / calls[...] (host),
 * and forgets the records.  Process-wide; not for concurrent scans. */
#define VRS_NUM_STAGES 6
vrs_status vrs_profile(int32_t enable);
vrs_status vrs_stage_times(double *ms, int64_t *calls);

/* Thread-local description of the last error (valid until the next call). */
const char *vrs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VRS_H */
