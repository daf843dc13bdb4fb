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

/* Filtered exact top-k for B queries sharing one predicate.
 *   q:        [B][d] float32 (device), finite.
 *   pred:     host pointer, one conjunction for the whole batch.
 *   1 <= k <= 256.
 *   out_idx:  [B][k] int64 row ids, ascending by (distance, id); -1 pads.
 *   out_dist: [B][k] float32 distances (FP64 value rounded); +inf pads.
 *   ws:       >= vrs_scan_workspace_bytes(t, B, k, opts) bytes, 256-aligned. */
vrs_status vrs_scan_topk(vrs_table t, const float *q, int32_t B, const vrs_pred *pred, int32_t k,
                         vrs_metric metric, int64_t *out_idx, float *out_dist, void *ws,
                         size_t ws_bytes, const vrs_opts *opts, void *stream);

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
