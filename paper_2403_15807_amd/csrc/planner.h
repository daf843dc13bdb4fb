// planner.h -- access-path planning for one scan call: strategy (mask vs
// gather, eq. 3), kernel configuration ("tile"), list sizes, workspace
// layout, and the launch sequence.
#pragma once

#include <string>

#include "internal.h"

namespace vrs {

// Kernel configurations the planner and the chooser pick from.
struct TileCfg {
    int kind;       // 0 = VALU streaming kernel, 1 = MFMA kernel
    int qt;         // queries per workgroup
    int wg_target;  // workgroups to aim for (fills 256 CUs several times)
};
int planner_num_tiles();
const TileCfg &planner_tile(int id);

// k' = screening survivors per query.
int kprime_rule(int k, vrs_dtype store, int kmult);
// Candidate-buffer length of the MFMA screening kernels for a list of Kp.
int mfma_cb(int Kp);

struct Plan {
    int strategy;        // VRS_STRATEGY_MASK or VRS_STRATEGY_GATHER
    int tile;            // index into the tile table
    bool mfma;           // MFMA screening kernel
    int qt, n_qtiles, n_chunks;
    int kprime, K, Kp, CB;
    int fb_chunks, fb_rows_per_chunk;
    bool two_pass;       // MFMA screening in two passes (a prefix sample, then everything)
    // workspace offsets (bytes)
    size_t o_qp, o_qnorm, o_qn2, o_qhl, o_gthr, o_cbuf, o_bitmap, o_blk, o_sel, o_selcnt, o_part, o_heads, o_fills, o_mid, o_merged, o_rrdist, o_fail,
        o_failcnt, o_fb, o_preds, o_kc, o_kps, total;
};

double estimate_selectivity(const vrs_table_s *t, const PredDev &p);

bool planner_tile_ok(const vrs_table_s *t, int B, int kmax, const vrs_opts *opts, int tile);

// Workspace bytes covering every plan the planner may pick for (B, k_max, opts).
size_t plan_workspace(const vrs_table_s *t, int B, int kmax, const vrs_opts *opts);

hipError_t run_scan(const vrs_table_s *t, const float *q, int B, const PredDev &p,
                    const vrs_pred *preds, const int32_t *ks, int k, vrs_metric metric,
                    int64_t *out_idx, float *out_dist, void *ws, const vrs_opts *opts,
                    hipStream_t s);

// Stage timing (vrs_profile / vrs_stage_times).
void prof_begin(int stage, hipStream_t s);
void prof_end(int stage, hipStream_t s);
void prof_enable(bool on);
void prof_quiet(bool on);  // this thread records no stage events (graph capture)
hipError_t prof_collect(double *ms, int64_t *calls);

// Planner decision (strategy, tile) for a call, with its raw chooser features.
void plan_decide(const vrs_table_s *t, int B, const PredDev &p, bool batched, int k, int metric,
                 const vrs_opts *opts, float feats[6], int *strategy_out, int *tile_out);

// Learned chooser (host inference of the MLP).
bool chooser_set(const float *params, const float *mean, const float *stdv);
void chooser_clear();
bool chooser_load(const char *path, std::string *err);
bool chooser_ready();
// Returns the arm index (strategy * num_tiles + tile) with the lowest
// predicted time among the allowed arms, or -1.
int chooser_pick(const float feats[6], const bool *allowed, int n_arms);
// The same, with the picked arm's predicted log(ms) in *value.
int chooser_pick_value(const float feats[6], const bool *allowed, int n_arms, float *value);
// The learned chooser's predicted time (ms) of its pick for a single-predicate
// scan call, or -1 without a network.
double plan_predict_ms(const vrs_table_s *t, int B, const PredDev &p, int k, int metric);

// ---- threshold selection (range.cpp)
size_t range_workspace(const vrs_table_s *t, int B, int cap);
hipError_t run_range(const vrs_table_s *t, const float *q, int B, const PredDev &p, vrs_metric metric,
                     const double *thr, int cap, int64_t *out_idx, float *out_dist, int64_t *out_count,
                     void *ws, const vrs_opts *opts, hipStream_t s);

// ---- vector join (join.cpp)
size_t join_workspace(const vrs_table_s *R, const vrs_table_s *S, int k, const vrs_opts *opts);
hipError_t run_join(const vrs_table_s *R, const vrs_table_s *S, const PredDev &p, int k,
                    vrs_metric metric, int64_t *out_idx, float *out_dist, void *ws,
                    const vrs_opts *opts, hipStream_t s);

// ---- probe path (probe.cpp)
hipError_t index_build(const vrs_table_s *t, int nlist, int iters, hipStream_t s, vrs_index_s **out,
                       std::string *err);
void index_free(vrs_index_s *ix);
void access_costs(const vrs_index_s *ix, int B, const PredDev &p, int k, int nprobe, int64_t cap_c,
                  double *scan_ms, double *probe_ms);
size_t probe_workspace(const vrs_index_s *ix, int B, int k, int nprobe, int64_t cap_c);
hipError_t run_probe(const vrs_index_s *ix, const float *q, int B, const PredDev &p, int k, vrs_metric metric,
                     int nprobe, int64_t min_cand, int64_t cap_c, int64_t *out_idx, float *out_dist,
                     int32_t *out_taken, void *ws, hipStream_t s);

// ---- batched uneven form (batched.cpp)
// A configuration of the batched launch: queries qualifying at most
// cap_frac * n rows go to the sparse gather kernel, the dense kernel aims at
// `rounds` resident-workgroup rounds of work items, and sparse items hold
// about seg_rows rows.
struct BatchCfg {
    double cap_frac;
    int rounds;
    int seg_rows;
};
int batched_num_cfgs();
const BatchCfg &batched_cfg(int i);
// The persistent dense kernel exists for this table, k_max and metric.
bool batched_native(const vrs_table_s *t, int kmax, int metric, const vrs_opts *opts);
// Workspace bytes covering every configuration.
size_t batched_workspace(const vrs_table_s *t, int B, int kmax, int metric, const vrs_opts *opts);
hipError_t run_batched(const vrs_table_s *t, const float *q, int B, const vrs_pred *preds,
                       const int32_t *ks, int kmax, vrs_metric metric, int64_t *out_idx,
                       float *out_dist, void *ws, const vrs_opts *opts, int cfg, hipStream_t s);
// Configuration for a call: opts->tile if set, else the tuned one for this
// (table, B, k_max, metric) if known, else the default.
int batched_pick(const vrs_table_s *t, int B, int kmax, int metric, const vrs_opts *opts);
// The tuned configuration for this shape, or -1.
int batched_tuned(const vrs_table_s *t, int B, int kmax, int metric, const vrs_opts *opts);
// Times every configuration on the given inputs (synchronizes), remembers
// and returns the fastest; ms[i] = time of configuration i (or -1).
hipError_t batched_tune(const vrs_table_s *t, const float *q, int B, const vrs_pred *preds,
                        const int32_t *ks, int kmax, vrs_metric metric, int64_t *out_idx,
                        float *out_dist, void *ws, const vrs_opts *opts, hipStream_t s, int *best,
                        float *ms);

}  // namespace vrs
