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
    // per-column equi-width histograms for selectivity estimates
    std::vector<int32_t> amin, amax;
    std::vector<std::vector<uint32_t>> hist;
};

namespace vrs {

constexpr int HIST_BINS = 256;

int elem_bytes(vrs_dtype t);
int pad_dim(int d, vrs_dtype t);

// ---- build kernels (k_build.hip)
hipError_t launch_build_rows(const float *vec, int64_t n, int32_t d, int32_t dp, vrs_dtype store,
                             int normalize, void *rows, float *scale, float *norm2,
                             unsigned long long *max_norm_bits, int *bad_flag, hipStream_t s);
hipError_t launch_attr_stats(const int32_t *attr, int64_t n, int32_t n_attr, int32_t *amin,
                             int32_t *amax, uint32_t *hist, hipStream_t s);

// ---- predicate pass (k_select.hip)
constexpr int SEL_BLOCK_ROWS = 8192;
hipError_t launch_select(const int32_t *attr, int64_t n, int64_t an, const PredDev &p,
                         uint32_t *bitmap, uint32_t *blkcnt, int32_t *ids, int64_t *count,
                         hipStream_t s);

// ---- query preparation (k_finish.hip)
hipError_t launch_prep_queries(const float *q, int32_t B, int32_t d, int32_t dp, float *qp,
                               double *qnorm, float *qn2, uint16_t *qhl, uint64_t *gthr,
                               int32_t *fail_count, hipStream_t s);
int screen_mfma_occupancy(int Kp, int CB, int qm);
hipError_t launch_prep_batched(const vrs_pred *preds, const int32_t *ks, int32_t B, int32_t kmax,
                               int32_t n_attr, int kmult, int f32_rule, PredDev *out,
                               int32_t *kc, int32_t *kps, hipStream_t s);

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
    uint64_t *partials;            // [B][n_chunks][K]
    uint64_t *cbuf;                // [B][n_chunks][CB] candidate buffers (MFMA kernels)
    uint64_t *gthr;                // [B] smallest K-th key published by any chunk
};
hipError_t launch_screen_stream(const ScreenArgs &a, int qt, hipStream_t s);
size_t screen_stream_lds(int qt, int Kp, int CB, int dp);
hipError_t launch_screen_mfma(const ScreenArgs &a, int qm, hipStream_t s);
size_t screen_mfma_lds(int dp, int qm);
hipError_t launch_screen_mfma_bf16(const ScreenArgs &a, hipStream_t s);
size_t screen_mfma_bf16_lds();
bool screen_mfma_bf16_supported(int dp, vrs_dtype store, int metric, int Kp, int CB);
bool screen_mfma_supported(int dp, vrs_dtype store, int Kp, int CB);

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
    uint64_t *merge_mid;           // [B][ceil(n_chunks/2048)][K] (two-level merge)
    uint64_t *merged;              // [B][K]
    double rel, abs_ip, abs_l2, max_norm;  // screening error model
    int32_t *fail_list;            // [B]
    int32_t *fail_count;           // [1]
    int64_t *out_idx;
    float *out_dist;
    int32_t *n_valid;
    uint8_t *certified;
    // exact fallback
    int32_t fb_rows_per_chunk, fb_chunks, fb_slots;
    uint64_t *fb_partials;         // [fb_slots][fb_chunks][kmax][2]
};
hipError_t launch_merge(const FinishArgs &a, hipStream_t s);
hipError_t launch_rerank(const FinishArgs &a, hipStream_t s);
hipError_t launch_fallback(const FinishArgs &a, hipStream_t s);

// ---- chooser network (k_mlp.hip)
hipError_t launch_mlp_forward(const float *p, const float *x, int nb, float *y, float *act,
                              hipStream_t s);
hipError_t launch_mlp_backward(const float *p, const float *x, const float *y, const float *act,
                               const float *t, const uint8_t *mask, int nb, float inv_count,
                               float *sig, float *sqerr, float *grad, float *loss, hipStream_t s);
hipError_t launch_mlp_adam(float *p, const float *g, float *m, float *v, int step, float lr,
                           float b1, float b2, float eps, hipStream_t s);

}  // namespace vrs
