// k_finish.hip -- everything after screening:
//   prep:     pad queries to the stored row width, FP64 query norms, reset
//             the fallback counter (a kernel, not a memset, so the sequence
//             can be captured into a HIP graph);
//   merge:    per query, the K smallest keys over all chunk lists (the
//             (k'+1)-th key bounds every candidate that was not kept);
//   rerank:   FP64 distances of the k' survivors with the exact formula of
//             the definition (coordinates in ascending order, one fused
//             multiply-add each), order by (distance, id), certificate;
//   fallback: for the queries whose certificate failed, an exact FP64 scan
//             of every qualifying row with (distance, id) keys.
#include "internal.h"

namespace vrs {

namespace {

__global__ __launch_bounds__(256) void prep_kernel(const float *__restrict__ q, int d, int dp,
                                                   float *__restrict__ qp,
                                                   double *__restrict__ qnorm,
                                                   int32_t *__restrict__ fail_count) {
    const int b = blockIdx.x;
    if (b == 0 && threadIdx.x == 0) *fail_count = 0;
    __shared__ double red[256];
    double acc = 0.0;
    for (int j = threadIdx.x; j < dp; j += 256) {
        float v = j < d ? q[(int64_t)b * d + j] : 0.0f;
        qp[(int64_t)b * dp + j] = v;
        acc += (double)v * (double)v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) qnorm[b] = sqrt(red[0]) * (1.0 + 0x1p-40);
}

// FP64 value of stored element j of row `row` as the exact formula uses it:
// the float32 / bfloat16 value, or the unscaled e4m3 code value.
template <int STORE>
__device__ __forceinline__ double code_at(const void *rows, int64_t row, int dp, int j) {
    if (STORE == VRS_F32) return (double)((const float *)rows)[row * dp + j];
    if (STORE == VRS_BF16) return (double)bf16_to_f32(((const uint16_t *)rows)[row * dp + j]);
    return (double)e4m3_to_f32(((const uint8_t *)rows)[row * dp + j]);
}

// Exact distance of the definition: j ascending, one fma per coordinate,
// accumulator from +0.0; IP applies the FP8 row scale to the finished sum;
// zero is returned as +0.0.
template <int STORE, int METRIC>
__device__ double exact_dist(const void *rows, const float *scale, int64_t row, int d, int dp,
                             const float *qrow /* LDS or global, d floats */) {
    double acc = 0.0;
    if (METRIC == VRS_L2SQ) {
        double sc = (STORE == VRS_FP8E4M3) ? (double)scale[row] : 1.0;
        for (int j = 0; j < d; ++j) {
            double t = (double)qrow[j] - sc * code_at<STORE>(rows, row, dp, j);
            acc = fma(t, t, acc);
        }
    } else {
        for (int j = 0; j < d; ++j) acc = fma((double)qrow[j], code_at<STORE>(rows, row, dp, j), acc);
        double sc = (STORE == VRS_FP8E4M3) ? (double)scale[row] : 1.0;
        acc = -(sc * acc);
    }
    return acc == 0.0 ? 0.0 : acc;
}

__device__ __forceinline__ int k_of(const FinishArgs &a, int b) { return a.ks ? a.ks[b] : a.k; }
__device__ __forceinline__ int kp_of(const FinishArgs &a, int b) {
    return a.kps ? a.kps[b] : a.kprime;
}

// ------------------------------------------------------------------ merge
// Workgroup (g, b) merges lists [g*G, (g+1)*G) of query b from `src` (each K
// sorted keys) into list g of `dst`.
constexpr int MERGE_PER_THREAD = 8;

__global__ __launch_bounds__(256) void merge_kernel(const uint64_t *__restrict__ src, int n_lists,
                                                    int G, int K, int Kp, int CB,
                                                    uint64_t *__restrict__ dst, int n_out) {
    const int g = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *keys = (uint64_t *)smem;
    uint64_t *thr = keys + (Kp + CB);
    int *cnt = (int *)(thr + 1);
    TopkLds<uint64_t> tk{keys, cnt, thr, 1, K, Kp, CB};
    tk.init(tid, 256);
    const int l0 = g * G, l1 = min(n_lists, l0 + G);
    const int64_t tot = (int64_t)(l1 - l0) * K;
    const uint64_t *s = src + ((int64_t)b * n_lists + l0) * K;
    constexpr int BATCH = 256 * MERGE_PER_THREAD;
    for (int64_t p0 = 0; p0 < tot; p0 += BATCH) {
        uint64_t v[MERGE_PER_THREAD];
#pragma unroll
        for (int e = 0; e < MERGE_PER_THREAD; ++e) {
            int64_t p = p0 + e * 256 + tid;
            v[e] = p < tot ? s[p] : KEY_INF;
        }
#pragma unroll
        for (int e = 0; e < MERGE_PER_THREAD; ++e)
            if (v[e] != KEY_INF) tk.push(0, v[e]);
        __syncthreads();
        if (tk.need_flush(BATCH)) tk.flush(tid, 256);
    }
    if (tk.need_flush(CB)) tk.flush(tid, 256);
    for (int i = tid; i < K; i += 256) dst[((int64_t)b * n_out + g) * K + i] = keys[i];
}

// ----------------------------------------------------------------- rerank
template <int STORE, int METRIC>
__global__ __launch_bounds__(256) void rerank_kernel(FinishArgs a) {
    const int b = blockIdx.x, tid = threadIdx.x;
    const int kb = k_of(a, b), kpb = kp_of(a, b);
    extern __shared__ __align__(16) unsigned char smem[];
    const int Mc = next_pow2(max(kpb, 2));
    Key128 *cand = (Key128 *)smem;                 // [Mc]
    float *qrow = (float *)(cand + Mc);            // [d]
    __shared__ int n_cand_s;
    for (int j = tid; j < a.d; j += 256) qrow[j] = a.q[(int64_t)b * a.d + j];
    if (tid == 0) n_cand_s = 0;
    __syncthreads();
    const uint64_t *lst = a.merged + (int64_t)b * a.K;
    int mycnt = 0;
    for (int i = tid; i < Mc; i += 256) {
        Key128 c = KeyOps<Key128>::inf();
        if (i < kpb) {
            uint64_t key = lst[i];
            if (key != KEY_INF) {
                int64_t row = (int64_t)(uint32_t)key;
                double dv = exact_dist<STORE, METRIC>(a.rows, a.scale, row, a.d, a.dp, qrow);
                c.hi = ord64(dv);
                c.lo = (uint64_t)row;
                ++mycnt;
            }
        }
        cand[i] = c;
    }
    atomicAdd(&n_cand_s, mycnt);
    __syncthreads();
    lds_bitonic_sort<Key128>(cand, 1, Mc, tid, 256);
    const int n_cand = n_cand_s;
    bool ok = true;
    const uint64_t akey = lst[kpb];  // (k'+1)-th smallest screening key
    if (akey != KEY_INF && n_cand >= kb) {
        double av = (double)unord32((uint32_t)(akey >> 32));
        double qn = a.qnorm[b];
        double E = a.rel * fabs(av) + a.abs_ip * qn * a.max_norm +
                   a.abs_l2 * (qn + a.max_norm) * (qn + a.max_norm);
        double ek = unord64(cand[kb - 1].hi);
        ok = ek < av - E;
    }
    if (ok) {
        const int m = min(kb, n_cand);
        for (int i = tid; i < a.kmax; i += 256) {
            int64_t o = (int64_t)b * a.kmax + i;
            if (i < m) {
                a.out_idx[o] = (int64_t)cand[i].lo;
                a.out_dist[o] = (float)unord64(cand[i].hi);
            } else {
                a.out_idx[o] = -1;
                a.out_dist[o] = __int_as_float(0x7f800000);
            }
        }
        if (tid == 0) {
            if (a.n_valid) a.n_valid[b] = m;
            if (a.certified) a.certified[b] = 1;
        }
    } else if (tid == 0) {
        if (a.certified) a.certified[b] = 0;
        int slot = atomicAdd(a.fail_count, 1);
        a.fail_list[slot] = b;
    }
}

// --------------------------------------------------------------- fallback
constexpr int FB_GRID = 1024;

template <int STORE, int METRIC>
__global__ __launch_bounds__(256) void fallback_scan_kernel(FinishArgs a) {
    const int tid = threadIdx.x;
    const int nf = *a.fail_count;
    const int64_t tasks = (int64_t)nf * a.fb_chunks;
    extern __shared__ __align__(16) unsigned char smem[];
    const int Kp = next_pow2(a.kmax);
    const int M = next_pow2(Kp + 256);
    const int CB = M - Kp;
    Key128 *keys = (Key128 *)smem;
    Key128 *thr = keys + M;
    int *cnt = (int *)(thr + 1);
    float *qrow = (float *)(cnt + 4);
    for (int64_t w = blockIdx.x; w < tasks; w += gridDim.x) {
        const int f = (int)(w / a.fb_chunks), c = (int)(w - (int64_t)f * a.fb_chunks);
        const int b = a.fail_list[f];
        const int kb = k_of(a, b);
        const PredDev p = a.preds ? a.preds[b] : a.pred;
        __syncthreads();  // previous task done with LDS
        for (int j = tid; j < a.d; j += 256) qrow[j] = a.q[(int64_t)b * a.d + j];
        TopkLds<Key128> tk{keys, cnt, thr, 1, kb, Kp, CB};
        tk.init(tid, 256);
        const int64_t r0 = (int64_t)c * a.fb_rows_per_chunk;
        const int64_t r1 = min(a.n, r0 + a.fb_rows_per_chunk);
        for (int64_t t0 = r0; t0 < r1; t0 += 256) {
            int64_t row = t0 + tid;
            if (row < r1 && pred_eval(p, a.attr, a.n, row)) {
                double dv = exact_dist<STORE, METRIC>(a.rows, a.scale, row, a.d, a.dp, qrow);
                tk.push(0, Key128{ord64(dv), (uint64_t)row});
            }
            __syncthreads();
            if (tk.need_flush(256)) tk.flush(tid, 256);
        }
        if (tk.need_flush(CB)) tk.flush(tid, 256);
        uint64_t *dst = a.fb_partials + ((int64_t)f * a.fb_chunks + c) * a.kmax * 2;
        for (int i = tid; i < a.kmax; i += 256) {
            Key128 k = i < kb ? keys[i] : KeyOps<Key128>::inf();
            dst[2 * i] = k.hi;
            dst[2 * i + 1] = k.lo;
        }
    }
}

__global__ __launch_bounds__(256) void fallback_merge_kernel(FinishArgs a) {
    const int tid = threadIdx.x;
    __shared__ int nvalid_s;
    const int nf = *a.fail_count;
    extern __shared__ __align__(16) unsigned char smem[];
    const int Kp = next_pow2(a.kmax);
    const int M = next_pow2(Kp + 256);
    const int CB = M - Kp;
    Key128 *keys = (Key128 *)smem;
    Key128 *thr = keys + M;
    int *cnt = (int *)(thr + 1);
    for (int f = blockIdx.x; f < nf; f += gridDim.x) {
        const int b = a.fail_list[f];
        const int kb = k_of(a, b);
        __syncthreads();
        TopkLds<Key128> tk{keys, cnt, thr, 1, kb, Kp, CB};
        tk.init(tid, 256);
        const uint64_t *src = a.fb_partials + (int64_t)f * a.fb_chunks * a.kmax * 2;
        const int64_t tot = (int64_t)a.fb_chunks * a.kmax;
        for (int64_t p0 = 0; p0 < tot; p0 += 256) {
            int64_t p = p0 + tid;
            if (p < tot) {
                Key128 k{src[2 * p], src[2 * p + 1]};
                if (k.hi != KEY_INF || k.lo != KEY_INF) tk.push(0, k);
            }
            __syncthreads();
            if (tk.need_flush(256)) tk.flush(tid, 256);
        }
        if (tk.need_flush(CB)) tk.flush(tid, 256);
        if (tid == 0) nvalid_s = 0;
        __syncthreads();
        int mine = 0;
        for (int i = tid; i < a.kmax; i += 256) {
            int64_t o = (int64_t)b * a.kmax + i;
            Key128 k = keys[i];
            bool valid = i < kb && !(k.hi == KEY_INF && k.lo == KEY_INF);
            if (valid) {
                a.out_idx[o] = (int64_t)k.lo;
                a.out_dist[o] = (float)unord64(k.hi);
                ++mine;
            } else {
                a.out_idx[o] = -1;
                a.out_dist[o] = __int_as_float(0x7f800000);
            }
        }
        atomicAdd(&nvalid_s, mine);
        __syncthreads();
        if (tid == 0 && a.n_valid) a.n_valid[b] = nvalid_s;
    }
}

}  // namespace

hipError_t launch_prep_queries(const float *q, int32_t B, int32_t d, int32_t dp, float *qp,
                               double *qnorm, int32_t *fail_count, hipStream_t s) {
    prep_kernel<<<B, 256, 0, s>>>(q, d, dp, qp, qnorm, fail_count);
    return hipGetLastError();
}

// Per-query predicates of the batched form: fold the int64 half-open bounds
// into inclusive int32 ranges (a term on a column outside [0, n_attr), or a
// term count outside [0, 4], selects nothing), clamp k into [1, kmax] and
// derive k' with the same rule as the host.
__global__ void prep_batched_kernel(const vrs_pred *__restrict__ preds,
                                    const int32_t *__restrict__ ks, int B, int kmax, int n_attr,
                                    int kmult, int f32_rule, PredDev *__restrict__ out,
                                    int32_t *__restrict__ kc, int32_t *__restrict__ kps) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    vrs_pred p = preds[b];
    PredDev o;
    o.nterms = 0;
    bool empty = p.nterms < 0 || p.nterms > VRS_MAX_TERMS;
    for (int t = 0; t < 4; ++t) {
        o.col[t] = 0;
        o.lo[t] = 0;
        o.hi[t] = -1;
    }
    if (!empty) {
        for (int t = 0; t < p.nterms; ++t) {
            const vrs_range &r = p.term[t];
            if (r.col < 0 || r.col >= n_attr) {
                empty = true;
                break;
            }
            int64_t lo = r.lo, hi = r.hi;
            if (hi <= lo || hi <= (int64_t)INT32_MIN || lo > (int64_t)INT32_MAX) {
                empty = true;
                break;
            }
            o.col[t] = r.col;
            o.lo[t] = (int32_t)(lo < (int64_t)INT32_MIN ? (int64_t)INT32_MIN : lo);
            o.hi[t] = (int32_t)(hi - 1 > (int64_t)INT32_MAX ? (int64_t)INT32_MAX : hi - 1);
        }
        o.nterms = empty ? 0 : p.nterms;
    }
    if (empty) o.nterms = -1;
    out[b] = o;
    int k = ks[b];
    k = k < 1 ? 1 : (k > kmax ? kmax : k);
    kc[b] = k;
    int kp = kmult > 0 ? k * kmult : (f32_rule ? max(2 * k, k + 32) : 4 * k);
    kps[b] = min(max(kp, k), 1024);
}

hipError_t launch_prep_batched(const vrs_pred *preds, const int32_t *ks, int32_t B, int32_t kmax,
                               int32_t n_attr, int kmult, int f32_rule, PredDev *out,
                               int32_t *kc, int32_t *kps, hipStream_t s) {
    prep_batched_kernel<<<(B + 255) / 256, 256, 0, s>>>(preds, ks, B, kmax, n_attr, kmult,
                                                        f32_rule, out, kc, kps);
    return hipGetLastError();
}

static int merge_cb(int Kp) { return next_pow2(Kp + 256 * MERGE_PER_THREAD) - Kp; }

hipError_t launch_merge(const FinishArgs &a, hipStream_t s) {
    const int Kp = next_pow2(a.K), CB = merge_cb(Kp);
    const size_t lds = (size_t)(Kp + CB) * 8 + 8 + 16;
    const int G = 32;
    if (a.n_chunks <= G) {
        merge_kernel<<<dim3(1, a.B), 256, lds, s>>>(a.partials, a.n_chunks, G, a.K, Kp, CB,
                                                    a.merged, 1);
        return hipGetLastError();
    }
    // two levels: groups of G lists, then the group results
    const int ng = (a.n_chunks + G - 1) / G;
    uint64_t *mid = a.merge_mid;
    merge_kernel<<<dim3(ng, a.B), 256, lds, s>>>(a.partials, a.n_chunks, G, a.K, Kp, CB, mid, ng);
    merge_kernel<<<dim3(1, a.B), 256, lds, s>>>(mid, ng, ng, a.K, Kp, CB, a.merged, 1);
    return hipGetLastError();
}

template <int STORE, int METRIC>
static hipError_t rerank_t(const FinishArgs &a, hipStream_t s, int kpmax) {
    size_t lds = (size_t)next_pow2(std::max(kpmax, 2)) * sizeof(Key128) + (size_t)a.d * 4 + 16;
    rerank_kernel<STORE, METRIC><<<a.B, 256, lds, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_rerank(const FinishArgs &a, hipStream_t s) {
    const int kpmax = a.K - 1;
    if (a.metric == VRS_L2SQ) {
        switch (a.store) {
        case VRS_F32: return rerank_t<VRS_F32, VRS_L2SQ>(a, s, kpmax);
        case VRS_BF16: return rerank_t<VRS_BF16, VRS_L2SQ>(a, s, kpmax);
        default: return rerank_t<VRS_FP8E4M3, VRS_L2SQ>(a, s, kpmax);
        }
    }
    switch (a.store) {
    case VRS_F32: return rerank_t<VRS_F32, VRS_IP>(a, s, kpmax);
    case VRS_BF16: return rerank_t<VRS_BF16, VRS_IP>(a, s, kpmax);
    default: return rerank_t<VRS_FP8E4M3, VRS_IP>(a, s, kpmax);
    }
}

template <int STORE, int METRIC>
static void fallback_t(const FinishArgs &a, hipStream_t s, size_t lds_scan, size_t lds_merge,
                       int grid) {
    fallback_scan_kernel<STORE, METRIC><<<grid, 256, lds_scan, s>>>(a);
    fallback_merge_kernel<<<std::min(grid, a.B), 256, lds_merge, s>>>(a);
}

hipError_t launch_fallback(const FinishArgs &a, hipStream_t s) {
    const int Kp = next_pow2(a.kmax), M = next_pow2(Kp + 256);
    const size_t lds_merge = (size_t)M * sizeof(Key128) + sizeof(Key128) + 16;
    const size_t lds_scan = lds_merge + (size_t)a.d * 4 + 16;
    const int grid = FB_GRID;
    if (a.metric == VRS_L2SQ) {
        switch (a.store) {
        case VRS_F32: fallback_t<VRS_F32, VRS_L2SQ>(a, s, lds_scan, lds_merge, grid); break;
        case VRS_BF16: fallback_t<VRS_BF16, VRS_L2SQ>(a, s, lds_scan, lds_merge, grid); break;
        default: fallback_t<VRS_FP8E4M3, VRS_L2SQ>(a, s, lds_scan, lds_merge, grid);
        }
    } else {
        switch (a.store) {
        case VRS_F32: fallback_t<VRS_F32, VRS_IP>(a, s, lds_scan, lds_merge, grid); break;
        case VRS_BF16: fallback_t<VRS_BF16, VRS_IP>(a, s, lds_scan, lds_merge, grid); break;
        default: fallback_t<VRS_FP8E4M3, VRS_IP>(a, s, lds_scan, lds_merge, grid);
        }
    }
    return hipGetLastError();
}

}  // namespace vrs
