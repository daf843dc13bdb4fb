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
                                                   float *__restrict__ qn2,
                                                   uint16_t *__restrict__ qhl,
                                                   uint64_t *__restrict__ gthr,
                                                   int32_t *__restrict__ fail_count,
                                                   const int32_t *__restrict__ perm,
                                                   const PredDev *__restrict__ pred_o,
                                                   const int32_t *__restrict__ kc_o,
                                                   const int32_t *__restrict__ kps_o,
                                                   PredDev *__restrict__ pred_p,
                                                   int32_t *__restrict__ kc_p,
                                                   int32_t *__restrict__ kps_p) {
    const int b = blockIdx.x;                 // position
    const int src = perm ? perm[b] : b;       // query
    if (threadIdx.x == 0) {
        gthr[b] = KEY_INF;
        if (perm) {
            pred_p[b] = pred_o[src];
            kc_p[b] = kc_o[src];
            kps_p[b] = kps_o[src];
        }
    }
    if (b == 0 && threadIdx.x == 0) *fail_count = 0;
    __shared__ double red[256];
    double acc = 0.0;
    for (int j = threadIdx.x; j < dp; j += 256) {
        float v = j < d ? q[(int64_t)src * d + j] : 0.0f;
        qp[(int64_t)b * dp + j] = v;
        acc += (double)v * (double)v;
        if (qhl) {  // bfloat16 hi/lo split (round to nearest-even both times)
            const uint32_t u = __float_as_uint(v);
            const uint32_t hi = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
            const float rest = v - __uint_as_float(hi << 16);  // exact
            const uint32_t r = __float_as_uint(rest);
            const uint32_t lo = (r + 0x7fffu + ((r >> 16) & 1u)) >> 16;
            // in the A-operand order of v_mfma_f32_16x16x32_bf16: 16-byte unit
            // ((b/16 * dp/32 + j/32) * 2 + part) * 64 + lane, lane = b%16 +
            // 16 ((j%32)/8), element j%8
            const int64_t unit = ((int64_t)(b >> 4) * (dp >> 5) + (j >> 5)) * 2;
            const int ln = (b & 15) + 16 * ((j & 31) >> 3);
            qhl[(unit * 64 + ln) * 8 + (j & 7)] = (uint16_t)hi;
            qhl[((unit + 1) * 64 + ln) * 8 + (j & 7)] = (uint16_t)lo;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        qnorm[b] = sqrt(red[0]) * (1.0 + 0x1p-40);
        qn2[b] = (float)red[0];
    }
}

// Exact distance of the definition: coordinates in ascending order, one
// fused multiply-add each, accumulator from +0.0; IP applies the FP8 row
// scale to the finished sum; zero is returned as +0.0.  The row is read in
// 16-byte blocks up to the padded width dp; `qrow` holds the query padded
// with zeros to dp, and a padded coordinate adds an exact zero (+0 + +0 or
// acc + 0), so the value equals the sum over the first d coordinates.
template <int STORE>
__device__ __forceinline__ void decode16(const uint4 &w, float *x);
template <>
__device__ __forceinline__ void decode16<VRS_F32>(const uint4 &w, float *x) {
    x[0] = __uint_as_float(w.x);
    x[1] = __uint_as_float(w.y);
    x[2] = __uint_as_float(w.z);
    x[3] = __uint_as_float(w.w);
}
template <>
__device__ __forceinline__ void decode16<VRS_BF16>(const uint4 &w, float *x) {
    const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        x[2 * i] = __uint_as_float(v[i] << 16);
        x[2 * i + 1] = __uint_as_float(v[i] & 0xffff0000u);
    }
}
template <>
__device__ __forceinline__ void decode16<VRS_FP8E4M3>(const uint4 &w, float *x) {
    const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) x[4 * i + j] = e4m3_to_f32((v[i] >> (8 * j)) & 0xffu);
}

template <int STORE, int METRIC>
__device__ double exact_dist(const void *rows, const float *scale, int64_t row, int dp,
                             const float *qrow /* dp floats, zero padded */) {
    constexpr int V = STORE == VRS_F32 ? 4 : (STORE == VRS_BF16 ? 8 : 16);
    constexpr int EB = 16 / V;
    const uint4 *p = (const uint4 *)((const char *)rows + row * (int64_t)dp * EB);
    const int nb = dp / V;
    const double sc = (STORE == VRS_FP8E4M3) ? (double)scale[row] : 1.0;
    double acc = 0.0;
    for (int c = 0; c < nb; c += 2) {
        uint4 w0 = p[c];
        uint4 w1 = (c + 1 < nb) ? p[c + 1] : make_uint4(0, 0, 0, 0);
        float x[2 * V];
        decode16<STORE>(w0, x);
        decode16<STORE>(w1, x + V);
        const int jn = min(2 * V, dp - c * V);
        for (int j = 0; j < jn; ++j) {
            const double qj = (double)qrow[c * V + j];
            if (METRIC == VRS_L2SQ) {
                double t = qj - sc * (double)x[j];
                acc = fma(t, t, acc);
            } else {
                acc = fma(qj, (double)x[j], acc);
            }
        }
    }
    if (METRIC == VRS_IP) acc = -(sc * acc);
    return acc == 0.0 ? 0.0 : acc;
}

__device__ __forceinline__ int k_of(const FinishArgs &a, int b) { return a.ks ? a.ks[b] : a.k; }
__device__ __forceinline__ int kp_of(const FinishArgs &a, int b) {
    return a.kps ? a.kps[b] : a.kprime;
}

// ------------------------------------------------------------------ merge
// Workgroup (g, b) merges lists [g*G, (g+1)*G) of query b from `src` (each K
// sorted keys, KEY_INF padded) into list g of `dst`.
//
// Every list is sorted, so the K-th smallest of the lists' first m entries
// ("heads") is an upper bound on the K-th smallest key overall: K keys at or
// below it exist.  Only the list prefixes at or below that bound are read
// and merged; with the chunk lists of a scan that is a few keys per list.
constexpr int MERGE_THREADS = 512;
constexpr int MERGE_HMAX = 4096;

__global__ __launch_bounds__(MERGE_THREADS) void merge_kernel(const uint64_t *__restrict__ src,
                                                              int n_lists, int G, int K, int Kp,
                                                              int CB, uint64_t *__restrict__ dst,
                                                              int n_out,
                                                              const int64_t *__restrict__ list_off,
                                                              const int32_t *__restrict__ nlists) {
    constexpr int T = MERGE_THREADS;
    const int g = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    // query b's lists: n_lists of them at b * n_lists, or (batched uneven
    // form) nlists[b] of them at list_off[b]
    const int nb = nlists ? nlists[b] : n_lists;
    const int64_t first = nlists ? list_off[b] : (int64_t)b * n_lists;
    const int l0 = g * G, l1 = min(nb, l0 + G), L = l1 - l0;
    if (L <= 0) {  // no list: an empty result
        for (int i = tid; i < K; i += T) dst[((int64_t)b * n_out + g) * K + i] = KEY_INF;
        return;
    }
    const uint64_t *lists = src + (first + l0) * K;
    const int M = Kp + CB;
    uint64_t *keys = (uint64_t *)smem;                         // heads, then the top-k list
    const int region = max(M, MERGE_HMAX);
    uint64_t *thr = keys + region;
    int *cnt = (int *)(thr + 1);
    __shared__ uint64_t bound_s;

    // phase 1: bound from the heads
    int m = max(1, min(K, (2 * K + L - 1) / L));
    if (L * m > MERGE_HMAX) m = max(1, MERGE_HMAX / L);
    const int H = min(L * m, MERGE_HMAX);
    const int HP = next_pow2(max(H, 2));
    for (int i = tid; i < HP; i += T) keys[i] = i < H ? lists[(int64_t)(i / m) * K + (i % m)] : KEY_INF;
    __syncthreads();
    lds_bitonic_sort<uint64_t>(keys, 1, HP, tid, T);
    if (tid == 0) bound_s = (H >= K) ? keys[K - 1] : KEY_INF;
    __syncthreads();
    const uint64_t bound = bound_s;

    // phase 2: merge every list prefix at or below the bound.  Thread tid owns
    // lists tid + j*T (j < 4, since G <= 4T); each round it reads the next two
    // entries of up to two of its lists, so most lists cost one round.
    TopkLds<uint64_t> tk{keys, cnt, thr, 1, K, Kp, CB};
    tk.init(tid, T);
    int pos[4] = {0, 0, 0, 0};
    bool live[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) live[j] = tid + j * T < L;
    for (;;) {
        int sel0 = -1, sel1 = -1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (live[j] && sel0 < 0) sel0 = j;
            else if (live[j] && sel1 < 0) sel1 = j;
        }
        uint64_t v[2][2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const int j = x == 0 ? sel0 : sel1;
            const int p = j >= 0 ? pos[j] : K;
            const uint64_t *lp = lists + (int64_t)(tid + max(j, 0) * T) * K;
            v[x][0] = (j >= 0 && p < K) ? lp[p] : KEY_INF;
            v[x][1] = (j >= 0 && p + 1 < K) ? lp[p + 1] : KEY_INF;
        }
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const int j = x == 0 ? sel0 : sel1;
            if (j < 0) continue;
            bool keep = true;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const uint64_t key = v[x][e];
                if (keep && key != KEY_INF && key <= bound)
                    tk.push(0, key);
                else
                    keep = false;
            }
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
                if (jj == j) {
                    pos[jj] += 2;
                    live[jj] = keep && pos[jj] < K;
                }
        }
        bool any = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) any = any || live[j];
        const bool more = __syncthreads_or(any);
        if (tk.need_flush(T * 4)) tk.flush(tid, T);
        if (!more) break;
    }
    if (tk.need_flush(CB)) tk.flush(tid, T);
    for (int i = tid; i < K; i += T) dst[((int64_t)b * n_out + g) * K + i] = keys[i];
}

// ----------------------------------------------------------------- rerank
// One workgroup per query.  Each lane owns one candidate and runs the exact
// FP64 formula over it in coordinate order; the rows themselves are loaded
// cooperatively (8 lanes per 128-byte block of a row, 8 loads in flight per
// lane) into LDS, one 128-byte column chunk of 64 rows per wave at a time.
constexpr int RR_CHUNK = 8;  // 16-byte blocks per row per chunk

template <int STORE, int METRIC>
__global__ __launch_bounds__(256) void rerank_kernel(FinishArgs a) {
    constexpr int V = STORE == VRS_F32 ? 4 : (STORE == VRS_BF16 ? 8 : 16);
    constexpr int EB = 16 / V;
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ob = a.perm ? a.perm[b] : b;  // the query at position b
    const int kb = k_of(a, b), kpb = kp_of(a, b);
    extern __shared__ __align__(16) unsigned char smem[];
    const int Mc = next_pow2(max(kpb, 2));
    Key128 *cand = (Key128 *)smem;                           // [Mc]
    uint4 *stage = (uint4 *)(cand + Mc);                     // [4][64][RR_CHUNK + 1]
    float *qrow = (float *)(stage + 4 * 64 * (RR_CHUNK + 1)); // [dp], zero padded
    __shared__ int n_cand_s;
    for (int j = tid; j < a.dp; j += 256) qrow[j] = j < a.d ? a.q[(int64_t)ob * a.d + j] : 0.0f;
    if (tid == 0) n_cand_s = 0;
    __syncthreads();
    const uint64_t *lst = a.merged + (int64_t)b * a.K;
    const int nb16 = a.dp / V;                               // 16-byte blocks per row
    const int64_t row_bytes = (int64_t)a.dp * EB;
    uint4 *my_stage = stage + (wave * 64) * (RR_CHUNK + 1);
    int mycnt = 0;
    for (int g0 = 0; g0 < Mc; g0 += 256) {
        const int ci = g0 + tid;
        int64_t myrow = -1;
        if (ci < kpb) {
            uint64_t key = lst[ci];
            if (key != KEY_INF) myrow = (int64_t)(uint32_t)key;
        }
        double acc = 0.0;
        const double sc = (STORE == VRS_FP8E4M3 && myrow >= 0) ? (double)a.scale[myrow] : 1.0;
        for (int c0 = 0; c0 < nb16; c0 += RR_CHUNK) {
            uint4 w[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int src = (lane >> 3) + 8 * i;
                const int64_t rr = __shfl(myrow, src);
                w[i] = rr >= 0 ? *(const uint4 *)((const char *)a.rows + rr * row_bytes +
                                                  (int64_t)(c0 + (lane & 7)) * 16)
                               : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) my_stage[((lane >> 3) + 8 * i) * (RR_CHUNK + 1) + (lane & 7)] = w[i];
            __syncthreads();
            if (myrow >= 0) {
                for (int blk = 0; blk < RR_CHUNK; ++blk) {
                    float x[V];
                    decode16<STORE>(my_stage[lane * (RR_CHUNK + 1) + blk], x);
                    const float *qj = qrow + (c0 + blk) * V;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        if (METRIC == VRS_L2SQ) {
                            double t = (double)qj[v] - sc * (double)x[v];
                            acc = fma(t, t, acc);
                        } else {
                            acc = fma((double)qj[v], (double)x[v], acc);
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (ci < Mc) {
            Key128 c = KeyOps<Key128>::inf();
            if (myrow >= 0) {
                if (METRIC == VRS_IP) acc = -(sc * acc);
                c.hi = ord64(acc == 0.0 ? 0.0 : acc);
                c.lo = (uint64_t)myrow;
                ++mycnt;
            }
            cand[ci] = c;
        }
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
            int64_t o = (int64_t)ob * a.kmax + i;
            if (i < m) {
                a.out_idx[o] = (int64_t)cand[i].lo;
                a.out_dist[o] = (float)unord64(cand[i].hi);
            } else {
                a.out_idx[o] = -1;
                a.out_dist[o] = __int_as_float(0x7f800000);
            }
        }
        if (tid == 0) {
            if (a.n_valid) a.n_valid[ob] = m;
            if (a.certified) a.certified[ob] = 1;
        }
    } else if (tid == 0) {
        if (a.certified) a.certified[ob] = 0;
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
        const int ob = a.perm ? a.perm[b] : b;
        const int kb = k_of(a, b);
        const PredDev p = a.preds ? a.preds[b] : a.pred;
        __syncthreads();  // previous task done with LDS
        for (int j = tid; j < a.dp; j += 256) qrow[j] = j < a.d ? a.q[(int64_t)ob * a.d + j] : 0.0f;
        TopkLds<Key128> tk{keys, cnt, thr, 1, kb, Kp, CB};
        tk.init(tid, 256);
        const int64_t r0 = (int64_t)c * a.fb_rows_per_chunk;
        const int64_t r1 = min(a.n, r0 + a.fb_rows_per_chunk);
        for (int64_t t0 = r0; t0 < r1; t0 += 256) {
            int64_t row = t0 + tid;
            if (row < r1 && pred_eval(p, a.attr, a.an, row)) {
                double dv = exact_dist<STORE, METRIC>(a.rows, a.scale, row, a.dp, qrow);
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
        const int ob = a.perm ? a.perm[b] : b;
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
            int64_t o = (int64_t)ob * a.kmax + i;
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
        if (tid == 0 && a.n_valid) a.n_valid[ob] = nvalid_s;
    }
}

}  // namespace

hipError_t launch_prep_queries(const float *q, int32_t B, int32_t d, int32_t dp, float *qp,
                               double *qnorm, float *qn2, uint16_t *qhl, uint64_t *gthr,
                               int32_t *fail_count, hipStream_t s) {
    prep_kernel<<<B, 256, 0, s>>>(q, d, dp, qp, qnorm, qn2, qhl, gthr, fail_count, nullptr, nullptr,
                                  nullptr, nullptr, nullptr, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_prep_permuted(const float *q, const int32_t *perm, int32_t B, int32_t d,
                                int32_t dp, const PredDev *pred_o, const int32_t *kc_o,
                                const int32_t *kps_o, float *qp, double *qnorm, float *qn2,
                                uint16_t *qhl, uint64_t *gthr, int32_t *fail_count,
                                PredDev *pred_p, int32_t *kc_p, int32_t *kps_p, hipStream_t s) {
    prep_kernel<<<B, 256, 0, s>>>(q, d, dp, qp, qnorm, qn2, qhl, gthr, fail_count, perm, pred_o, kc_o,
                                  kps_o, pred_p, kc_p, kps_p);
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
    out[b] = fold_pred_dev(preds[b], n_attr);
    int k = ks[b];
    k = k < 1 ? 1 : (k > kmax ? kmax : k);
    kc[b] = k;
    kps[b] = kprime_dev(k, kmult, f32_rule);
}

hipError_t launch_prep_batched(const vrs_pred *preds, const int32_t *ks, int32_t B, int32_t kmax,
                               int32_t n_attr, int kmult, int f32_rule, PredDev *out,
                               int32_t *kc, int32_t *kps, hipStream_t s) {
    prep_batched_kernel<<<(B + 255) / 256, 256, 0, s>>>(preds, ks, B, kmax, n_attr, kmult,
                                                        f32_rule, out, kc, kps);
    return hipGetLastError();
}

static int merge_cb(int Kp) { return next_pow2(Kp + MERGE_THREADS * 4) - Kp; }

hipError_t launch_merge(const FinishArgs &a, hipStream_t s) {
    const int Kp = next_pow2(a.K), CB = merge_cb(Kp);
    const size_t lds = (size_t)std::max(Kp + CB, MERGE_HMAX) * 8 + 8 + 16;
    const int G = 2048;
    if (a.n_chunks <= G) {
        merge_kernel<<<dim3(1, a.B), MERGE_THREADS, lds, s>>>(a.partials, a.n_chunks, G, a.K, Kp,
                                                             CB, a.merged, 1, a.list_off, a.nlists);
        return hipGetLastError();
    }
    // two levels: groups of G lists, then the group results
    const int ng = (a.n_chunks + G - 1) / G;
    uint64_t *mid = a.merge_mid;
    merge_kernel<<<dim3(ng, a.B), MERGE_THREADS, lds, s>>>(a.partials, a.n_chunks, G, a.K, Kp, CB,
                                                          mid, ng, a.list_off, a.nlists);
    merge_kernel<<<dim3(1, a.B), MERGE_THREADS, lds, s>>>(mid, ng, ng, a.K, Kp, CB, a.merged, 1,
                                                         nullptr, nullptr);
    return hipGetLastError();
}

template <int STORE, int METRIC>
static hipError_t rerank_t(const FinishArgs &a, hipStream_t s, int kpmax) {
    size_t lds = (size_t)next_pow2(std::max(kpmax, 2)) * sizeof(Key128) +
                 (size_t)4 * 64 * (RR_CHUNK + 1) * 16 + (size_t)a.dp * 4 + 16;
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
    const size_t lds_scan = lds_merge + (size_t)a.dp * 4 + 16;
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
