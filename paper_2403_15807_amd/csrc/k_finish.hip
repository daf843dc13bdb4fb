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
#include "exact64.h"

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
                                                   int32_t *__restrict__ kps_p,
                                                   uint64_t *__restrict__ heads, int n_heads) {
    const int b = blockIdx.x;                 // position
    const int src = perm ? perm[b] : b;       // query
    // the query's per-chunk best keys of the streaming screen start empty
    if (heads)
        for (int j = threadIdx.x; j < n_heads; j += 256) heads[(int64_t)b * n_heads + j] = KEY_INF;
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
// below it exist.  Only the list prefixes at or below that bound can hold
// one of the K smallest; with the chunk lists of a scan that is a few keys
// per list.  Those keys are collected and sorted once; if there are more
// than fit, they go through an LDS top-k list instead.
constexpr int MERGE_THREADS = 512;
constexpr int MERGE_HMAX = 4096;
constexpr int MERGE_RANK_MAX = 1024;  // collected keys sorted by ranking

__global__ __launch_bounds__(MERGE_THREADS) void merge_kernel(const uint64_t *__restrict__ src,
                                                              int n_lists, int G, int K, int Kp,
                                                              int CB, uint64_t *__restrict__ dst,
                                                              int n_out,
                                                              const int64_t *__restrict__ list_off,
                                                              const int32_t *__restrict__ nlists,
                                                              const uint64_t *__restrict__ heads,
                                                              const int32_t *__restrict__ limit,
                                                              const int32_t *__restrict__ fills,
                                                              int one_head) {
    constexpr int T = MERGE_THREADS;
    const int g = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    // query b's lists: n_lists of them at b * n_lists, or (batched uneven
    // form) nlists[b] of them at list_off[b]
    const int nb = nlists ? nlists[b] : n_lists;
    const int64_t first = nlists ? list_off[b] : (int64_t)b * n_lists;
    const int l0 = g * G, l1 = min(nb, l0 + G), L = (limit && b >= *limit) ? 0 : l1 - l0;
    uint64_t *out = dst + ((int64_t)b * n_out + g) * K;
    if (L <= 0) {  // no list (or a position past the limit): an empty result
        for (int i = tid; i < K; i += T) out[i] = KEY_INF;
        return;
    }
    const uint64_t *lists = src + (first + l0) * K;
    // keys list l holds (with a count array its later entries are unread)
    const int32_t *fl = fills ? fills + first + l0 : nullptr;
    const int M = Kp + CB;
    uint64_t *keys = (uint64_t *)smem;  // heads, then the collected keys
    const int region = max(M, MERGE_HMAX);
    uint64_t *thr = keys + region;
    int *cnt = (int *)(thr + 1);
    __shared__ uint32_t bound_s;
    __shared__ int ncol_s;

    // phase 1: the K-th smallest head's distance bits bound every key of
    // the result (keys with the same distance bits are all kept).  With
    // one_head, first one head per list (few lists: a few), from the
    // screening kernel's side array of first keys when it wrote one; if that
    // collects more keys than the ranking takes, and otherwise from the
    // start, the bound comes from as many heads per list as fit (lists whose
    // rows are all near the query, e.g. the few selected rows of one chunk
    // from one cluster, each put a single key below a one-head bound and
    // leave many more at or under it).
    const int m_max = max(1, min(K, MERGE_HMAX / L));
    int m = m_max;
    if (one_head) {
        m = max(1, min(K, (2 * K + L - 1) / L));
        if (L * m > MERGE_HMAX) m = max(1, MERGE_HMAX / L);
    }
    uint64_t bound = 0;
    int C = 0;
    for (int attempt = 0;; ++attempt) {
        const int H = min(L * m, MERGE_HMAX);
        // with one head per list, a side array of the lists' first keys (when
        // the screening kernel wrote one) is read instead of the lists
        const uint64_t *hd = (heads && m == 1) ? heads + first + l0 : nullptr;
        if (tid == 0) ncol_s = 0;
        if (H < K) {
            if (tid == 0) bound_s = 0xffffffffu;
        } else {
            constexpr int S = MERGE_HMAX / T;
            uint32_t v[S];
#pragma unroll
            for (int e = 0; e < S; ++e) {
                const int i = min(e * T + tid, H - 1);
                const int li = i / m, lj = i - li * m;
                const uint64_t key = hd ? hd[i] : ((!fl || lj < fl[li]) ? lists[(int64_t)li * K + lj] : KEY_INF);
                v[e] = (uint32_t)(key >> 32);
            }
            uint32_t *hist = (uint32_t *)keys;  // the collection area is free until phase 2
            const uint32_t bd = block_kth_u32<S, T>(v, H, K, hist, hist + 256);
            if (tid == 0) bound_s = bd;
        }
        __syncthreads();
        bound = ((uint64_t)bound_s << 32) | 0xffffffffu;

        // phase 2: collect every list prefix at or below the bound.  Thread tid
        // owns lists tid + j*T (j < 4, since G <= 4T); each round it reads the
        // next two entries of up to two of its lists, so most lists cost one
        // round.
        int pos[4] = {0, 0, 0, 0};
        int len[4];
        bool live[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int l = tid + j * T;
            len[j] = (fl && l < L) ? fl[l] : K;
            live[j] = l < L && len[j] > 0 && (!hd || hd[min(l, L - 1)] <= bound);
        }
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
                int n = 0;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    if (jj == j) n = len[jj];
                const int p = j >= 0 ? pos[j] : K;
                const uint64_t *lp = lists + (int64_t)(tid + max(j, 0) * T) * K;
                v[x][0] = (j >= 0 && p < n) ? lp[p] : KEY_INF;
                v[x][1] = (j >= 0 && p + 1 < n) ? lp[p + 1] : KEY_INF;
            }
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const int j = x == 0 ? sel0 : sel1;
                if (j < 0) continue;
                bool keep = true;
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const uint64_t key = v[x][e];
                    if (keep && key != KEY_INF && key <= bound) {
                        const int slot = atomicAdd(&ncol_s, 1);
                        if (slot < region) keys[slot] = key;
                    } else {
                        keep = false;
                    }
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    if (jj == j) {
                        pos[jj] += 2;
                        live[jj] = keep && pos[jj] < len[jj];
                    }
            }
            bool any = false;
#pragma unroll
            for (int j = 0; j < 4; ++j) any = any || live[j];
            if (!__syncthreads_or(any)) break;
        }
        C = ncol_s;
        if (C <= MERGE_RANK_MAX || m >= m_max || attempt > 0) break;
        m = m_max;
        __syncthreads();  // every thread has read the count before it is reset
    }
    if (C <= MERGE_RANK_MAX) {
        // keys are distinct (each row has one), so a key's rank among the
        // collected ones is its place in the result
        const int C8 = (C + 7) & ~7;
        if (tid < C8 - C) keys[C + tid] = KEY_INF;
        __syncthreads();
        const uint64_t k0 = tid < C ? keys[tid] : KEY_INF;
        const uint64_t k1 = tid + T < C ? keys[tid + T] : KEY_INF;
        int r0 = 0, r1 = 0;
        for (int j = 0; j < C8; j += 8) {
            uint64_t a8[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) a8[e] = keys[j + e];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                r0 += a8[e] < k0;
                r1 += a8[e] < k1;
            }
        }
        if (tid < C && r0 < K) out[r0] = k0;
        if (tid + T < C && r1 < K) out[r1] = k1;
        for (int i = C + tid; i < K; i += T) out[i] = KEY_INF;
        return;
    }
    if (C <= region) {
        const int CP = next_pow2(C);
        for (int i = C + tid; i < CP; i += T) keys[i] = KEY_INF;
        __syncthreads();
        lds_bitonic_sort<uint64_t>(keys, 1, CP, tid, T);
        for (int i = tid; i < K; i += T) out[i] = i < C ? keys[i] : KEY_INF;
        return;
    }

    // more candidates than fit: merge them through an LDS top-k list
    __syncthreads();
    TopkLds<uint64_t> tk{keys, cnt, thr, 1, K, Kp, CB};
    tk.init(tid, T);
    int pos[4];
    bool live[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        pos[j] = 0;
        live[j] = tid + j * T < L;
    }
    for (;;) {
        bool any = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!live[j]) continue;
            const uint64_t key = lists[(int64_t)(tid + j * T) * K + pos[j]];
            if (key != KEY_INF && key <= bound) {
                tk.push(0, key);
                ++pos[j];
                live[j] = pos[j] < K;
            } else {
                live[j] = false;
            }
            any = any || live[j];
        }
        const bool more = __syncthreads_or(any);
        if (tk.need_flush(T * 4)) tk.flush(tid, T);
        if (!more) break;
    }
    if (tk.need_flush(CB)) tk.flush(tid, T);
    for (int i = tid; i < K; i += T) out[i] = keys[i];
}

// ----------------------------------------------------------------- rerank
// One candidate per lane, so that every exact distance is the definition's
// single chain: coordinates in ascending order, one fused multiply-add each
// (the same order as exact_dist and the fallback; a different association
// can round differently, and rows with equal exact distances would then
// rank differently).  A task is 64 consecutive candidates of a query, taken
// by one wave; workgroup s of S takes tasks s, s + S, ... over its waves.
// The wave stages its 64 rows through its own LDS area one 128-byte column
// chunk at a time (coalesced 16-byte loads: eight lanes per row chunk, two
// chunks in flight in registers), then every lane runs its chain over its
// row's chunk.  Spreading one query's tasks over several workgroups (small
// batches) puts several CUs' load queues on the scattered rows.  One
// workgroup per query then ranks the candidates by exact distance, checks
// the certificate and writes the result.
constexpr int RR_THREADS = 512;
constexpr int RR_WAVES = RR_THREADS / 64;
constexpr size_t RR_STAGE_BYTES = (size_t)RR_WAVES * X64_WAVE_LDS;
// k' <= 1024 = 2 RR_THREADS: the candidate sort holds at most two keys per thread
static_assert(2 * RR_THREADS >= 1024, "rerank sort width");

__device__ __forceinline__ bool k128_less(uint64_t ah, uint32_t al, uint64_t bh, uint32_t bl) {
    return ah < bh || (ah == bh && al < bl);
}

// Ascending bitonic sort of the RR_THREADS*E keys (hi, lo) held E per
// thread, element i in thread i % RR_THREADS, slot i / RR_THREADS.  Strides
// below 64 exchange through lane shuffles, strides of a whole wave or more
// but below RR_THREADS through LDS (xh, xl), larger ones inside a thread.
template <int E>
__device__ void rr_bitonic(uint64_t (&h)[E], uint32_t (&l)[E], uint64_t *xh, uint32_t *xl) {
    constexpr int T = RR_THREADS;
    const int tid = threadIdx.x;
    for (int k = 2; k <= T * E; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= T) {
                const int je = j / T;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int p = e ^ je;
                    if (p > e) {
                        const bool up = ((e * T + tid) & k) == 0;
                        if (k128_less(h[p], l[p], h[e], l[e]) == up) {
                            const uint64_t th = h[e];
                            const uint32_t tl = l[e];
                            h[e] = h[p]; l[e] = l[p];
                            h[p] = th; l[p] = tl;
                        }
                    }
                }
                continue;
            }
            uint64_t ph[E];
            uint32_t pl[E];
            if (j >= 64) {
                __syncthreads();
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    xh[e * T + tid] = h[e];
                    xl[e * T + tid] = l[e];
                }
                __syncthreads();
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    ph[e] = xh[e * T + (tid ^ j)];
                    pl[e] = xl[e * T + (tid ^ j)];
                }
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    ph[e] = shfl_xor_u64(h[e], j);
                    pl[e] = (uint32_t)__shfl_xor((int)l[e], j);
                }
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int i = e * T + tid;
                const bool take_min = ((i & j) == 0) == ((i & k) == 0);
                const bool pless = k128_less(ph[e], pl[e], h[e], l[e]);
                if (pless == take_min) {
                    h[e] = ph[e];
                    l[e] = pl[e];
                }
            }
        }
    }
}

// Rank the first n candidates of cand by exact key and keep the first kb
// (in order) in srt.
template <int E>
__device__ void rr_sort(const Key128 *cand, int n, int kb, Key128 *srt, uint64_t *xh, uint32_t *xl) {
    constexpr int T = RR_THREADS;
    const int tid = threadIdx.x;
    uint64_t h[E];
    uint32_t l[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = e * T + tid;
        h[e] = i < n ? cand[i].hi : ~0ull;
        l[e] = i < n ? (uint32_t)cand[i].lo : ~0u;
    }
    rr_bitonic<E>(h, l, xh, xl);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = e * T + tid;
        if (i < kb && i < n) srt[i] = Key128{h[e], (uint64_t)l[e]};
    }
}

// LDS of the rerank: the FP64 query [dp], then one area used first for the
// waves' row staging and afterwards (every wave done) for the sort buffers,
// the candidates and the ranked result.
__host__ __device__ inline size_t rr_sort_bytes(int K) {
    return (size_t)2 * RR_THREADS * 12 + (size_t)2 * ((K + 7) & ~7) * sizeof(Key128);
}
__host__ __device__ inline size_t rr_lds_bytes(int dp, int K) {
    const size_t sb = rr_sort_bytes(K);
    return (size_t)dp * 8 + (sb > RR_STAGE_BYTES ? sb : RR_STAGE_BYTES);
}

// PHASE 0: one workgroup per query does both parts; PHASE 1: the exact
// distances, split over the workgroups of a query; PHASE 2 (a later launch,
// one workgroup per query): the ranking and the certificate.  The kernel
// boundary between phases 1 and 2 orders the distances before their use, so
// no device-scope fence is needed (on this GPU such a fence writes back the
// XCD's L2).
template <int STORE, int METRIC, int PHASE>
__global__ __launch_bounds__(RR_THREADS) void rerank_kernel(FinishArgs a) {
    constexpr int T = RR_THREADS;
    const int s = blockIdx.x, b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kpb = kp_of(a, b);
    // the k' survivors, and with error diagnostics also the (k'+1)-th key
    const int nc = kpb + (a.err_ratio ? 1 : 0);
    const int ntask = (nc + 63) / 64;
    const int S = gridDim.x;
    const int ns = min(S, ntask);  // workgroups with work for query b
    if (s >= ns) return;
    const int ob = a.perm ? a.perm[b] : b;  // the query at position b
    extern __shared__ __align__(16) unsigned char smem[];
    double *qd = (double *)smem;                                  // [dp]
    unsigned char *area = smem + (size_t)a.dp * 8;
    x64_u32x4 *stage = (x64_u32x4 *)(area + (size_t)wave * X64_WAVE_LDS);  // this wave's rows
    uint64_t *xh = (uint64_t *)area;                              // [2T]   (final phase)
    uint32_t *xl = (uint32_t *)(xh + 2 * T);                      // [2T]
    Key128 *cand = (Key128 *)(xl + 2 * T);                        // [round8(K)]
    Key128 *srt = cand + ((a.K + 7) & ~7);                        // [k] in exact order
    __shared__ int n_cand_s, ratio_s;
    if (tid == 0) {
        n_cand_s = 0;
        ratio_s = 0;
    }
    const uint64_t *lst = a.merged + (int64_t)b * a.K;
    double *dist = a.rr_dist + (int64_t)b * a.K;
    if (PHASE != 2) {
        for (int j = tid; j < a.dp; j += T) qd[j] = j < a.d ? (double)a.q[(int64_t)ob * a.d + j] : 0.0;
        __syncthreads();
        for (int t = s + S * wave; t < ntask; t += S * RR_WAVES) {
            const int ci = t * 64 + lane;
            const uint64_t key = ci < nc ? lst[ci] : KEY_INF;
            const bool has = key != KEY_INF;
            // a lane without a candidate stages row 0 and drops its value
            const int row = has ? (int)(uint32_t)key : 0;
            const double dv = exact64_wave<STORE, METRIC>(a.rows, a.scale, row, has, qd, a.dp, stage);
            if (ci < nc && has) dist[ci] = dv;
        }
    }
    if (PHASE == 1) return;
    __syncthreads();  // every wave's distances written, the staging area free

    // the screening keys are sorted with empty slots last, so the candidates
    // are the first n_cand of them
    const int kb = k_of(a, b);
    const double qn = a.qnorm[b];
    const double eabs = a.abs_ip * qn * a.max_norm + a.abs_l2 * (qn + a.max_norm) * (qn + a.max_norm);
    int valid = 0;
    float ratio = 0.0f;  // largest |screening - exact| / bound over the reranked keys
    for (int ci = tid; ci < nc; ci += T) {
        const uint64_t key = lst[ci];
        if (key == KEY_INF) continue;
        const double dv = dist[ci];
        if (ci < kpb) {
            cand[ci] = Key128{ord64(dv == 0.0 ? 0.0 : dv), (uint64_t)(uint32_t)key};
            ++valid;
        }
        if (a.err_ratio) {
            const double sv = (double)unord32((uint32_t)(key >> 32));
            const double E = a.rel * fabs(dv) + eabs;
            const double err = fabs(sv - dv);
            const float r = E > 0.0 ? (float)(err / E) : (err > 0.0 ? __int_as_float(0x7f800000) : 0.0f);
            ratio = fmaxf(ratio, r);
        }
    }
    if (valid) atomicAdd(&n_cand_s, valid);
    // (non-negative floats order like their bit patterns)
    if (a.err_ratio && ratio > 0.0f) atomicMax(&ratio_s, __float_as_int(ratio));
    __syncthreads();
    if (a.err_ratio && tid == 0) a.err_ratio[ob] = __int_as_float(ratio_s);
    const int n_cand = n_cand_s;
    if (n_cand <= T)
        rr_sort<1>(cand, n_cand, kb, srt, xh, xl);
    else
        rr_sort<2>(cand, n_cand, kb, srt, xh, xl);
    __syncthreads();
    bool ok = true;
    const uint64_t akey = lst[kpb];  // (k'+1)-th smallest screening key
    if (akey != KEY_INF && n_cand >= kb) {
        const double av = (double)unord32((uint32_t)(akey >> 32));
        const double E = a.rel * fabs(av) + eabs;
        ok = unord64(srt[kb - 1].hi) < av - E;
    }
    if (ok) {
        const int m = min(kb, n_cand);
        for (int i = tid; i < a.kmax; i += T) {
            const int64_t o = (int64_t)ob * a.kmax + i;
            if (i < m) {
                a.out_idx[o] = (int64_t)srt[i].lo;
                a.out_dist[o] = (float)unord64(srt[i].hi);
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
        const int slot = atomicAdd(a.fail_count, 1);
        a.fail_list[slot] = b;
    }
}

// --------------------------------------------------------------- fallback
constexpr int FB_GRID = 1024;

template <int STORE, int METRIC>
__global__ __launch_bounds__(256) void fallback_scan_kernel(FinishArgs a) {
    const int tid = threadIdx.x, wave = tid >> 6;
    const int nf = *a.fail_count;
    const int64_t tasks = (int64_t)nf * a.fb_chunks;
    extern __shared__ __align__(16) unsigned char smem[];
    const int Kp = next_pow2(a.kmax);
    const int M = next_pow2(Kp + 256);
    const int CB = M - Kp;
    // the waves' row staging, the FP64 query, then the top-k list
    x64_u32x4 *stage = (x64_u32x4 *)(smem + (size_t)wave * X64_WAVE_LDS);
    double *qd = (double *)(smem + 4 * X64_WAVE_LDS);
    Key128 *keys = (Key128 *)(qd + a.dp);
    Key128 *thr = keys + M;
    int *cnt = (int *)(thr + 1);
    for (int64_t w = blockIdx.x; w < tasks; w += gridDim.x) {
        const int f = (int)(w / a.fb_chunks), c = (int)(w - (int64_t)f * a.fb_chunks);
        const int b = a.fail_list[f];
        const int ob = a.perm ? a.perm[b] : b;
        const int kb = k_of(a, b);
        const PredDev p = a.preds ? a.preds[b] : a.pred;
        __syncthreads();  // previous task done with LDS
        for (int j = tid; j < a.dp; j += 256) qd[j] = j < a.d ? (double)a.q[(int64_t)ob * a.d + j] : 0.0;
        TopkLds<Key128> tk{keys, cnt, thr, 1, kb, Kp, CB};
        tk.init(tid, 256);
        const int64_t r0 = (int64_t)c * a.fb_rows_per_chunk;
        const int64_t r1 = min(a.n, r0 + a.fb_rows_per_chunk);
        // wave w takes rows t0 + 64 w .. + 63, one per lane, staged together
        for (int64_t t0 = r0; t0 < r1; t0 += 256) {
            const int64_t row = t0 + tid;
            const bool has = row < r1 && pred_eval(p, a.attr, a.an, row);
            if (__ballot(has) != 0) {  // (wave-uniform)
                const double dv =
                    exact64_wave<STORE, METRIC>(a.rows, a.scale, has ? (int)row : 0, has, qd, a.dp, stage);
                if (has) tk.push(0, Key128{ord64(dv), (uint64_t)row});
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

__global__ void set_bound_kernel(const uint64_t *__restrict__ merged, int K, int B,
                                 const int32_t *__restrict__ kps, uint64_t *__restrict__ gthr,
                                 int32_t *__restrict__ zero8) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (zero8 && b < 8) zero8[b] = 0;
    if (b >= B) return;
    const int kb = kps ? min(K, kps[b] + 1) : K;
    const uint64_t v = merged[(int64_t)b * K + kb - 1];
    // the next pass rebuilds its lists from empty and admits keys strictly
    // below the bound, so the bound is the key after v (v itself must come
    // back); bounds the first pass's lists published are all at or above v
    gthr[b] = v == KEY_INF ? KEY_INF : v + 1;
}

}  // namespace

hipError_t launch_prep_queries(const float *q, int32_t B, int32_t d, int32_t dp, float *qp,
                               double *qnorm, float *qn2, uint16_t *qhl, uint64_t *gthr,
                               int32_t *fail_count, uint64_t *heads, int32_t n_heads, hipStream_t s) {
    prep_kernel<<<B, 256, 0, s>>>(q, d, dp, qp, qnorm, qn2, qhl, gthr, fail_count, nullptr, nullptr,
                                  nullptr, nullptr, nullptr, nullptr, nullptr, heads, n_heads);
    return hipGetLastError();
}

hipError_t launch_prep_permuted(const float *q, const int32_t *perm, int32_t B, int32_t d,
                                int32_t dp, const PredDev *pred_o, const int32_t *kc_o,
                                const int32_t *kps_o, float *qp, double *qnorm, float *qn2,
                                uint16_t *qhl, uint64_t *gthr, int32_t *fail_count,
                                PredDev *pred_p, int32_t *kc_p, int32_t *kps_p, hipStream_t s) {
    prep_kernel<<<B, 256, 0, s>>>(q, d, dp, qp, qnorm, qn2, qhl, gthr, fail_count, perm, pred_o, kc_o,
                                  kps_o, pred_p, kc_p, kps_p, nullptr, 0);
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

hipError_t launch_set_bound(const FinishArgs &a, uint64_t *gthr, int32_t *zero8, hipStream_t s) {
    set_bound_kernel<<<(std::max(a.B, 8) + 255) / 256, 256, 0, s>>>(a.merged, a.K, a.B, a.kps, gthr, zero8);
    return hipGetLastError();
}

hipError_t launch_merge(const FinishArgs &a, hipStream_t s) {
    const int Kp = next_pow2(a.K), CB = merge_cb(Kp);
    const size_t lds = (size_t)std::max(Kp + CB, MERGE_HMAX) * 8 + 8 + 16;
    const int G = 2048;
    if (a.n_chunks <= G) {
        merge_kernel<<<dim3(1, a.B), MERGE_THREADS, lds, s>>>(a.partials, a.n_chunks, G, a.K, Kp,
                                                             CB, a.merged, 1, a.list_off, a.nlists,
                                                             a.heads, a.merge_limit, a.fills, a.merge_one_head);
        return hipGetLastError();
    }
    // two levels: groups of G lists, then the group results
    const int ng = (a.n_chunks + G - 1) / G;
    uint64_t *mid = a.merge_mid;
    merge_kernel<<<dim3(ng, a.B), MERGE_THREADS, lds, s>>>(a.partials, a.n_chunks, G, a.K, Kp, CB,
                                                          mid, ng, a.list_off, a.nlists, a.heads,
                                                          a.merge_limit, a.fills, a.merge_one_head);
    merge_kernel<<<dim3(1, a.B), MERGE_THREADS, lds, s>>>(mid, ng, ng, a.K, Kp, CB, a.merged, 1,
                                                         nullptr, nullptr, nullptr,
                                                         a.merge_limit, nullptr, a.merge_one_head);
    return hipGetLastError();
}

template <int STORE, int METRIC>
static hipError_t rerank_t(const FinishArgs &a, hipStream_t s, int kpmax) {
    const size_t lds = rr_lds_bytes(a.dp, a.K);
    ensure_dyn_lds((const void *)rerank_kernel<STORE, METRIC, 0>, lds);
    ensure_dyn_lds((const void *)rerank_kernel<STORE, METRIC, 1>, lds);
    ensure_dyn_lds((const void *)rerank_kernel<STORE, METRIC, 2>, lds);
    // Several workgroups per query for the distances when the batch alone
    // cannot fill the GPU (their rows come from many CUs at once), then one
    // per query for the ranking; one per query for both from 256 queries on.
    const int tasks = (kpmax + (a.err_ratio ? 1 : 0) + 63) / 64;
    const int S = std::max(1, std::min(tasks, (256 + a.B - 1) / a.B));
    if (S == 1) {
        rerank_kernel<STORE, METRIC, 0><<<dim3(1, a.B), RR_THREADS, lds, s>>>(a);
    } else {
        rerank_kernel<STORE, METRIC, 1><<<dim3(S, a.B), RR_THREADS, lds, s>>>(a);
        rerank_kernel<STORE, METRIC, 2><<<dim3(1, a.B), RR_THREADS, lds, s>>>(a);
    }
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
    ensure_dyn_lds((const void *)fallback_scan_kernel<STORE, METRIC>, lds_scan);
    fallback_scan_kernel<STORE, METRIC><<<grid, 256, lds_scan, s>>>(a);
    fallback_merge_kernel<<<std::min(grid, a.B), 256, lds_merge, s>>>(a);
}

hipError_t launch_fallback(const FinishArgs &a, hipStream_t s) {
    const int Kp = next_pow2(a.kmax), M = next_pow2(Kp + 256);
    const size_t lds_merge = (size_t)M * sizeof(Key128) + sizeof(Key128) + 16;
    const size_t lds_scan = 4 * X64_WAVE_LDS + (size_t)a.dp * 8 + lds_merge;
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
