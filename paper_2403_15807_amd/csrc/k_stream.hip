// k_stream.hip -- VALU screening kernel for small query batches (the 1:N
// strategy of Section 3.1: one query against a batch of data vectors, with
// the relational predicate either checked on the fly per row (mask) or
// pushed down into a selection vector first (gather), eq. 3).
//
// A workgroup owns QT queries and one chunk of rows.  Rows stream from HBM
// with 16-byte loads, 8 lanes per row, so every wave instruction reads eight
// full 128-byte segments.  Each lane accumulates the FP32 distance of its
// slice for every query of the tile; three xor-shuffles finish the row sums.
// Candidates below the query's current threshold go to an LDS append buffer
// that is merged into the query's sorted list when it fills (TopkLds).  The
// chunk's K smallest keys are written out sorted for the cross-chunk merge.
#include "internal.h"
#include "topk_sized.h"

namespace vrs {

namespace {

constexpr int U = 2;                 // rows per lane-group per iteration
constexpr int TILE = 4 * 8 * U;      // rows per workgroup iteration
constexpr int NB = 4;                // 128-byte column blocks loaded together

typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));

// One-query workgroups: publish this chunk's best key (its list's first)
// in the query's row of heads, then take the K-th smallest distance of all
// chunks' published best keys as a bound: K chunks each hold a key at or
// below it, so the query's K-th key is too (unpublished chunks read
// KEY_INF; a stale entry is a larger key of the same chunk, still valid).
// Early in the scan this is far tighter than any one chunk's own K-th key,
// which is the K-th of the few rows that chunk has seen.  Whole workgroup.
__device__ void bound_from_heads(const ScreenArgs &a, int chunk, uint64_t best, uint64_t *thr,
                                 uint32_t *hist, int tid) {
    uint64_t *hq = a.heads + (int64_t)(blockIdx.y) * a.n_chunks;  // one query per workgroup row
    if (tid == 0) __atomic_store_n((unsigned long long *)(hq + chunk), (unsigned long long)best,
                                   __ATOMIC_RELAXED);
    constexpr int S = 4;
    uint32_t v[S];
#pragma unroll
    for (int e = 0; e < S; ++e) {
        const int i = e * 256 + tid;
        v[e] = i < a.n_chunks
                   ? (uint32_t)(__atomic_load_n((const unsigned long long *)(hq + i), __ATOMIC_RELAXED) >> 32)
                   : 0xffffffffu;
    }
    const uint32_t bd = block_kth_u32<S, 256>(v, a.n_chunks, a.K, hist, hist + 256);
    if (tid == 0 && bd != 0xffffffffu) {
        const uint64_t bk = ((uint64_t)bd << 32) | 0xffffffffu;
        if (bk < thr[0]) thr[0] = bk;
    }
}
__device__ __forceinline__ uint4 load_nt(const uint4 *p) {
    v4u32 v = __builtin_nontemporal_load((const v4u32 *)p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

template <int QT, int METRIC, int STORE, bool GATHER, bool BATCHED>
__global__ __launch_bounds__(256) void screen_stream_kernel(ScreenArgs a) {
    constexpr int V = Elem<STORE>::V;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane >> 3, s = lane & 7;
    const int qt0 = blockIdx.y * QT;
    const int chunk = blockIdx.x;

    extern __shared__ __align__(16) unsigned char smem[];
    const int M = a.Kp + a.CB;
    uint64_t *keys = (uint64_t *)smem;
    uint64_t *thr = keys + QT * M;
    int *cnt = (int *)(thr + QT);
    float *qs = (float *)(cnt + QT + 2);  // 8-byte aligned; [QT][dp]
    qs = (float *)(((uintptr_t)qs + 15) & ~(uintptr_t)15);
    uint32_t *hist = (uint32_t *)(qs + QT * a.dp);  // [256 + 2] radix-select scratch

    TopkLds<uint64_t> tk{keys, cnt, thr, QT, a.K, a.Kp, a.CB};
    for (int i = tid; i < QT * a.dp; i += 256) {
        int b = i / a.dp, j = i - b * a.dp;
        qs[i] = (qt0 + b < a.B) ? a.qp[(int64_t)(qt0 + b) * a.dp + j] : 0.0f;
    }
    tk.init(tid, 256);  // includes a barrier

    PredDev qpred[QT];
    if (BATCHED) {
#pragma unroll
        for (int b = 0; b < QT; ++b)
            qpred[b] = (qt0 + b < a.B) ? a.preds[qt0 + b] : PredDev{0, {0}, {0}, {0}};
    }

    const int64_t total = GATHER ? *a.sel_count : a.n;
    int64_t per = (total + a.n_chunks - 1) / a.n_chunks;
    // (masked rows: whole tiles per chunk, so that row loads stay aligned;
    // gathered rows are scattered anyway, and a selective predicate's few
    // ids then spread over every chunk instead of filling a few chunks'
    // lists, which the merge would read a few keys at a time)
    if (!GATHER) per = (per + TILE - 1) / TILE * TILE;
    const int64_t c0 = (int64_t)chunk * per;
    const int64_t c1 = min(total, c0 + per);
    const int eb = (STORE == VRS_F32) ? 4 : (STORE == VRS_BF16 ? 2 : 1);
    const int64_t row_bytes = (int64_t)a.dp * eb;
    const int nblk = (int)(row_bytes / 128);   // 128-byte column blocks per row
    const char *base = (const char *)a.rows;

    // Row ids and raw predicate columns of a tile are fetched one tile ahead,
    // so their latency overlaps the current tile's vector loads.
    auto fetch = [&](int64_t t0, int64_t(&rw)[U], bool(&vd)[U], int32_t(&av)[U][4]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t pos = t0 + u * 32 + wave * 8 + r;
            vd[u] = pos < c1;
            rw[u] = GATHER ? (vd[u] ? (int64_t)a.sel_ids[pos] : 0) : pos;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                av[u][t] = (!GATHER && !BATCHED && vd[u] && t < a.pred.nterms)
                               ? a.attr[(int64_t)a.pred.col[t] * a.an + rw[u]]
                               : 0;
        }
    };
    auto decide = [&](const bool(&vd)[U], const int32_t(&av)[U][4], bool(&ql)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            bool ok = vd[u];
            if (!GATHER && !BATCHED) {
                ok = ok && a.pred.nterms >= 0;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (t < a.pred.nterms) ok = ok && av[u][t] >= a.pred.lo[t] && av[u][t] <= a.pred.hi[t];
            }
            ql[u] = ok;
        }
    };
    int64_t row[U], nrow[U];
    bool qual[U], nvd[U];
    int32_t nav[U][4];
    {
        bool vd[U];
        int32_t av[U][4];
        fetch(c0, row, vd, av);
        decide(vd, av, qual);
    }
    for (int64_t t0 = c0; t0 < c1; t0 += TILE) {
        fetch(t0 + TILE, nrow, nvd, nav);
        bool any = false;
#pragma unroll
        for (int u = 0; u < U; ++u) any = any || qual[u];
        if (__ballot(any) != 0) {
            float acc[U][QT];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int b = 0; b < QT; ++b) acc[u][b] = 0.0f;
            // Issue the loads of NB column blocks of every row before using
            // any of them, so each lane keeps U*NB 16-byte loads in flight.
            // Rows are read once per scan: non-temporal loads.
            for (int cg = 0; cg < nblk; cg += NB) {
                uint4 w[U][NB];
#pragma unroll
                for (int c = 0; c < NB; ++c)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (qual[u] && cg + c < nblk)
                            w[u][c] = load_nt((const uint4 *)(base + row[u] * row_bytes + (cg + c) * 128 + s * 16));
                        else
                            w[u][c] = make_uint4(0, 0, 0, 0);
                    }
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    if (cg + c >= nblk) break;
                    const int e0 = ((cg + c) * 128 + s * 16) / eb;  // first element of the slice
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        float x[V];
                        Elem<STORE>::decode(w[u][c], x);
#pragma unroll
                        for (int b = 0; b < QT; ++b) {
                            const float *qb = qs + b * a.dp + e0;
#pragma unroll
                            for (int v = 0; v < V; ++v) {
                                if (METRIC == VRS_L2SQ) {
                                    float t = qb[v] - x[v];
                                    acc[u][b] = fmaf(t, t, acc[u][b]);
                                } else {
                                    acc[u][b] = fmaf(qb[v], x[v], acc[u][b]);
                                }
                            }
                        }
                    }
                }
            }
            // finish the row sums across the 8 lanes of each row
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int b = 0; b < QT; ++b) {
                    float v = acc[u][b];
                    v += __shfl_xor(v, 1);
                    v += __shfl_xor(v, 2);
                    v += __shfl_xor(v, 4);
                    acc[u][b] = v;
                }
            // lane s of each row pushes query s
#pragma unroll
            for (int u = 0; u < U; ++u) {
                float mine = 0.0f;
#pragma unroll
                for (int b = 0; b < QT; ++b)
                    if (b == s) mine = acc[u][b];
                bool ok = qual[u] && s < QT && qt0 + s < a.B;
                if (BATCHED && ok) {
#pragma unroll
                    for (int b = 0; b < QT; ++b)
                        if (b == s) ok = pred_eval(qpred[b], a.attr, a.an, row[u]);
                }
                if (ok) {
                    float dist;
                    if (METRIC == VRS_L2SQ)
                        dist = mine;
                    else if (STORE == VRS_FP8E4M3)
                        dist = -(a.scale[row[u]] * mine);
                    else
                        dist = -mine;
                    tk.push(s, make_key(dist, (uint32_t)row[u]));
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) row[u] = nrow[u];
        decide(nvd, nav, qual);
        __syncthreads();
        if (tk.need_flush(TILE)) {
            flush_sized<uint64_t, 256>(tk, tid);
            // publish this chunk's K-th key per query and adopt the best one
            if (tid < QT && qt0 + tid < a.B && thr[tid] != KEY_INF) {
                const uint64_t prev = atomicMin((unsigned long long *)(a.gthr + qt0 + tid),
                                                (unsigned long long)thr[tid]);
                if (prev < thr[tid]) thr[tid] = prev;
            }
            if (QT == 1 && !BATCHED && a.heads_bound && a.n_chunks >= a.K && a.n_chunks <= 4 * 256)
                bound_from_heads(a, chunk, keys[0], thr, hist, tid);
            __syncthreads();
        }
    }
    if (tk.need_flush(a.CB)) flush_sized<uint64_t, 256>(tk, tid);  // any pending candidate
    for (int i = tid; i < QT * a.K; i += 256) {
        int b = i / a.K, j = i - b * a.K;
        if (qt0 + b < a.B)
            a.partials[((int64_t)(qt0 + b) * a.n_chunks + chunk) * a.K + j] = keys[b * M + j];
    }
    // the lists' first keys side by side, for the merge's bound
    if (a.heads && tid < QT && qt0 + tid < a.B)
        a.heads[(int64_t)(qt0 + tid) * a.n_chunks + chunk] = keys[tid * M];
}

template <int QT, int METRIC, int STORE>
hipError_t launch_q(const ScreenArgs &a, hipStream_t s) {
    dim3 grid(a.n_chunks, (a.B + QT - 1) / QT), block(256);
    size_t lds = screen_stream_lds(QT, a.Kp, a.CB, a.dp);
    if (a.preds) {
        if (a.gather) return hipErrorInvalidValue;
        screen_stream_kernel<QT, METRIC, STORE, false, true><<<grid, block, lds, s>>>(a);
    } else if (a.gather) {
        screen_stream_kernel<QT, METRIC, STORE, true, false><<<grid, block, lds, s>>>(a);
    } else {
        screen_stream_kernel<QT, METRIC, STORE, false, false><<<grid, block, lds, s>>>(a);
    }
    return hipGetLastError();
}

template <int QT>
hipError_t launch_qt(const ScreenArgs &a, hipStream_t s) {
    if (a.metric == VRS_L2SQ) {
        if (a.store != VRS_F32) return hipErrorInvalidValue;
        return launch_q<QT, VRS_L2SQ, VRS_F32>(a, s);
    }
    switch (a.store) {
    case VRS_F32: return launch_q<QT, VRS_IP, VRS_F32>(a, s);
    case VRS_BF16: return launch_q<QT, VRS_IP, VRS_BF16>(a, s);
    default: return launch_q<QT, VRS_IP, VRS_FP8E4M3>(a, s);
    }
}

}  // namespace

size_t screen_stream_lds(int qt, int Kp, int CB, int dp) {
    return (size_t)qt * (Kp + CB) * 8 + qt * 8 + (qt + 2) * 4 + 16 + (size_t)qt * dp * 4 + 258 * 4;
}

hipError_t launch_screen_stream(const ScreenArgs &a, int qt, hipStream_t s) {
    switch (qt) {
    case 1: return launch_qt<1>(a, s);
    case 2: return launch_qt<2>(a, s);
    case 4: return launch_qt<4>(a, s);
    default: return launch_qt<8>(a, s);
    }
}

}  // namespace vrs
