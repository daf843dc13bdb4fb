// k_range.hip -- threshold selection: for every query b, the rows i that
// satisfy the relational predicate and whose exact FP64 distance is below
// thr[b], ascending by row id.  This is the selection with a query vector and
// a similarity predicate of Section 3 (eq. 1), with the relational predicate
// pushed down as in eq. 3; the paper's evaluation uses a cosine-similarity
// threshold (Section 5, "Dataset"): on normalised rows and a normalised
// query, similarity > t is IP distance < -t.
//
//   prep:   per query the screening admission bound tf >= thr + E, rounded up
//           to float (E bounds |FP32 screening - FP64 distance|), an empty
//           bitmap and a zero candidate counter;
//   screen: VALU streaming pass, eight lanes per 128-byte row block: the
//           FP32 distance of every qualifying (query, row) pair; rows below
//           tf are candidates, appended per query with one atomic per wave
//           step that has any;
//   exact:  the exact FP64 distance of every candidate (64 per wave, one per
//           lane: the definition's chain); rows below thr set their bit in
//           the query's bitmap.  A query with more candidates than its slots
//           goes to the overflow list instead;
//   full:   overflowed queries: the exact distance of every qualifying row;
//   count, ids: order-preserving compaction of each bitmap (the first cap
//           ids, ascending) and the number of selected rows;
//   dist:   the exact distance of every written id, rounded to float, and
//           the padding (-1, +inf) after the last one.
#include "exact64.h"

namespace vrs {

namespace {

constexpr int RG_STEPS = RANGE_BLOCK_ROWS / 256;  // 256-row steps per compaction block

__global__ __launch_bounds__(256) void range_prep_kernel(RangeArgs a) {
    const int b = blockIdx.y;
    uint32_t *bm = a.bitmap + (int64_t)b * a.words;
    for (int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x; w < a.words; w += (int64_t)gridDim.x * 256)
        bm[w] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.cnt[b] = 0u;
        if (b == 0) *a.ovf_count = 0;
        // (thr = +inf admits every row, -inf or NaN none: inf - inf and NaN
        // comparisons are false)
        const double th = a.thr[b], qn = a.qnorm[b];
        const double E = a.rel * fabs(th) + a.abs_ip * qn * a.max_norm +
                         a.abs_l2 * (qn + a.max_norm) * (qn + a.max_norm);
        const double t = th + E;
        float f = (float)t;
        if ((double)f < t) f = nextafterf(f, __int_as_float(0x7f800000));
        a.tf[b] = f;
    }
}

// QT queries per workgroup (grid.y = query groups), chunk blockIdx.x of the
// rows (or of the selection vector).  Wave w, lane group r = lane / 8 holds
// row t0 + u * 32 + w * 8 + r; lane s = lane % 8 reads the 16-byte slots s,
// s + 8, ... of it, four 128-byte blocks at a time.
template <int QT, int METRIC, int STORE, bool GATHER>
__global__ __launch_bounds__(256) void range_screen_kernel(RangeArgs a) {
    constexpr int V = STORE == VRS_F32 ? 4 : (STORE == VRS_BF16 ? 8 : 16);  // elements per 16 B
    constexpr int EB = 16 / V;
    constexpr int U = 2;
    constexpr int STEP = 4 * 8 * U;
    constexpr int NB = 4;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r = lane >> 3, sl = lane & 7;
    const int qt0 = blockIdx.y * QT;
    extern __shared__ __align__(16) unsigned char smem[];
    float *qs = (float *)smem;  // [QT][dp]
    __shared__ float tfs[QT];
    for (int i = tid; i < QT * a.dp; i += 256) {
        const int b = i / a.dp, j = i - b * a.dp;
        qs[i] = qt0 + b < a.B ? a.qp[(int64_t)(qt0 + b) * a.dp + j] : 0.0f;
    }
    // a query slot past the batch admits nothing (x < -inf is false)
    if (tid < QT) tfs[tid] = qt0 + tid < a.B ? a.tf[qt0 + tid] : __int_as_float(0xff800000);
    __syncthreads();
    const int64_t total = GATHER ? *a.sel_count : a.n;
    int64_t per = (total + a.n_chunks - 1) / a.n_chunks;
    per = (per + STEP - 1) / STEP * STEP;
    const int64_t c0 = (int64_t)blockIdx.x * per;
    const int64_t c1 = min(total, c0 + per);
    const int64_t row_bytes = (int64_t)a.dp * EB;
    const int nblk = (int)(row_bytes / 128);
    const char *base = (const char *)a.rows;
    const uint64_t lt = (1ull << lane) - 1ull;
    // the next step's rows (gather: their ids; mask: their predicate
    // columns) are fetched while this step's rows are loaded and multiplied
    int64_t prow[U];
    bool pin[U];
    int32_t pav[U][4];
    auto fetch = [&](int64_t t) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t pos = t + u * 32 + wave * 8 + r;
            pin[u] = pos < c1;
            prow[u] = GATHER ? (pin[u] ? (int64_t)a.sel_ids[pos] : 0) : (pin[u] ? pos : 0);
#pragma unroll
            for (int tt = 0; tt < 4; ++tt)
                pav[u][tt] = (!GATHER && pin[u] && tt < a.pred.nterms)
                                 ? a.attr[(int64_t)a.pred.col[tt] * a.an + prow[u]]
                                 : 0;
        }
    };
    fetch(c0);
    for (int64_t t0 = c0; t0 < c1; t0 += STEP) {
        int64_t row[U];
        bool ok[U];
        bool any = false;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            row[u] = prow[u];
            bool q = pin[u];
            if (!GATHER) {
                q = q && a.pred.nterms >= 0;
#pragma unroll
                for (int tt = 0; tt < 4; ++tt)
                    if (tt < a.pred.nterms) q = q && pav[u][tt] >= a.pred.lo[tt] && pav[u][tt] <= a.pred.hi[tt];
            }
            ok[u] = q;
            any = any || q;
        }
        if (t0 + STEP < c1) fetch(t0 + STEP);
        if (__ballot(any) == 0) continue;  // (wave-uniform)
        float acc[U][QT];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int b = 0; b < QT; ++b) acc[u][b] = 0.0f;
        for (int blk = 0; blk < nblk; blk += NB) {
            uint4 w[U][NB];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < NB; ++k)
                    if (blk + k < nblk) {  // (non-temporal: each row is read once;
                        w[u][k] = make_uint4(0u, 0u, 0u, 0u);  //  rows the predicate drops are not read)
                        if (ok[u]) {
                            const x64_u32x4 v = __builtin_nontemporal_load(
                                (const x64_u32x4 *)(base + row[u] * row_bytes + (int64_t)(blk + k) * 128 + sl * 16));
                            w[u][k] = make_uint4(v.x, v.y, v.z, v.w);
                        }
                    }
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if (blk + k >= nblk) break;
                const int j0 = ((blk + k) * 128 + sl * 16) / EB;  // first coordinate of the slot
                float x[U][V];
#pragma unroll
                for (int u = 0; u < U; ++u) decode16<STORE>(w[u][k], x[u]);
#pragma unroll
                for (int b = 0; b < QT; ++b) {
                    const float *qq = qs + b * a.dp + j0;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const float qv = qq[v];
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            if (METRIC == VRS_L2SQ) {
                                const float t = qv - x[u][v];
                                acc[u][b] = fmaf(t, t, acc[u][b]);
                            } else {
                                acc[u][b] = fmaf(qv, x[u][v], acc[u][b]);
                            }
                        }
                    }
                }
            }
        }
        float sc[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            sc[u] = (STORE == VRS_FP8E4M3 && ok[u]) ? a.scale[row[u]] : 1.0f;
#pragma unroll
        for (int b = 0; b < QT; ++b) {
            uint64_t m[U];
            int c = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                float v = acc[u][b];
                v += __shfl_xor(v, 1);
                v += __shfl_xor(v, 2);
                v += __shfl_xor(v, 4);
                const float dist = METRIC == VRS_IP ? -(sc[u] * v) : v;
                m[u] = __ballot(sl == 0 && ok[u] && dist < tfs[b]);
                c += __popcll(m[u]);
            }
            if (c == 0) continue;  // (wave-uniform)
            uint32_t basec = 0;
            if (lane == 0) basec = atomicAdd(&a.cnt[qt0 + b], (uint32_t)c);
            basec = __shfl(basec, 0);
            uint32_t before = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if ((m[u] >> lane) & 1ull) {
                    const uint32_t pos = basec + before + (uint32_t)__popcll(m[u] & lt);
                    if (pos < (uint32_t)a.cap_c) a.cand[(int64_t)(qt0 + b) * a.cap_c + pos] = (int32_t)row[u];
                }
                before += (uint32_t)__popcll(m[u]);
            }
        }
    }
}

// LDS: the FP64 query [dp], then four waves' staging areas.
size_t range_x64_lds(int dp) { return (size_t)dp * 8 + 4 * X64_WAVE_LDS; }

__device__ __forceinline__ void fill_qd(const RangeArgs &a, int b, double *qd) {
    for (int j = threadIdx.x; j < a.dp; j += 256) qd[j] = j < a.d ? (double)a.q[(int64_t)b * a.d + j] : 0.0;
}

__device__ __forceinline__ void set_bit(const RangeArgs &a, int b, int row) {
    atomicOr(&a.bitmap[(int64_t)b * a.words + (row >> 5)], 1u << (row & 31));
}

template <int STORE, int METRIC>
__global__ __launch_bounds__(256) void range_exact_kernel(RangeArgs a) {
    const int b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nc = a.cnt[b];
    if (nc > (uint32_t)a.cap_c) {  // more candidates than slots: exact pass over every row
        if (blockIdx.x == 0 && tid == 0) a.ovf_list[atomicAdd(a.ovf_count, 1)] = b;
        return;
    }
    const int ntask = (int)((nc + 63) / 64);
    if ((int)blockIdx.x * 4 >= ntask) return;
    extern __shared__ __align__(16) unsigned char smem[];
    double *qd = (double *)smem;
    x64_u32x4 *stage = (x64_u32x4 *)(smem + (size_t)a.dp * 8 + (size_t)wave * X64_WAVE_LDS);
    fill_qd(a, b, qd);
    __syncthreads();
    const double th = a.thr[b];
    for (int t = blockIdx.x * 4 + wave; t < ntask; t += gridDim.x * 4) {
        const int ci = t * 64 + lane;
        const bool has = ci < (int)nc;
        const int row = has ? a.cand[(int64_t)b * a.cap_c + ci] : 0;
        const double dv = exact64_wave<STORE, METRIC>(a.rows, a.scale, row, has, qd, a.dp, stage);
        if (has && dv < th) set_bit(a, b, row);
    }
}

template <int STORE, int METRIC, bool GATHER>
__global__ __launch_bounds__(256) void range_full_kernel(RangeArgs a) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nf = *a.ovf_count;
    if (nf == 0) return;
    extern __shared__ __align__(16) unsigned char smem[];
    double *qd = (double *)smem;
    x64_u32x4 *stage = (x64_u32x4 *)(smem + (size_t)a.dp * 8 + (size_t)wave * X64_WAVE_LDS);
    const int64_t total = GATHER ? *a.sel_count : a.n;
    const int64_t per = ((total + a.fb_chunks - 1) / a.fb_chunks + 63) / 64 * 64;
    const int64_t tasks = (int64_t)nf * a.fb_chunks;
    for (int64_t task = blockIdx.x; task < tasks; task += gridDim.x) {
        const int b = a.ovf_list[task / a.fb_chunks];
        const int64_t c0 = (task % a.fb_chunks) * per, c1 = min(total, c0 + per);
        __syncthreads();  // every wave done with the previous query
        fill_qd(a, b, qd);
        __syncthreads();
        const double th = a.thr[b];
        for (int64_t p0 = c0 + wave * 64; p0 < c1; p0 += 256) {
            const int64_t pos = p0 + lane;
            bool has = pos < c1;
            const int row = has ? (GATHER ? a.sel_ids[pos] : (int)pos) : 0;
            if (!GATHER && has) has = pred_eval(a.pred, a.attr, a.an, row);
            const double dv = exact64_wave<STORE, METRIC>(a.rows, a.scale, row, has, qd, a.dp, stage);
            if (has && dv < th) set_bit(a, b, row);
        }
    }
}

// Selected rows per block of RANGE_BLOCK_ROWS rows (256 bitmap words).
__global__ __launch_bounds__(256) void range_count_kernel(RangeArgs a) {
    const int b = blockIdx.y;
    const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t c = w < a.words ? (uint32_t)__popc(a.bitmap[(int64_t)b * a.words + w]) : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    __shared__ uint32_t wc[4];
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) a.blkcnt[(int64_t)b * a.nblk + blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

// Order-preserving compaction of query b's bitmap, block blockIdx.x: row
// base + s * 256 + tid belongs to thread tid at step s (the layout of the
// selection pass).  Ids at positions >= cap are dropped; the last block
// writes the count.
__global__ __launch_bounds__(256) void range_ids_kernel(RangeArgs a) {
    const int b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ uint64_t red[256];
    __shared__ uint32_t pre[RG_STEPS * 4];
    __shared__ uint32_t wtot;
    const uint32_t *bm = a.bitmap + (int64_t)b * a.words;
    const int64_t base = (int64_t)blockIdx.x * RANGE_BLOCK_ROWS + tid;
    uint32_t wd[RG_STEPS];
#pragma unroll
    for (int s = 0; s < RG_STEPS; ++s) {
        const int64_t row = base + s * 256;
        wd[s] = row < a.n ? bm[row >> 5] : 0u;
    }
    uint64_t part = 0;
    const uint32_t *bc = a.blkcnt + (int64_t)b * a.nblk;
    for (int j = tid; j < (int)blockIdx.x; j += 256) part += bc[j];
    red[tid] = part;
    uint64_t m[RG_STEPS];
#pragma unroll
    for (int s = 0; s < RG_STEPS; ++s) {
        const int64_t row = base + s * 256;
        m[s] = __ballot(row < a.n && ((wd[s] >> (row & 31)) & 1u));
        if (lane == 0) pre[s * 4 + wave] = (uint32_t)__popcll(m[s]);
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const uint64_t off = red[0];
    static_assert(RG_STEPS * 4 == 128, "two waves scan the step counts");
    uint32_t c = 0, inc = 0;
    if (tid < 128) {
        c = pre[tid];
        inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        if (tid == 63) wtot = inc;
    }
    __syncthreads();
    if (tid < 128) {
        const uint32_t ex = inc - c + (tid >= 64 ? wtot : 0u);
        pre[tid] = ex;
        if (tid == 127 && (int)blockIdx.x == a.nblk - 1) a.out_count[b] = (int64_t)(off + ex + c);
    }
    __syncthreads();
    const uint64_t lt = (1ull << lane) - 1ull;
    int64_t *oi = a.out_idx + (int64_t)b * a.cap;
#pragma unroll
    for (int s = 0; s < RG_STEPS; ++s) {
        if ((m[s] >> lane) & 1ull) {
            const uint64_t pos = off + pre[s * 4 + wave] + (uint32_t)__popcll(m[s] & lt);
            if (pos < (uint64_t)a.cap) oi[pos] = base + s * 256;
        }
    }
}

template <int STORE, int METRIC>
__global__ __launch_bounds__(256) void range_dist_kernel(RangeArgs a) {
    const int b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t m = min(a.out_count[b], (int64_t)a.cap);
    extern __shared__ __align__(16) unsigned char smem[];
    double *qd = (double *)smem;
    x64_u32x4 *stage = (x64_u32x4 *)(smem + (size_t)a.dp * 8 + (size_t)wave * X64_WAVE_LDS);
    if ((int64_t)blockIdx.x * 256 < m) {  // (block-uniform)
        fill_qd(a, b, qd);
        __syncthreads();
    }
    int64_t *oi = a.out_idx + (int64_t)b * a.cap;
    float *od = a.out_dist + (int64_t)b * a.cap;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t * 64 < a.cap; t += (int64_t)gridDim.x * 4) {
        const int64_t p = t * 64 + lane;
        if (t * 64 < m) {  // (wave-uniform)
            const bool has = p < m;
            const int row = has ? (int)oi[p] : 0;
            const double dv = exact64_wave<STORE, METRIC>(a.rows, a.scale, row, has, qd, a.dp, stage);
            if (has) od[p] = (float)dv;
        }
        if (p < a.cap && p >= m) {
            oi[p] = -1;
            od[p] = __int_as_float(0x7f800000);
        }
    }
}

template <int STORE, int METRIC>
hipError_t range_step(const RangeArgs &a, int qt, int step, hipStream_t s) {
    const int B = a.B;
    if (step == 0) {
        const int gx = (int)std::max<int64_t>(1, std::min<int64_t>((a.words + 255) / 256, 1024 / B + 1));
        range_prep_kernel<<<dim3(gx, B), 256, 0, s>>>(a);
    } else if (step == 1) {
        const size_t lds_q = (size_t)qt * a.dp * 4;
        const dim3 gs(a.n_chunks, (B + qt - 1) / qt);
#define RG_SCREEN(QT_)                                                                        \
    if (a.gather) {                                                                           \
        ensure_dyn_lds((const void *)range_screen_kernel<QT_, METRIC, STORE, true>, lds_q);   \
        range_screen_kernel<QT_, METRIC, STORE, true><<<gs, 256, lds_q, s>>>(a);              \
    } else {                                                                                  \
        ensure_dyn_lds((const void *)range_screen_kernel<QT_, METRIC, STORE, false>, lds_q);  \
        range_screen_kernel<QT_, METRIC, STORE, false><<<gs, 256, lds_q, s>>>(a);             \
    }
        switch (qt) {
        case 1: RG_SCREEN(1) break;
        case 2: RG_SCREEN(2) break;
        case 4: RG_SCREEN(4) break;
        default: RG_SCREEN(8) break;
        }
#undef RG_SCREEN
    } else if (step == 2) {
        const size_t lds_x = range_x64_lds(a.dp);
        const int gx = std::max(1, std::min((a.cap_c + 255) / 256, 1024 / B + 1));
        ensure_dyn_lds((const void *)range_exact_kernel<STORE, METRIC>, lds_x);
        range_exact_kernel<STORE, METRIC><<<dim3(gx, B), 256, lds_x, s>>>(a);
        if (a.gather) {
            ensure_dyn_lds((const void *)range_full_kernel<STORE, METRIC, true>, lds_x);
            range_full_kernel<STORE, METRIC, true><<<1024, 256, lds_x, s>>>(a);
        } else {
            ensure_dyn_lds((const void *)range_full_kernel<STORE, METRIC, false>, lds_x);
            range_full_kernel<STORE, METRIC, false><<<1024, 256, lds_x, s>>>(a);
        }
    } else {
        range_count_kernel<<<dim3(a.nblk, B), 256, 0, s>>>(a);
        range_ids_kernel<<<dim3(a.nblk, B), 256, 0, s>>>(a);
        const size_t lds_x = range_x64_lds(a.dp);
        const int gd = std::max(1, std::min((a.cap + 255) / 256, 1024 / B + 1));
        ensure_dyn_lds((const void *)range_dist_kernel<STORE, METRIC>, lds_x);
        range_dist_kernel<STORE, METRIC><<<dim3(gd, B), 256, lds_x, s>>>(a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_range(const RangeArgs &a, int qt, int step, hipStream_t s) {
    if (a.metric == VRS_L2SQ) return range_step<VRS_F32, VRS_L2SQ>(a, qt, step, s);  // float32 tables only
    switch (a.store) {
    case VRS_F32: return range_step<VRS_F32, VRS_IP>(a, qt, step, s);
    case VRS_BF16: return range_step<VRS_BF16, VRS_IP>(a, qt, step, s);
    default: return range_step<VRS_FP8E4M3, VRS_IP>(a, qt, step, s);
    }
}

}  // namespace vrs
