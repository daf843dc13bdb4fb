// k_batched.hip -- the batched uneven form: thousands of concurrent queries,
// each with its own conjunctive range predicate and its own k, in one
// launch sequence that never returns to the host (so it can be captured
// into a HIP graph and replayed).
//
// The paper's batched (tensor) form stages one shared filter before the
// batch (Sections 3.1-3.2); with a predicate per query the two ways of
// pushing the predicate down (Section 3.2: checked on the fly per pair, or
// staged into a selection vector first) are chosen per query:
//   * dense queries (many qualifying rows) run on the MFMA screening kernel,
//     64 queries per work item sharing every row read, with the predicate
//     checked per (query, row) pair (compute-then-mask);
//   * sparse queries (few qualifying rows) get their own selection vector
//     and a gather-then-compute VALU pass over exactly those rows.
// The split is decided on the device: a histogram estimate proposes the
// sparse candidates, one selection pass writes every candidate's qualifying
// row ids (up to the cap) and counts them exactly (a query whose count
// exceeds the cap goes dense), and the queries are permuted so that the
// dense ones occupy positions [0, n_dense).
//
// The selection pass is organised by 1024-row sub-blocks; the candidates
// are split over 8 waves per sub-block, each of which keeps its rows'
// values of the first two columns in registers and walks its share of the
// candidates, so the columns are read a few times however many queries
// there are; qualifying rows are found 64 at a time with one ballot per row
// group and term.  A candidate's list is its own region of the pool, filled
// in sub-block runs (ascending within a run, runs in the order their waves
// reserve them): the gather screening does not depend on the order.
#include "internal.h"
#include "topk_sized.h"

namespace vrs {

namespace {

constexpr int GROUPS = BSUB_ROWS / 64;  // 64-row groups per sub-block
constexpr int QSPLIT = 8;               // waves sharing one sub-block's queries

__device__ __forceinline__ bool eval_cached(const PredDev &p, int32_t v0, int32_t v1,
                                            const int32_t *__restrict__ attr, int64_t an,
                                            int64_t row) {
    bool ok = p.nterms >= 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (t < p.nterms) {
            const int c = p.col[t];
            const int32_t v = c == 0 ? v0 : (c == 1 ? v1 : attr[(int64_t)c * an + row]);
            ok = ok && v >= p.lo[t] && v <= p.hi[t];
        }
    }
    return ok;
}

// Estimated fraction of rows satisfying p: per term, the histogram mass of
// the range (uniform within a bin), multiplied over terms (independence).
__device__ double est_fraction(const void *dstats, int n_attr, const PredDev &p) {
    if (p.nterms < 0) return 0.0;
    const int32_t *amin = (const int32_t *)dstats, *amax = amin + 64;
    const uint32_t *hist = (const uint32_t *)(amax + 64);
    double sel = 1.0;
    for (int t = 0; t < p.nterms; ++t) {
        const int c = p.col[t];
        const int64_t lo = amin[c], span = (int64_t)amax[c] - lo + 1;
        double hit = 0.0, tot = 0.0;
        for (int b = 0; b < HIST_BINS; ++b) {
            const int64_t v0 = lo + ((int64_t)b * span + HIST_BINS - 1) / HIST_BINS;
            const int64_t v1 = lo + ((int64_t)(b + 1) * span + HIST_BINS - 1) / HIST_BINS;
            const double cb = (double)hist[(int64_t)c * HIST_BINS + b];
            tot += cb;
            if (v1 <= v0 || cb == 0.0) continue;
            const int64_t a = max(v0, (int64_t)p.lo[t]), z = min(v1 - 1, (int64_t)p.hi[t]);
            if (z >= a) hit += cb * (double)(z - a + 1) / (double)(v1 - v0);
        }
        sel *= tot > 0.0 ? hit / tot : 0.0;
    }
    return sel;
}

__global__ void batch_reset_kernel(int32_t *ctl) {
    if (threadIdx.x < BC_WORDS) ctl[threadIdx.x] = 0;
}

// Fold predicates and k, propose sparse candidates (appended to `cands`).
__global__ __launch_bounds__(256) void batch_prepare_kernel(BatchArgs a) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.B) return;
    const PredDev o = fold_pred_dev(a.preds[b], a.n_attr);
    a.pred_o[b] = o;
    int k = a.ks[b];
    k = k < 1 ? 1 : (k > a.kmax ? a.kmax : k);
    a.kc_o[b] = k;
    a.kps_o[b] = kprime_dev(k, a.kmult, a.f32_rule, a.kfloor);
    const QRange r = range_form(b, o);
    a.qr[b] = r;
    bool cand = false;
    if (a.rows_cap > 0) {
        if (o.nterms < 0)
            cand = true;
        else if (o.nterms > 0)
            cand = est_fraction(a.dstats, a.n_attr, o) * (double)a.n <= 4.0 * (double)a.rows_cap + 1024.0;
    }
    a.cand[b] = cand;
    a.tot[b] = cand ? 0 : -1;  // (candidates: the selection pass adds its counts)
    if (cand) a.cands[atomicAdd(&a.ctl[BC_NCAND], 1)] = r;
}

// Load the first two attribute columns of a wave's sub-block (lane l holds
// rows row0 + 64 g + l); rows past the table read the last row (their
// results are masked out by the caller).
__device__ __forceinline__ void load_sub(const BatchArgs &a, int64_t row0, int lane,
                                         int32_t (&v0)[GROUPS], int32_t (&v1)[GROUPS]) {
    const int32_t *c0 = a.attr;
    const int32_t *c1 = a.attr + (a.n_attr > 1 ? a.an : 0);
#pragma unroll
    for (int g = 0; g < GROUPS; ++g) {
        const int64_t row = min(row0 + g * 64 + lane, a.n - 1);
        v0[g] = c0[row];
        v1[g] = c1[row];
    }
}

// Lane mask of the qualifying rows of 64-row group g; `valid` is the mask
// of rows inside the table.
__device__ __forceinline__ uint64_t range_mask(const QRange &r, int32_t v0, int32_t v1) {
    // (one ballot per term: each compare writes its lane mask directly)
    return __ballot((uint32_t)(v0 - r.lo0) <= r.span0) & __ballot((uint32_t)(v1 - r.lo1) <= r.span1);
}

__device__ __forceinline__ uint64_t general_mask(const BatchArgs &a, const QRange &r, int32_t v0,
                                              int32_t v1, int64_t row) {
    return __ballot(eval_cached(a.pred_o[r.b], v0, v1, a.attr, a.an, min(row, a.n - 1)));
}

// Qualifying rows of query r in 64-row group g (lane mask); FULL: the
// whole sub-block lies inside the table.
template <bool FULL>
__device__ __forceinline__ uint64_t group_mask(const BatchArgs &a, const QRange &r, int32_t v0,
                                               int32_t v1, int64_t row0, int g, int lane) {
    uint64_t m = r.kind == 0 ? range_mask(r, v0, v1)
                             : general_mask(a, r, v0, v1, row0 + g * 64 + lane);
    if (!FULL) {
        const int64_t in = a.n - row0 - g * 64;
        if (in < 64) m &= in <= 0 ? 0ull : ((1ull << in) - 1ull);
    }
    return m;
}

// Query ranges are read 64 at a time, one per lane (all in flight together),
// and each query's fields are then taken from its lane (v_readlane: uniform
// values, no memory access inside the per-query loop).
__device__ __forceinline__ QRange range_of_lane(const QRange &mine, int t) {
    QRange r;
    r.b = __builtin_amdgcn_readlane(mine.b, t);
    r.kind = __builtin_amdgcn_readlane(mine.kind, t);
    r.lo0 = __builtin_amdgcn_readlane(mine.lo0, t);
    r.lo1 = __builtin_amdgcn_readlane(mine.lo1, t);
    r.span0 = (uint32_t)__builtin_amdgcn_readlane((int)mine.span0, t);
    r.span1 = (uint32_t)__builtin_amdgcn_readlane((int)mine.span1, t);
    return r;
}

// Rows of the sub-block that satisfy query r (the kind test is taken once,
// so the 16 row groups of the range form are independent instructions).
template <bool FULL>
__device__ __forceinline__ uint32_t count_query(const BatchArgs &a, const QRange &r, int64_t row0, int lane,
                                                const int32_t (&v0)[GROUPS], const int32_t (&v1)[GROUPS]) {
    uint32_t c = 0;
    if (r.kind == 0) {
#pragma unroll
        for (int g = 0; g < GROUPS; ++g) {
            uint64_t m = range_mask(r, v0[g], v1[g]);
            if (!FULL) {
                const int64_t in = a.n - row0 - g * 64;
                if (in < 64) m &= in <= 0 ? 0ull : ((1ull << in) - 1ull);
            }
            c += (uint32_t)__popcll(m);
        }
    } else if (r.kind == 1) {
#pragma unroll
        for (int g = 0; g < GROUPS; ++g) c += (uint32_t)__popcll(group_mask<FULL>(a, r, v0[g], v1[g], row0, g, lane));
    }
    return c;
}

// The selection pass of one wave: its share of the candidates against its
// sub-block, 64 candidates at a time: the count of each (lane t keeps
// candidate t's), one atomic per candidate with rows here for the first of
// its slots (the atomic also makes tot[b] the candidate's exact count once
// every sub-block has added its own), then the ids, slots past the cap
// dropped.
template <bool FULL>
__device__ __forceinline__ void select_sub(const BatchArgs &a, int part, int lane, int64_t row0,
                                           const int32_t (&v0)[GROUPS], const int32_t (&v1)[GROUPS]) {
    const uint64_t below = (1ull << lane) - 1ull;
    const int nc = a.ctl[BC_NCAND];
    const int j0 = (int)((int64_t)nc * part / QSPLIT), j1 = (int)((int64_t)nc * (part + 1) / QSPLIT);
    for (int jb = j0; jb < j1; jb += 64) {
        const QRange mine = jb + lane < j1 ? a.cands[jb + lane] : QRange{0, 2, 0, 0, 0u, 0u};
        const int m = min(64, j1 - jb);
        uint32_t myc = 0;
        for (int t = 0; t < m; ++t) {
            const uint32_t c = count_query<FULL>(a, range_of_lane(mine, t), row0, lane, v0, v1);
            myc = lane == t ? c : myc;
        }
        uint32_t base = 0;
        if (myc > 0) base = (uint32_t)atomicAdd(&a.tot[mine.b], (int32_t)myc);
        uint64_t todo = __ballot(myc > 0);
        while (todo) {
            const int t = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            const QRange r = range_of_lane(mine, t);
            uint32_t pos = (uint32_t)__builtin_amdgcn_readlane((int)base, t);
            int32_t *dst = a.pool + (int64_t)r.b * a.rows_cap;
#pragma unroll
            for (int g = 0; g < GROUPS; ++g) {
                const uint64_t mk = group_mask<FULL>(a, r, v0[g], v1[g], row0, g, lane);
                if (mk == 0) continue;  // (uniform: most groups of a selective query are empty)
                const uint32_t p = pos + (uint32_t)__popcll(mk & below);
                if (((mk >> lane) & 1ull) && p < (uint32_t)a.rows_cap) dst[p] = (int32_t)(row0 + g * 64 + lane);
                pos += (uint32_t)__popcll(mk);
            }
        }
    }
}

// Selection pass: wave (sub-block, part) takes part `part` of the candidate
// list.
__global__ __launch_bounds__(256, 3) void batch_select_kernel(BatchArgs a) {
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int sub = w / QSPLIT, part = w % QSPLIT;
    if (sub >= a.nsub || a.n_attr == 0 || a.ctl[BC_NCAND] == 0) return;
    const int64_t row0 = (int64_t)sub * BSUB_ROWS;
    int32_t v0[GROUPS], v1[GROUPS];
    load_sub(a, row0, lane, v0, v1);
    if (row0 + BSUB_ROWS <= a.n)
        select_sub<true>(a, part, lane, row0, v0, v1);
    else
        select_sub<false>(a, part, lane, row0, v0, v1);
}

// Exclusive prefix sum over the 1024 threads of the block; returns the total.
template <typename T>
__device__ T block_scan_1024(T v, T &excl, T *wsum /* [16] LDS */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    T before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
        const T s = wsum[w];
        if (w < wave) before += s;
        total += s;
    }
    __syncthreads();
    excl = before + x - v;
    return total;
}

// Final split and the permutation (dense queries first, each side in query
// order), list layout, sparse list offsets and work-item prefix sums.
__global__ __launch_bounds__(1024) void batch_order_kernel(BatchArgs a) {
    __shared__ int32_t ws32[16];
    const int tid = threadIdx.x;
    auto is_sparse = [&](int b) { return a.cand[b] && a.tot[b] >= 0 && (int64_t)a.tot[b] <= a.rows_cap; };
    int32_t ns = 0;
    for (int c0 = 0; c0 < a.B; c0 += 1024) {
        const int b = c0 + tid;
        int32_t e;
        ns += block_scan_1024<int32_t>(b < a.B && is_sparse(b) ? 1 : 0, e, ws32);
    }
    const int32_t nd = a.B - ns;
    const int32_t ndt = (nd + a.qm - 1) / a.qm;
    int32_t nc = ndt > 0 ? a.items_target / ndt : a.nc_cap;
    nc = nc / 8 * 8;
    nc = max(8, min(a.nc_cap, nc));
    int32_t run_d = 0, run_s = 0, run_seg = 0;
    for (int c0 = 0; c0 < a.B; c0 += 1024) {
        const int b = c0 + tid;
        const bool in = b < a.B;
        const bool sp = in && is_sparse(b);
        const int32_t cnt = sp ? a.tot[b] : 0;
        const int32_t segs = cnt == 0 ? 0 : min(a.seg_max, (cnt + a.seg_rows - 1) / a.seg_rows);
        int32_t rd, rs, rseg;
        const int32_t td = block_scan_1024<int32_t>(in && !sp ? 1 : 0, rd, ws32);
        const int32_t ts = block_scan_1024<int32_t>(sp ? 1 : 0, rs, ws32);
        const int32_t tseg = block_scan_1024<int32_t>(segs, rseg, ws32);
        if (in) {
            if (!sp) {
                const int pos = run_d + rd;
                a.perm[pos] = b;
                a.list_off[pos] = (int64_t)pos * nc;
                a.nlists[pos] = nc;
                a.sp_off[pos] = 0;
                a.sp_cnt[pos] = 0;
            } else {
                const int j = run_s + rs, pos = nd + j;
                a.perm[pos] = b;
                a.sp_off[pos] = (int64_t)b * a.rows_cap;  // (the query's own pool region)
                a.sp_cnt[pos] = cnt;
                a.seg_pre[j] = run_seg + rseg;
                a.list_off[pos] = (int64_t)nd * nc + run_seg + rseg;
                a.nlists[pos] = segs;
            }
        }
        run_d += td;
        run_s += ts;
        run_seg += tseg;
    }
    if (tid == 0) {
        a.seg_pre[ns] = run_seg;
        a.ctl[BC_NDENSE] = nd;
        a.ctl[BC_NSPARSE] = ns;
        a.ctl[BC_NC] = nc;
    }
}

// ------------------------------------------------- sparse gather screening
// Persistent: every workgroup takes (query, segment) items from a queue
// until none is left.  An item is a contiguous part of one query's
// selection vector; its rows are read with 16-byte loads, 8 lanes per
// 128-byte block as in the streaming kernel, and the FP32 distances go to
// an LDS top-k list whose K smallest keys become one list of the merge.
constexpr int SU = 2;                  // rows per lane-group per step
constexpr int STILE = 4 * 8 * SU;      // rows per workgroup step
constexpr int SNB = 4;                 // 128-byte blocks loaded together
constexpr int SP_CB_MIN = 256;

typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 load_nt(const uint4 *p) {
    v4u32 v = __builtin_nontemporal_load((const v4u32 *)p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

__host__ __device__ inline int sparse_m(int K) { return next_pow2(next_pow2(K) + SP_CB_MIN); }

template <int STORE, int METRIC>
__global__ __launch_bounds__(256) void screen_sparse_kernel(ScreenArgs a) {
    constexpr int V = Elem<STORE>::V;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane >> 3, s = lane & 7;
    const int M = sparse_m(a.K);
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *keys = (uint64_t *)smem;
    uint64_t *thr = keys + M;
    int *cnt = (int *)(thr + 1);
    float *qs = (float *)(((uintptr_t)(cnt + 4) + 15) & ~(uintptr_t)15);  // [dp]
    __shared__ int item_s;

    const int nd = a.bctl[BC_NDENSE], ns = a.bctl[BC_NSPARSE], nc = a.bctl[BC_NC];
    const int n_items = a.seg_pre[ns];
    const int eb = STORE == VRS_F32 ? 4 : (STORE == VRS_BF16 ? 2 : 1);
    const int64_t row_bytes = (int64_t)a.dp * eb;
    const int nblk = (int)(row_bytes / 128);
    const char *base = (const char *)a.rows;

    for (;;) {
        if (tid == 0) item_s = atomicAdd(&a.bctl[BC_QSPARSE], 1);
        __syncthreads();
        const int it = item_s;
        if (it >= n_items) break;
        // the sparse query j owning item `it`: seg_pre[j] <= it < seg_pre[j + 1]
        int lo = 0, hi = ns;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (a.seg_pre[mid] <= it) lo = mid;
            else hi = mid;
        }
        const int j = lo, pos = nd + j;
        const int seg = it - a.seg_pre[j], segs = a.seg_pre[j + 1] - a.seg_pre[j];
        const int64_t cntq = a.sp_cnt[pos];
        const int64_t r0 = cntq * seg / segs, r1 = cntq * (seg + 1) / segs;
        const int32_t *ids = a.sp_pool + a.sp_off[pos];
        const int Kq = a.kps[pos] + 1;
        const int Kp = next_pow2(Kq);
        TopkLds<uint64_t> tk{keys, cnt, thr, 1, Kq, Kp, M - Kp};
        for (int i = tid; i < a.dp; i += 256) qs[i] = a.qp[(int64_t)pos * a.dp + i];
        tk.init(tid, 256);  // barrier: item_s, qs and the list are ready

        for (int64_t t0 = r0; t0 < r1; t0 += STILE) {
            int64_t row[SU];
            bool ok[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int64_t p = t0 + u * 32 + wave * 8 + r;
                ok[u] = p < r1;
                row[u] = ok[u] ? (int64_t)ids[p] : 0;
            }
            float acc[SU] = {};
            for (int cg = 0; cg < nblk; cg += SNB) {
                uint4 w[SU][SNB];
#pragma unroll
                for (int c = 0; c < SNB; ++c)
#pragma unroll
                    for (int u = 0; u < SU; ++u)
                        w[u][c] = (ok[u] && cg + c < nblk)
                                      ? load_nt((const uint4 *)(base + row[u] * row_bytes + (cg + c) * 128 + s * 16))
                                      : make_uint4(0, 0, 0, 0);
#pragma unroll
                for (int c = 0; c < SNB; ++c) {
                    if (cg + c >= nblk) break;
                    const float *qb = qs + ((cg + c) * 128 + s * 16) / eb;
#pragma unroll
                    for (int u = 0; u < SU; ++u) {
                        float x[V];
                        Elem<STORE>::decode(w[u][c], x);
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            if (METRIC == VRS_L2SQ) {
                                const float t = qb[v] - x[v];
                                acc[u] = fmaf(t, t, acc[u]);
                            } else {
                                acc[u] = fmaf(qb[v], x[v], acc[u]);
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                float v = acc[u];
                v += __shfl_xor(v, 1);
                v += __shfl_xor(v, 2);
                v += __shfl_xor(v, 4);
                if (s == 0 && ok[u]) {
                    float dist;
                    if (METRIC == VRS_L2SQ)
                        dist = v;
                    else if (STORE == VRS_FP8E4M3)
                        dist = -(a.scale[row[u]] * v);
                    else
                        dist = -v;
                    tk.push(0, make_key(dist, (uint32_t)row[u]));
                }
            }
            __syncthreads();
            if (tk.need_flush(STILE)) {
                flush_sized<uint64_t, 256>(tk, tid);
                if (tid == 0 && thr[0] != KEY_INF) {
                    const uint64_t prev = atomicMin((unsigned long long *)(a.gthr + pos),
                                                    (unsigned long long)thr[0]);
                    if (prev < thr[0]) thr[0] = prev;
                }
                __syncthreads();
            }
        }
        if (tk.need_flush(M - Kp)) flush_sized<uint64_t, 256>(tk, tid);
        uint64_t *dst = a.partials + ((int64_t)nd * nc + a.seg_pre[j] + seg) * a.K;
        for (int i = tid; i < a.K; i += 256) dst[i] = i < Kq ? keys[i] : KEY_INF;
        __syncthreads();  // LDS and item_s are reused by the next item
    }
}

}  // namespace

hipError_t launch_batch_classify(const BatchArgs &b, hipStream_t s) {
    batch_reset_kernel<<<1, 64, 0, s>>>(b.ctl);
    batch_prepare_kernel<<<(b.B + 255) / 256, 256, 0, s>>>(b);
    if (b.rows_cap > 0) batch_select_kernel<<<(b.nsub * QSPLIT + 3) / 4, 256, 0, s>>>(b);
    batch_order_kernel<<<1, 1024, 0, s>>>(b);
    return hipGetLastError();
}

size_t screen_sparse_lds(int K, int dp) { return (size_t)sparse_m(K) * 8 + 8 + 16 + 16 + (size_t)dp * 4; }

hipError_t launch_screen_sparse(const ScreenArgs &a, int grid, hipStream_t s) {
    const size_t lds = screen_sparse_lds(a.K, a.dp);
    if (a.metric == VRS_L2SQ) {
        if (a.store != VRS_F32) return hipErrorInvalidValue;
        screen_sparse_kernel<VRS_F32, VRS_L2SQ><<<grid, 256, lds, s>>>(a);
    } else if (a.store == VRS_F32) {
        screen_sparse_kernel<VRS_F32, VRS_IP><<<grid, 256, lds, s>>>(a);
    } else if (a.store == VRS_BF16) {
        screen_sparse_kernel<VRS_BF16, VRS_IP><<<grid, 256, lds, s>>>(a);
    } else {
        screen_sparse_kernel<VRS_FP8E4M3, VRS_IP><<<grid, 256, lds, s>>>(a);
    }
    return hipGetLastError();
}

}  // namespace vrs
