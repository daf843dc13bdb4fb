// k_probe.hip -- the probe-based access path (Section 4): a partition index
// over the vector column and its filtered probe with pre-filtering (Section
// 4.1: the relational predicate decides which rows may enter the result,
// not which partitions are visited).
//
// Index build (k-means, squared L2 on the stored vectors; the assignment of
// rows to their exact nearest centroid is a vector join against the
// centroid table, done by the host code with the scan kernels):
//   list_count / list_prefix / list_place: the rows of every partition,
//       ascending, as one id array with per-partition offsets (each row block
//       is placed by one thread in row order, so the layout is fixed);
//   centroid_mean: the mean of every partition, an FP64 running sum over its
//       rows in ascending order, divided by the count, rounded to float32
//       (an empty partition keeps its centroid).
// Probe (after the coarse scan: every query's partitions ordered by the
// exact distance of their centroids):
//   probe_prefix: per query, the rows in the first i partitions of its walk
//       and the row budget's limit on the walk;
//   probe_count / probe_decide: rounds over growing windows of the walk,
//       counting the qualifying rows per partition with many workgroups per
//       query, then applying the walk's rules (nprobe partitions, then on
//       while fewer than min_cand rows qualified);
//   probe_score: the visited partitions' rows in fixed chunks, filtered by
//       the predicate into LDS, exact FP64 distances (64 per wave, one per
//       lane), the k smallest (distance, id) keys of every workgroup;
//   probe_merge: per query the k smallest of its workgroups' keys, written
//       out.
#include "exact64.h"
#include "topk_sized.h"

namespace vrs {

namespace {

__global__ __launch_bounds__(256) void list_count_kernel(const int64_t *__restrict__ assign, int64_t n,
                                                         int nlist, uint32_t *__restrict__ cnt) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *h = (uint32_t *)smem;  // [nlist]
    for (int c = threadIdx.x; c < nlist; c += 256) h[c] = 0u;
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * PROBE_LIST_BLOCK;
    const int64_t r1 = min(n, r0 + PROBE_LIST_BLOCK);
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) atomicAdd(&h[(int)assign[r]], 1u);
    __syncthreads();
    for (int c = threadIdx.x; c < nlist; c += 256) cnt[(int64_t)blockIdx.x * nlist + c] = h[c];
}

// One thread per partition: its first slot in every row block (turning the
// block counts into exclusive prefix sums over the blocks) and its size.
__global__ __launch_bounds__(256) void list_blocks_kernel(uint32_t *__restrict__ cnt, int nblk, int nlist,
                                                          int64_t *__restrict__ size) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= nlist) return;
    uint32_t run = 0;
    for (int b = 0; b < nblk; ++b) {
        uint32_t *p = cnt + (int64_t)b * nlist + c;
        const uint32_t v = *p;
        *p = run;
        run += v;
    }
    size[c] = run;
}

// Partition offsets: exclusive prefix sum of the sizes (one workgroup).
__global__ __launch_bounds__(1024) void list_offsets_kernel(const int64_t *__restrict__ size, int nlist,
                                                            int64_t *__restrict__ off) {
    __shared__ int64_t wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int64_t carry = 0;
    for (int c0 = 0; c0 < nlist; c0 += 1024) {
        const int c = c0 + tid;
        const int64_t v = c < nlist ? size[c] : 0;
        int64_t x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        int64_t before = 0, total = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wave) before += wsum[w];
            total += wsum[w];
        }
        if (c < nlist) off[c] = carry + before + x - v;
        carry += total;
        __syncthreads();
    }
    if (tid == 0) off[nlist] = carry;
}

// One thread per row block places the block's rows in row order.
__global__ __launch_bounds__(64) void list_place_kernel(const int64_t *__restrict__ assign, int64_t n,
                                                        int nlist, const uint32_t *__restrict__ cnt,
                                                        const int64_t *__restrict__ off, int32_t *__restrict__ ids) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *local = (uint32_t *)smem;  // [nlist]
    for (int c = threadIdx.x; c < nlist; c += 64) local[c] = 0u;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const uint32_t *base = cnt + (int64_t)blockIdx.x * nlist;
    const int64_t r0 = (int64_t)blockIdx.x * PROBE_LIST_BLOCK;
    const int64_t r1 = min(n, r0 + PROBE_LIST_BLOCK);
    for (int64_t r = r0; r < r1; ++r) {
        const int c = (int)assign[r];
        ids[off[c] + base[c] + local[c]++] = (int32_t)r;
    }
}

// Workgroup c: the mean of partition c over its rows (ascending), one
// coordinate per thread, FP64 running sum.
__global__ __launch_bounds__(256) void centroid_mean_kernel(const float *__restrict__ x32, int d,
                                                            const int64_t *__restrict__ off,
                                                            const int32_t *__restrict__ ids,
                                                            float *__restrict__ cent) {
    const int c = blockIdx.x;
    const int64_t m0 = off[c], m1 = off[c + 1];
    if (m1 == m0) return;  // an empty partition keeps its centroid
    const double cntd = (double)(m1 - m0);
    for (int j = threadIdx.x; j < d; j += 256) {
        double acc = 0.0;
        for (int64_t m = m0; m < m1; ++m) acc += (double)x32[(int64_t)ids[m] * d + j];
        cent[(int64_t)c * d + j] = (float)(acc / cntd);
    }
}

// Workgroup (x, b): the exact FP64 squared distances of query b to
// centroids [256 x, 256 x + 256) (64 per wave, one per lane) as (distance,
// centroid id) keys: with at most PROBE_SORT_MAX centroids the coarse scan is
// spread over ceil(nlist / 256) workgroups per query, so every query's
// centroid rows are read at once rather than 256 at a time by one
// workgroup.
__global__ __launch_bounds__(256) void probe_cdist_kernel(ProbeArgs a) {
    const int b = blockIdx.y, tid = threadIdx.x, wave = tid >> 6;
    extern __shared__ __align__(16) unsigned char smem[];
    x64_u32x4 *stage = (x64_u32x4 *)(smem + (size_t)wave * X64_WAVE_LDS);
    double *qd = (double *)(smem + 4 * X64_WAVE_LDS);
    for (int j = tid; j < a.cdp; j += 256) qd[j] = j < a.d ? (double)a.q[(int64_t)b * a.d + j] : 0.0;
    __syncthreads();
    const int c = blockIdx.x * 256 + tid;
    const bool has = c < a.nlist;
    if (__ballot(has) == 0) return;  // (wave-uniform; no barrier follows)
    const double dv = exact64_wave<VRS_F32, VRS_L2SQ>(a.cent_rows, nullptr, has ? c : 0, has, qd, a.cdp, stage);
    if (has) ((Key128 *)a.ckeys)[(int64_t)b * next_pow2(a.nlist) + c] = Key128{ord64(dv), (uint64_t)c};
}

// Compare-exchange: afterwards x <= y if up, y <= x otherwise.
__device__ __forceinline__ void key_ce(Key128 &x, Key128 &y, bool up) {
    const bool sw = up ? KeyOps<Key128>::less(y, x) : KeyOps<Key128>::less(x, y);
    if (sw) {
        const Key128 t = x;
        x = y;
        y = t;
    }
}

// Ascending bitonic sort of 256 R keys held by the 256 threads of a
// workgroup, thread t holding positions R t .. R t + R - 1 in k[] (on entry
// and on exit).  Pairs at a distance below R are in one thread, below 64 R
// in one wave (exchanged by shuffles); only the larger distances go through
// LDS (lds: 256 R keys) with workgroup barriers.
template <int R>
__device__ void block_sort_keys(Key128 (&k)[R], Key128 *lds) {
    const int tid = threadIdx.x;
    constexpr int P = 256 * R;
#pragma unroll
    for (int size = 2; size <= P; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride < R) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (!(r & stride)) key_ce(k[r], k[r | stride], ((R * tid + r) & size) == 0);
                continue;
            }
            if (stride >= 64 * R) {
                __syncthreads();  // (the previous stage's readers are done)
#pragma unroll
                for (int r = 0; r < R; ++r) lds[R * tid + r] = k[r];
                __syncthreads();
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = R * tid + r;
                Key128 y;
                if (stride >= 64 * R) {
                    y = lds[i ^ stride];
                } else {
                    y.hi = __shfl_xor(k[r].hi, stride / R);
                    y.lo = __shfl_xor(k[r].lo, stride / R);
                }
                // the lower position of an ascending pair (or the upper one
                // of a descending pair) keeps the smaller key
                const bool keep_min = ((i & stride) == 0) == ((i & size) == 0);
                const bool y_less = KeyOps<Key128>::less(y, k[r]);
                if (keep_min ? y_less : !y_less) k[r] = y;
            }
        }
    }
}

// Workgroup b: the `walk` centroids nearest to query b, in order of
// (distance, centroid id), into coarse[b], from the keys of every centroid
// (probe_cdist_kernel; at most PROBE_SORT_MAX of them, padded with
// KEY_INF keys to 256 R).
template <int R>
__global__ __launch_bounds__(256) void probe_sort_kernel(ProbeArgs a) {
    const int b = blockIdx.x, tid = threadIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    const int P = next_pow2(a.nlist);
    const Key128 *ck = (const Key128 *)a.ckeys + (int64_t)b * P;
    Key128 k[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int c = R * tid + r;
        k[r] = c < a.nlist ? ck[c] : Key128{KEY_INF, KEY_INF};
    }
    block_sort_keys<R>(k, (Key128 *)smem);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = R * tid + r;
        if (i < a.walk)
            a.coarse_out[(int64_t)b * a.walk + i] =
                (k[r].hi == KEY_INF && k[r].lo == KEY_INF) ? -1 : (int64_t)k[r].lo;
    }
}

// Workgroup b, more than PROBE_SORT_MAX centroids: the exact FP64
// squared-L2 distance of query b to every centroid (64 centroids per wave,
// one per lane) into a running top-`walk` list, and the `walk` nearest by
// (distance, centroid id), in order, into coarse[b].
__global__ __launch_bounds__(256) void probe_coarse_kernel(ProbeArgs a) {
    const int b = blockIdx.x, tid = threadIdx.x, wave = tid >> 6;
    extern __shared__ __align__(16) unsigned char smem[];
    x64_u32x4 *stage = (x64_u32x4 *)(smem + (size_t)wave * X64_WAVE_LDS);
    double *qd = (double *)(smem + 4 * X64_WAVE_LDS);
    Key128 *keys = (Key128 *)(qd + a.cdp);
    for (int j = tid; j < a.cdp; j += 256) qd[j] = j < a.d ? (double)a.q[(int64_t)b * a.d + j] : 0.0;
    const int Kp = next_pow2(a.walk);
    const int M = next_pow2(Kp + 256);
    Key128 *thr = keys + M;
    int *cnt = (int *)(thr + 1);
    TopkLds<Key128> tk{keys, cnt, thr, 1, a.walk, Kp, M - Kp};
    tk.init(tid, 256);  // (includes a barrier)
    for (int c0 = 0; c0 < a.nlist; c0 += 256) {
        const int c = c0 + tid;
        const bool has = c < a.nlist;
        if (__ballot(has) != 0) {  // (wave-uniform)
            const double dv = exact64_wave<VRS_F32, VRS_L2SQ>(a.cent_rows, nullptr, has ? c : 0, has, qd,
                                                              a.cdp, stage);
            if (has) tk.push(0, Key128{ord64(dv), (uint64_t)c});
        }
        __syncthreads();
        if (tk.need_flush(256)) tk.flush(tid, 256);
    }
    if (tk.need_flush(M - Kp)) tk.flush(tid, 256);
    for (int i = tid; i < a.walk; i += 256) {
        const Key128 kk = keys[i];
        a.coarse_out[(int64_t)b * a.walk + i] = (kk.hi == KEY_INF && kk.lo == KEY_INF) ? -1 : (int64_t)kk.lo;
    }
}

// Position m of the walk's rows -> the walk position i in [lo, hi) of its
// partition: the largest i with pre[i] <= m (pre[lo] <= m < pre[hi]).
__device__ __forceinline__ int walk_find(const int64_t *pre, int lo, int hi, int64_t m) {
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= m) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Workgroup b: the row prefix of query b's walk (pre[i] = rows in its first
// i partitions in centroid order) and its limit: the first partition always,
// each later one only while the rows visited stay within cap_c.  Opens the
// query's walk: position 0, no qualifying rows yet, counts cleared.
__global__ __launch_bounds__(PROBE_MAX_WALK) void probe_prefix_kernel(ProbeArgs a) {
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ int64_t wsum[PROBE_MAX_WALK / 64];
    __shared__ int lim;
    const int64_t *co = a.coarse + (int64_t)b * a.walk;
    int64_t *pre = a.pre + (int64_t)b * (a.walk + 1);
    const bool valid = tid < a.walk && co[tid] >= 0;
    const int64_t sz = valid ? a.list_off[co[tid] + 1] - a.list_off[co[tid]] : 0;
    int64_t x = sz;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    if (tid == 0) lim = a.walk;
    __syncthreads();
    int64_t incl = x;  // rows of the first tid + 1 partitions
    for (int w = 0; w < wave; ++w) incl += wsum[w];
    if (tid < a.walk) {
        pre[tid + 1] = incl;
        a.cnt[(int64_t)b * a.walk + tid] = 0u;
        if (!(valid && (tid == 0 || incl <= a.cap_c))) atomicMin(&lim, tid);
    }
    if (tid == 0) pre[0] = 0;
    __syncthreads();
    if (tid == 0) {
        int64_t *st = a.state + 4 * (int64_t)b;
        st[0] = lim > 0 ? 1 : 0;
        st[1] = 0;
        st[2] = 0;
        st[3] = lim;
        if (lim == 0 && a.taken) a.taken[b] = 0;
    }
}

// Task (g, b), one round of query b's walk: the qualifying rows of every
// partition at walk positions [w0, w1) within the limit, counted by gc
// workgroups (steps of 256 * PROBE_COUNT_R rows, the predicate columns read
// in partition order).  Lanes hold consecutive
// rows, so a wave's rows fall into a few runs of one partition each; every
// run adds its count with one LDS atomic.
__global__ __launch_bounds__(256) void probe_count_kernel(ProbeArgs a) {
    const int g = blockIdx.x, b = blockIdx.y, tid = threadIdx.x, lane = tid & 63;
    int64_t *st = a.state + 4 * (int64_t)b;
    if (st[0] == 0) return;  // decided by an earlier round (uniform)
    __shared__ int64_t spre[PROBE_MAX_WALK + 1];
    __shared__ int64_t sbase[PROBE_MAX_WALK];
    __shared__ uint32_t hist[PROBE_MAX_WALK];
    const int lim = (int)st[3];
    const int e0 = min(a.w0, lim), e1 = min(a.w1, lim), nw = e1 - e0;
    const int64_t *pre = a.pre + (int64_t)b * (a.walk + 1);
    const int64_t *co = a.coarse + (int64_t)b * a.walk;
    for (int i = tid; i <= nw; i += 256) spre[i] = pre[e0 + i];
    for (int i = tid; i < nw; i += 256) {
        sbase[i] = a.list_off[co[e0 + i]];
        hist[i] = 0u;
    }
    __syncthreads();
    const PredDev p = a.pred;
    const int64_t r0 = spre[0], r1 = spre[nw];
    constexpr int R = PROBE_COUNT_R;
    for (int64_t c0 = r0 + (int64_t)g * (256 * R); c0 < r1; c0 += (int64_t)a.gc * (256 * R)) {
        int32_t id[R];
        int li[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t m = c0 + j * 256 + tid;
            li[j] = -1;
            id[j] = 0;
            if (m < r1) {
                li[j] = walk_find(spre, 0, nw, m);
                id[j] = (int32_t)(sbase[li[j]] + (m - spre[li[j]]));  // position in partition order
            }
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const bool q = li[j] >= 0 && pred_eval(p, a.attr, a.an, id[j]);
            const int up = __shfl_up(li[j], 1);
            const bool head = li[j] >= 0 && (lane == 0 || up != li[j]);
            const uint64_t heads = __ballot(head), qb = __ballot(q);
            if (head) {
                const uint64_t later = heads & ~((2ull << lane) - 1ull);  // heads after this lane
                const uint64_t upto = later ? (later & (~later + 1ull)) - 1ull : ~0ull;
                const uint32_t n = (uint32_t)__popcll(qb & upto & ~((1ull << lane) - 1ull));
                if (n != 0u) atomicAdd(&hist[li[j]], n);
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < nw; i += 256)
        if (hist[i] != 0u) atomicAdd(&a.cnt[(int64_t)b * a.walk + e0 + i], hist[i]);
}

// Thread b, after a counting round (the kernel boundary orders the counts
// before it): the walk's rules over the counts so far.  The first nprobe
// partitions are visited; past them the walk goes on only while fewer than
// min_cand rows qualified, and never past the limit.  A query whose walk is
// decided records the partitions visited, and later rounds skip it.
__global__ __launch_bounds__(256) void probe_decide_kernel(ProbeArgs a) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= a.B) return;
    int64_t *st = a.state + 4 * (int64_t)b;
    if (st[0] == 0) return;
    const int64_t lim = st[3];
    int64_t i = st[1], got = st[2];
    bool decided = false;
    for (;;) {
        if (i >= lim || (i >= a.nprobe && got >= a.min_cand)) {
            decided = true;
            break;
        }
        if (i >= a.w1) break;  // counted so far: the rules need the next round
        got += a.cnt[(int64_t)b * a.walk + i];
        ++i;
    }
    st[1] = i;
    st[2] = got;
    if (decided) {
        st[0] = 0;
        if (a.taken) a.taken[b] = (int32_t)i;
    }
}

// LDS layout of the scoring workgroup (R rows per thread in a step; the
// candidate list holds one step's rows and fewer than 256 left over).
struct ScoreLds {
    size_t qd, keys, pre, base, list, lcount, total;
};
__host__ __device__ inline ScoreLds score_lds(int dp, int k, int R) {
    const int Kp = next_pow2(k), M = next_pow2(Kp + 256);
    ScoreLds L;
    L.qd = 4 * (size_t)X64_WAVE_LDS;
    L.keys = L.qd + (size_t)dp * 8;
    L.pre = L.keys + (size_t)M * 16 + 32;  // keys, the threshold key, the count
    L.base = L.pre + 8 * (size_t)(PROBE_MAX_WALK + 2);
    L.list = L.base + 8 * (size_t)PROBE_MAX_WALK;
    L.lcount = L.list + 4 * (size_t)(256 * R + 256);
    L.total = L.lcount + 16;
    return L;
}

// Task (g, b): steps g, g + gs, ... of 256 R rows of the partitions query b
// visits (read in partition order from the index's copies of the rows and
// predicate columns).  Each step appends the rows that satisfy the predicate
// to a candidate list in LDS; whenever 256 or more are waiting (and after the
// task's last step, all of them) their exact FP64 distances are taken (64
// rows per wave, one per lane) and the k smallest (distance, id) keys over
// the task are kept.  A query's candidates are all qualifying rows of its
// visited partitions, so the k smallest keys over its tasks do not depend on
// how the rows are split.
template <int STORE, int METRIC, int R>
__global__ __launch_bounds__(256) void probe_score_kernel(ProbeArgs a) {
    constexpr int STEP = 256 * R;
    const int g = blockIdx.x, b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int T = (int)a.state[4 * (int64_t)b + 1];
    const int64_t *pre = a.pre + (int64_t)b * (a.walk + 1);
    const int64_t rows = pre[T];
    const int64_t nst = (rows + STEP - 1) / STEP;
    if (g >= nst) return;  // the merge reads the first min(gs, steps) tasks' keys (uniform)
    extern __shared__ __align__(16) unsigned char smem[];
    const ScoreLds L = score_lds(a.dp, a.k, R);
    x64_u32x4 *stage = (x64_u32x4 *)(smem + (size_t)wave * X64_WAVE_LDS);
    double *qd = (double *)(smem + L.qd);
    const int Kp = next_pow2(a.k);
    const int M = next_pow2(Kp + 256);
    Key128 *keys = (Key128 *)(smem + L.keys);
    Key128 *thr = keys + M;
    int *cnt = (int *)(thr + 1);
    int64_t *spre = (int64_t *)(smem + L.pre);
    int64_t *sbase = (int64_t *)(smem + L.base);
    int32_t *list = (int32_t *)(smem + L.list);
    int *lcount = (int *)(smem + L.lcount);
    const int64_t *co = a.coarse + (int64_t)b * a.walk;
    for (int j = tid; j < a.dp; j += 256) qd[j] = j < a.d ? (double)a.q[(int64_t)b * a.d + j] : 0.0;
    for (int i = tid; i <= T; i += 256) spre[i] = pre[i];
    for (int i = tid; i < T; i += 256) sbase[i] = a.list_off[co[i]];
    if (tid == 0) *lcount = 0;
    TopkLds<Key128> tk{keys, cnt, thr, 1, a.k, Kp, M - Kp};
    tk.init(tid, 256);  // (includes a barrier)
    const PredDev p = a.pred;
    for (int64_t c = g; c < nst; c += a.gs) {
        const int64_t m0 = c * STEP;
        int32_t id[R];
        bool in[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t m = m0 + j * 256 + tid;
            in[j] = m < rows;
            id[j] = 0;
            if (in[j]) {
                const int i = walk_find(spre, 0, T, m);
                id[j] = (int32_t)(sbase[i] + (m - spre[i]));  // position in partition order
            }
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const bool q = in[j] && pred_eval(p, a.attr, a.an, id[j]);
            const uint64_t bal = __ballot(q);
            int base = 0;
            if (lane == 0 && bal != 0ull) base = atomicAdd(lcount, __popcll(bal));
            base = __shfl(base, 0);
            if (q) list[base + __popcll(bal & ((1ull << lane) - 1ull))] = id[j];
        }
        __syncthreads();
        const int nl = *lcount;
        __syncthreads();  // every thread has read the count
        const bool last = c + a.gs >= nst;
        if (nl >= 256 || last) {
            const int nfull = last ? nl : (nl & ~255);
            for (int t0 = 0; t0 < nfull; t0 += 256) {
                const int ci = t0 + tid;
                const bool has = ci < nfull;
                const int pos = has ? list[ci] : 0;
                if (__ballot(has) != 0) {  // (wave-uniform)
                    const double dv = exact64_wave<STORE, METRIC>(a.rows, a.scale, pos, has, qd, a.dp, stage);
                    if (has) tk.push(0, Key128{ord64(dv), (uint64_t)(uint32_t)a.ids[pos]});
                }
                __syncthreads();
                if (tk.need_flush(256)) flush_sized<Key128, 256>(tk, tid);
            }
            // the fewer than 256 rows left over move to the front of the list
            const int rem = nl - nfull;
            const int v = tid < rem ? list[nfull + tid] : 0;
            __syncthreads();
            if (tid < rem) list[tid] = v;
            if (tid == 0) *lcount = rem;
            __syncthreads();
        }
    }
    if (tk.need_flush(M - Kp)) flush_sized<Key128, 256>(tk, tid);
    uint64_t *dst = a.part + ((int64_t)b * a.gs + g) * a.k * 2;
    for (int i = tid; i < a.k; i += 256) {
        dst[2 * i] = keys[i].hi;
        dst[2 * i + 1] = keys[i].lo;
    }
}

// The k smallest keys of F2 (a power of two) ascending lists of k keys in
// LDS (list l at L + l k), into list 0: pairwise merges, each list truncated
// to its k smallest (the k smallest of a union are among the k smallest of
// each part); output t of a pair is found by a binary search along the merge
// path (how many of the first t outputs come from the first list).
constexpr int PROBE_MERGE_KEYS = 4096;  // lists x k held in LDS at once
__device__ void merge_sorted_lists(Key128 *L, int F2, int k) {
    constexpr int MAXO = PROBE_MERGE_KEYS / 2 / 256;  // outputs per thread and level
    const int tid = threadIdx.x;
    for (int w = 1; w < F2; w <<= 1) {
        const int tasks = (F2 / (2 * w)) * k;
        Key128 out[MAXO];
#pragma unroll
        for (int r = 0; r < MAXO; ++r) {
            const int task = tid + r * 256;
            if (task >= tasks) continue;
            const int pr = task / k, t = task - pr * k;
            const Key128 *A = L + (size_t)(2 * w * pr) * k, *Bl = A + (size_t)w * k;
            // lo = the j in [0, t] where A[j] < B[t - 1 - j] stops holding:
            // a fixed number of halving steps (t < k <= 256), so that the
            // searches of a thread's outputs run side by side
            int lo = 0;
#pragma unroll
            for (int step = 256; step > 0; step >>= 1) {
                const int j = lo + step - 1;
                if (j < t && KeyOps<Key128>::less(A[j], Bl[t - 1 - j])) lo += step;
            }
            const Key128 x = A[lo], y = Bl[t - lo];
            out[r] = KeyOps<Key128>::less(y, x) ? y : x;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < MAXO; ++r) {
            const int task = tid + r * 256;
            if (task >= tasks) continue;
            const int pr = task / k, t = task - pr * k;
            L[(size_t)(2 * w * pr) * k + t] = out[r];
        }
        __syncthreads();
    }
}

// Workgroup (j, b): the k smallest keys of query b's partial lists
// [j * fan, (j + 1) * fan) (level 0: the scoring tasks' lists; level 1: the
// merged groups of PROBE_FAN of them), into dst, or, when dst is null (one
// workgroup per query over all lists), into the outputs.  Every list is
// ascending (a running list's final state); when they fit in LDS together
// they are merged pairwise (merge_sorted_lists), otherwise their keys are
// offered to a running list, four per thread at a time.
__global__ __launch_bounds__(256) void probe_merge_kernel(ProbeArgs a, const uint64_t *src, int src_stride,
                                                          int level, int fan, uint64_t *dst, int dst_stride) {
    const int j = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    const int T = (int)a.state[4 * (int64_t)b + 1];
    const int64_t rows = a.pre[(int64_t)b * (a.walk + 1) + T];
    const int64_t used0 = min((int64_t)a.gs, (rows + a.srows - 1) / a.srows);
    const int n_in = (int)(level == 0 ? used0 : (used0 + PROBE_FAN - 1) / PROBE_FAN);
    const int l0 = dst ? j * fan : 0, l1 = dst ? min(n_in, (j + 1) * fan) : n_in;
    if (dst && l0 >= l1) return;  // (uniform)
    extern __shared__ __align__(16) unsigned char smem[];
    Key128 *keys = (Key128 *)smem;
    const uint64_t *s0 = src + ((int64_t)b * src_stride + l0) * a.k * 2;
    const int F = max(0, l1 - l0), F2 = next_pow2(max(F, 1));
    if (F2 * a.k <= PROBE_MERGE_KEYS && a.k <= 256) {
        for (int p = tid; p < F2 * a.k; p += 256)
            keys[p] = p < F * a.k ? Key128{s0[2 * p], s0[2 * p + 1]} : Key128{KEY_INF, KEY_INF};
        __syncthreads();
        merge_sorted_lists(keys, F2, a.k);
    } else {
        const int Kp = next_pow2(a.k);
        const int M = next_pow2(Kp + 256);
        Key128 *thr = keys + M;
        int *cnt = (int *)(thr + 1);
        TopkLds<Key128> tk{keys, cnt, thr, 1, a.k, Kp, M - Kp};
        tk.init(tid, 256);
        const int64_t tot = (int64_t)F * a.k;
        constexpr int RM = 4;
        for (int64_t p0 = 0; p0 < tot; p0 += 256 * RM) {
            Key128 kk[RM];
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                const int64_t pi = p0 + r * 256 + tid;
                kk[r] = pi < tot ? Key128{s0[2 * pi], s0[2 * pi + 1]} : Key128{KEY_INF, KEY_INF};
            }
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                if (kk[r].hi != KEY_INF || kk[r].lo != KEY_INF) tk.push(0, kk[r]);
                __syncthreads();
                if (tk.need_flush(256)) tk.flush(tid, 256);
            }
        }
        if (tk.need_flush(M - Kp)) tk.flush(tid, 256);
    }
    if (dst) {
        uint64_t *o = dst + ((int64_t)b * dst_stride + j) * a.k * 2;
        for (int i = tid; i < a.k; i += 256) {
            o[2 * i] = keys[i].hi;
            o[2 * i + 1] = keys[i].lo;
        }
        return;
    }
    for (int i = tid; i < a.k; i += 256) {
        const int64_t o = (int64_t)b * a.k + i;
        const Key128 kk = keys[i];
        if (!(kk.hi == KEY_INF && kk.lo == KEY_INF)) {
            a.out_idx[o] = (int64_t)kk.lo;
            a.out_dist[o] = (float)unord64(kk.hi);
        } else {
            a.out_idx[o] = -1;
            a.out_dist[o] = __int_as_float(0x7f800000);
        }
    }
}

// Thread per 16-byte slot of the copied rows: slot s of position m = s / spr.
__global__ __launch_bounds__(256) void list_rows_kernel(const int32_t *__restrict__ ids, int64_t n,
                                                        const uint4 *__restrict__ rows, int spr,
                                                        uint4 *__restrict__ rows_p) {
    const int64_t total = n * spr;
    for (int64_t sl = (int64_t)blockIdx.x * 256 + threadIdx.x; sl < total; sl += (int64_t)gridDim.x * 256) {
        const int64_t m = sl / spr;
        rows_p[sl] = rows[(int64_t)ids[m] * spr + (sl - m * spr)];
    }
}

// Thread per position: its row's FP8 scale and predicate values.
__global__ __launch_bounds__(256) void list_attr_kernel(const int32_t *__restrict__ ids, int64_t n,
                                                        const float *__restrict__ scale,
                                                        const int32_t *__restrict__ attr, int n_attr, int64_t an,
                                                        float *__restrict__ scale_p, int32_t *__restrict__ attr_p) {
    for (int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x; m < n; m += (int64_t)gridDim.x * 256) {
        const int64_t r = ids[m];
        if (scale) scale_p[m] = scale[r];
        for (int c = 0; c < n_attr; ++c) attr_p[(int64_t)c * n + m] = attr[(int64_t)c * an + r];
    }
}

// Initial centroids: the rows at positions floor(i n / nlist).
__global__ __launch_bounds__(256) void centroid_init_kernel(const float *__restrict__ x32, int64_t n, int nlist,
                                                            int d, float *__restrict__ cent) {
    const int c = blockIdx.x;
    const int64_t r = (int64_t)c * n / nlist;
    for (int j = threadIdx.x; j < d; j += 256) cent[(int64_t)c * d + j] = x32[r * d + j];
}

template <int STORE, int METRIC, int R>
hipError_t probe_score_r(const ProbeArgs &a, hipStream_t s) {
    const size_t lds = score_lds(a.dp, a.k, R).total;
    ensure_dyn_lds((const void *)probe_score_kernel<STORE, METRIC, R>, lds);
    probe_score_kernel<STORE, METRIC, R><<<dim3(a.gs, a.B), 256, lds, s>>>(a);
    return hipGetLastError();
}

template <int STORE, int METRIC>
hipError_t probe_score_t(const ProbeArgs &a, hipStream_t s) {
    return a.srows == 256 * 16 ? probe_score_r<STORE, METRIC, 16>(a, s) : probe_score_r<STORE, METRIC, 2>(a, s);
}

}  // namespace

hipError_t launch_index_lists(const int64_t *assign, int64_t n, int nlist, uint32_t *cnt, int64_t *size,
                              int64_t *off, int32_t *ids, hipStream_t s) {
    const int nblk = (int)((n + PROBE_LIST_BLOCK - 1) / PROBE_LIST_BLOCK);
    const size_t lds = (size_t)nlist * 4;
    ensure_dyn_lds((const void *)list_count_kernel, lds);
    ensure_dyn_lds((const void *)list_place_kernel, lds);
    list_count_kernel<<<nblk, 256, lds, s>>>(assign, n, nlist, cnt);
    list_blocks_kernel<<<(nlist + 255) / 256, 256, 0, s>>>(cnt, nblk, nlist, size);
    list_offsets_kernel<<<1, 1024, 0, s>>>(size, nlist, off);
    list_place_kernel<<<nblk, 64, lds, s>>>(assign, n, nlist, cnt, off, ids);
    return hipGetLastError();
}

hipError_t launch_list_gather(const int32_t *ids, int64_t n, const void *rows, int64_t row_bytes,
                              const float *scale, const int32_t *attr, int n_attr, int64_t an, void *rows_p,
                              float *scale_p, int32_t *attr_p, hipStream_t s) {
    const int spr = (int)(row_bytes / 16);
    const int64_t slots = n * spr;
    const int g1 = (int)std::min<int64_t>((slots + 255) / 256, 65536);
    list_rows_kernel<<<std::max(g1, 1), 256, 0, s>>>(ids, n, (const uint4 *)rows, spr, (uint4 *)rows_p);
    const int g2 = (int)std::min<int64_t>((n + 255) / 256, 65536);
    list_attr_kernel<<<std::max(g2, 1), 256, 0, s>>>(ids, n, scale, attr, n_attr, an, scale_p, attr_p);
    return hipGetLastError();
}

hipError_t launch_centroid_init(const float *x32, int64_t n, int nlist, int d, float *cent, hipStream_t s) {
    centroid_init_kernel<<<nlist, 256, 0, s>>>(x32, n, nlist, d, cent);
    return hipGetLastError();
}

hipError_t launch_centroid_mean(const float *x32, int nlist, int d, const int64_t *off, const int32_t *ids,
                                float *cent, hipStream_t s) {
    centroid_mean_kernel<<<nlist, 256, 0, s>>>(x32, d, off, ids, cent);
    return hipGetLastError();
}

hipError_t launch_probe(const ProbeArgs &a, hipStream_t s) {
    if (a.nlist <= PROBE_SORT_MAX) {
        const size_t ldsd = 4 * X64_WAVE_LDS + (size_t)a.cdp * 8;
        ensure_dyn_lds((const void *)probe_cdist_kernel, ldsd);
        probe_cdist_kernel<<<dim3((a.nlist + 255) / 256, a.B), 256, ldsd, s>>>(a);
        const int R = std::max(1, next_pow2(a.nlist) / 256);
        const size_t lds = (size_t)256 * R * sizeof(Key128);
        auto launch_sort = [&](auto kern) {
            ensure_dyn_lds((const void *)kern, lds);
            kern<<<a.B, 256, lds, s>>>(a);
        };
        switch (R) {
        case 1: launch_sort(probe_sort_kernel<1>); break;
        case 2: launch_sort(probe_sort_kernel<2>); break;
        case 4: launch_sort(probe_sort_kernel<4>); break;
        case 8: launch_sort(probe_sort_kernel<8>); break;
        default: launch_sort(probe_sort_kernel<16>);
        }
    } else {
        const int Kp = next_pow2(a.walk), M = next_pow2(Kp + 256);
        const size_t lds = 4 * X64_WAVE_LDS + (size_t)a.cdp * 8 + (size_t)M * sizeof(Key128) + sizeof(Key128) + 16;
        ensure_dyn_lds((const void *)probe_coarse_kernel, lds);
        probe_coarse_kernel<<<a.B, 256, lds, s>>>(a);
    }
    probe_prefix_kernel<<<a.B, PROBE_MAX_WALK, 0, s>>>(a);
    // Rounds of the walk: positions [0, nprobe), then windows growing fourfold
    // up to the walk's end (at most 16 queries: the rest of the walk in one
    // window, since each round costs two launches and a few queries' rows
    // are few); a query leaves the rounds once its walk is decided.
    ProbeArgs r = a;
    r.w0 = 0;
    r.w1 = std::min(a.nprobe, a.walk);
    for (;;) {
        probe_count_kernel<<<dim3(a.gc, a.B), 256, 0, s>>>(r);
        probe_decide_kernel<<<(a.B + 255) / 256, 256, 0, s>>>(r);
        if (r.w1 >= a.walk) break;
        r.w0 = r.w1;
        r.w1 = a.B <= 16 ? a.walk : std::min(a.walk, 4 * r.w1);
    }
    hipError_t e;
    if (a.metric == VRS_L2SQ) {
        e = probe_score_t<VRS_F32, VRS_L2SQ>(a, s);  // float32 tables only
    } else {
        switch (a.store) {
        case VRS_F32: e = probe_score_t<VRS_F32, VRS_IP>(a, s); break;
        case VRS_BF16: e = probe_score_t<VRS_BF16, VRS_IP>(a, s); break;
        default: e = probe_score_t<VRS_FP8E4M3, VRS_IP>(a, s);
        }
    }
    if (e != hipSuccess) return e;
    const int Kp = next_pow2(a.k), M = next_pow2(Kp + 256);
    const size_t lds = std::max((size_t)M * sizeof(Key128) + sizeof(Key128) + 16,
                                (size_t)PROBE_MERGE_KEYS * sizeof(Key128));
    ensure_dyn_lds((const void *)probe_merge_kernel, lds);
    if (a.part2) {  // groups of PROBE_FAN lists first, then one list per query
        const int g2 = (a.gs + PROBE_FAN - 1) / PROBE_FAN;
        probe_merge_kernel<<<dim3(g2, a.B), 256, lds, s>>>(a, a.part, a.gs, 0, PROBE_FAN, a.part2, g2);
        probe_merge_kernel<<<dim3(1, a.B), 256, lds, s>>>(a, a.part2, g2, 1, 0, nullptr, 0);
    } else {
        probe_merge_kernel<<<dim3(1, a.B), 256, lds, s>>>(a, a.part, a.gs, 0, 0, nullptr, 0);
    }
    return hipGetLastError();
}

}  // namespace vrs
