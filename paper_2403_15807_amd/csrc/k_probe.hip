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
// Probe (after the nearest-centroid scan of the queries):
//   probe_collect: per query, the partitions in centroid order, each
//       contributing its rows that satisfy the predicate, until enough rows
//       qualified or the visited-row budget would be passed;
//   probe_score: exact FP64 distances of the collected rows (64 per wave, one
//       per lane), the k smallest (distance, id) keys of every chunk;
//   probe_merge: per query the k smallest of its chunks' keys, written out.
#include "exact64.h"

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

// Workgroup b: walk query b's partitions in centroid order.  A partition is
// skipped (and the walk ends) when some partition was already taken and
// taking it would pass cap_c visited rows; after a partition, the walk ends
// once min_cand rows qualified.  Qualifying rows are written in walk order
// (partition order, then ascending within a partition).
__global__ __launch_bounds__(256) void probe_collect_kernel(ProbeArgs a) {
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ uint32_t wc[4];
    const PredDev p = a.pred;
    const int64_t *co = a.coarse + (int64_t)b * a.nprobe;
    int32_t *cand = a.cand + (int64_t)b * a.cand_cap;
    int64_t visited = 0, got = 0;
    int taken = 0;
    for (int li = 0; li < a.nprobe; ++li) {
        const int64_t lst = co[li];
        if (lst < 0) break;
        const int64_t m0 = a.list_off[lst], m1 = a.list_off[lst + 1];
        if (taken >= 1 && visited + (m1 - m0) > a.cap_c) break;
        for (int64_t c0 = m0; c0 < m1; c0 += 256) {
            const int64_t m = c0 + tid;
            const int row = m < m1 ? a.ids[m] : 0;
            const bool q = m < m1 && pred_eval(p, a.attr, a.an, row);
            const uint64_t bal = __ballot(q);
            if (lane == 0) wc[wave] = (uint32_t)__popcll(bal);
            __syncthreads();
            uint32_t before = 0, tot = 0;
            for (int w = 0; w < 4; ++w) {
                if (w < wave) before += wc[w];
                tot += wc[w];
            }
            if (q) cand[got + before + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull))] = row;
            got += tot;
            __syncthreads();
        }
        visited += m1 - m0;
        ++taken;
        if (got >= a.min_cand) break;
    }
    if (tid == 0) {
        a.ncand[b] = (int32_t)got;
        if (a.taken) a.taken[b] = taken;
    }
}

// Task (chunk, b): the k smallest exact keys of candidates [chunk * PROBE_CHUNK,
// +PROBE_CHUNK) of query b.
template <int STORE, int METRIC>
__global__ __launch_bounds__(256) void probe_score_kernel(ProbeArgs a) {
    const int chunk = blockIdx.x, b = blockIdx.y, tid = threadIdx.x, wave = tid >> 6;
    const int nc = a.ncand[b];
    const int64_t c0 = (int64_t)chunk * PROBE_CHUNK, c1 = min((int64_t)nc, c0 + PROBE_CHUNK);
    uint64_t *dst = a.part + ((int64_t)b * a.nchunk + chunk) * a.k * 2;
    if (c0 >= c1) {  // no candidates here: an empty list
        for (int i = tid; i < a.k; i += 256) {
            dst[2 * i] = KEY_INF;
            dst[2 * i + 1] = KEY_INF;
        }
        return;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    x64_u32x4 *stage = (x64_u32x4 *)(smem + (size_t)wave * X64_WAVE_LDS);
    double *qd = (double *)(smem + 4 * X64_WAVE_LDS);
    const int Kp = next_pow2(a.k);
    const int M = next_pow2(Kp + 256);
    Key128 *keys = (Key128 *)(qd + a.dp);
    Key128 *thr = keys + M;
    int *cnt = (int *)(thr + 1);
    for (int j = tid; j < a.dp; j += 256) qd[j] = j < a.d ? (double)a.q[(int64_t)b * a.d + j] : 0.0;
    TopkLds<Key128> tk{keys, cnt, thr, 1, a.k, Kp, M - Kp};
    tk.init(tid, 256);  // (includes a barrier)
    const int32_t *cand = a.cand + (int64_t)b * a.cand_cap;
    for (int64_t t0 = c0; t0 < c1; t0 += 256) {
        const int64_t ci = t0 + tid;
        const bool has = ci < c1;
        const int row = has ? cand[ci] : 0;
        if (__ballot(has) != 0) {  // (wave-uniform)
            const double dv = exact64_wave<STORE, METRIC>(a.rows, a.scale, row, has, qd, a.dp, stage);
            if (has) tk.push(0, Key128{ord64(dv), (uint64_t)(uint32_t)row});
        }
        __syncthreads();
        if (tk.need_flush(256)) tk.flush(tid, 256);
    }
    if (tk.need_flush(M - Kp)) tk.flush(tid, 256);
    for (int i = tid; i < a.k; i += 256) {
        dst[2 * i] = keys[i].hi;
        dst[2 * i + 1] = keys[i].lo;
    }
}

__global__ __launch_bounds__(256) void probe_merge_kernel(ProbeArgs a) {
    const int b = blockIdx.x, tid = threadIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    const int Kp = next_pow2(a.k);
    const int M = next_pow2(Kp + 256);
    Key128 *keys = (Key128 *)smem;
    Key128 *thr = keys + M;
    int *cnt = (int *)(thr + 1);
    TopkLds<Key128> tk{keys, cnt, thr, 1, a.k, Kp, M - Kp};
    tk.init(tid, 256);
    const int used = (int)min((int64_t)a.nchunk, ((int64_t)a.ncand[b] + PROBE_CHUNK - 1) / PROBE_CHUNK);
    const uint64_t *src = a.part + (int64_t)b * a.nchunk * a.k * 2;
    const int64_t tot = (int64_t)used * a.k;
    for (int64_t p0 = 0; p0 < tot; p0 += 256) {
        const int64_t pi = p0 + tid;
        if (pi < tot) {
            const Key128 kk{src[2 * pi], src[2 * pi + 1]};
            if (kk.hi != KEY_INF || kk.lo != KEY_INF) tk.push(0, kk);
        }
        __syncthreads();
        if (tk.need_flush(256)) tk.flush(tid, 256);
    }
    if (tk.need_flush(M - Kp)) tk.flush(tid, 256);
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

// Initial centroids: the rows at positions floor(i n / nlist).
__global__ __launch_bounds__(256) void centroid_init_kernel(const float *__restrict__ x32, int64_t n, int nlist,
                                                            int d, float *__restrict__ cent) {
    const int c = blockIdx.x;
    const int64_t r = (int64_t)c * n / nlist;
    for (int j = threadIdx.x; j < d; j += 256) cent[(int64_t)c * d + j] = x32[r * d + j];
}

template <int STORE, int METRIC>
hipError_t probe_score_t(const ProbeArgs &a, hipStream_t s) {
    const int Kp = next_pow2(a.k), M = next_pow2(Kp + 256);
    const size_t lds = 4 * X64_WAVE_LDS + (size_t)a.dp * 8 + (size_t)M * sizeof(Key128) + sizeof(Key128) + 16;
    ensure_dyn_lds((const void *)probe_score_kernel<STORE, METRIC>, lds);
    probe_score_kernel<STORE, METRIC><<<dim3(a.nchunk, a.B), 256, lds, s>>>(a);
    return hipGetLastError();
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
    probe_collect_kernel<<<a.B, 256, 0, s>>>(a);
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
    probe_merge_kernel<<<a.B, 256, (size_t)M * sizeof(Key128) + sizeof(Key128) + 16, s>>>(a);
    return hipGetLastError();
}

}  // namespace vrs
