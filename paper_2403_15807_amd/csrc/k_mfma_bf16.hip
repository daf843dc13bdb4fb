// k_mfma_bf16.hip -- MFMA screening for bfloat16 and FP8 (e4m3fn + row
// scale) tables, inner-product metric: the batched tensor formulation of
// Section 3.1 on low-precision storage.
//
// Q X^T runs on v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  Every
// query is split as q = q_hi + q_lo (two bfloat16 parts, |q - q_hi - q_lo|
// <= 2^-16 |q|) and both parts are multiplied against the same stored row,
// into separate accumulators; FP8 rows are widened to bfloat16 exactly while
// they are staged into LDS, and the row scale is applied to the finished sum.
// The screening distance therefore differs from the exact one by less than
// (gamma_dp + 2^-16 + ...) |q| max|x|, which the rerank's certificate uses.
//
// Workgroup = 8 waves x 32 queries (two 16-query MFMA blocks per wave) = 256
// queries against one chunk of rows, rows in tiles of 128, coordinates in
// chunks of 128 (or 64 where 128 does not divide the padded dimension, and
// in the persistent form); a batch of up to 256 queries reads every row
// once, and one such workgroup fills a CU.  Only the rows go through LDS
// (double-buffered: the next chunk's loads are in flight while the current
// one is multiplied, one barrier per chunk); the query parts are read
// straight into registers from a fragment-ordered copy made by the query
// preparation (one 1 KB load per wave and operand), one k-step ahead, in
// two register sets that alternate by k-step.  Every 16-row B fragment read
// from LDS feeds four MFMAs (two query blocks x hi/lo).  Top-k state is
// wave-private as in the float32 kernel.
#include "internal.h"
#include "wave_topk.h"

namespace vrs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));

constexpr int QW = 32;          // queries per wave
constexpr int NWAVE = 8;        // waves per workgroup
constexpr int NT = 64 * NWAVE;  // threads per workgroup
constexpr int QM = NWAVE * QW;  // queries per workgroup
constexpr int BR = 128;         // rows per tile
constexpr int NB = BR / 16;     // 16-row MFMA blocks per tile
// KC = coordinates per chunk (one workgroup barrier each): 128 (four
// k-steps of 32) when it divides the padded dimension, else 64; LDS rows are
// KC + 8 bfloat16 long (144 or 272 bytes: the 16 rows of a B fragment start
// on distinct bank quads)
constexpr int kc_for(int dp) { return dp % 128 == 0 ? 128 : 64; }
constexpr int SLOTS = 3;        // rotating row-record slots

// An e4m3fn code's value as an f32: its 7 magnitude bits placed as the top
// of an f32 exponent and mantissa field, times 2^(127-7) (exact for normal
// codes, and for subnormal ones since FP32 denormals are kept).  Every e4m3
// value has at most 4 significant bits, so its f32 has a zero low half and
// the high half is the exact bfloat16.
__device__ __forceinline__ uint32_t e4m3_f32_bits(uint32_t c) {
    return __float_as_uint(__uint_as_float((c & 0x7fu) << 20) * 0x1p120f) | ((c & 0x80u) << 24);
}

// 4 e4m3fn codes -> 4 bfloat16 (exact), packed in two 32-bit words.
__device__ __forceinline__ uint2 e4m3x4_to_bf16x4(uint32_t w) {
    const uint32_t f0 = e4m3_f32_bits(w & 0xffu), f1 = e4m3_f32_bits((w >> 8) & 0xffu);
    const uint32_t f2 = e4m3_f32_bits((w >> 16) & 0xffu), f3 = e4m3_f32_bits(w >> 24);
    return make_uint2((f0 >> 16) | (f1 & 0xffff0000u), (f2 >> 16) | (f3 & 0xffff0000u));
}

__device__ __forceinline__ bf8v as_bf8(const uint4 &u) {
    bf8v v;
    __builtin_memcpy(&v, &u, 16);
    return v;
}

struct Lds {
    uint16_t *xs;      // [2][BR][KC + 8]
    int *rid;          // [SLOTS][BR]
    int *rok;          // [SLOTS][BR] row exists (and, shared predicate, qualifies)
    float *rsc;        // [SLOTS][BR] FP8 row scale
    uint32_t *pm;      // [SLOTS][BR][QM/32] per-query predicates: query q qualifies row r
    int *cnt;          // [QM] keys in the append buffer
    int *fill;         // [QM] keys in the list (its first entries)
    uint64_t *thr;     // [QM]
    QRange *qrg;       // [QM] per-query predicates (range form)
};

template <int KC>
__device__ __forceinline__ Lds carve(unsigned char *smem) {
    Lds L;
    L.xs = (uint16_t *)smem;
    L.rid = (int *)(L.xs + 2 * BR * (KC + 8));
    L.rok = L.rid + SLOTS * BR;
    L.rsc = (float *)(L.rok + SLOTS * BR);
    L.pm = (uint32_t *)(L.rsc + SLOTS * BR);
    L.cnt = (int *)(L.pm + SLOTS * BR * (QM / 32));
    L.fill = L.cnt + QM;
    L.thr = (uint64_t *)(L.fill + QM);
    L.qrg = (QRange *)(L.thr + QM);
    return L;
}

// One work item: queries [q0, q0 + QM) (of Bq) against row chunk `chunk` of
// `nchunks`; its lists are (query, chunk) lists of the partials.
template <int STORE, bool GATHER, bool BATCHED, int E, int KC>
__device__ __forceinline__ void bf16_tile(const ScreenArgs &a, const int chunk, const int nchunks,
                                          const int q0, const int Bq, unsigned char *smem) {
    // 16-byte row loads per thread per chunk (BR rows x KC coordinates over NT threads)
    constexpr int LDK = KC + 8;
    constexpr int TPR = KC * (STORE == VRS_BF16 ? 2 : 1) / 16;  // threads per row of a chunk
    constexpr int XLD = BR * TPR / NT;
    static_assert(XLD >= 1 && XLD * NT == BR * TPR, "a chunk must give every thread the same loads");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int dp = a.dp;
    const int nkc = dp / KC, nks = dp / 32;
    const Lds L = carve<KC>(smem);

    const int K = a.K, CBq = a.CB;
    if (tid < QM) {
        L.cnt[tid] = 0;
        L.fill[tid] = 0;
        // start from the best bound any chunk (or a first pass) has published
        L.thr[tid] = q0 + tid < Bq
                         ? __atomic_load_n((const unsigned long long *)(a.gthr + q0 + tid), __ATOMIC_RELAXED)
                         : KEY_INF;
        if (BATCHED) {
            PredDev p{-1, {0}, {0}, {0}};
            if (q0 + tid < Bq) p = a.preds[q0 + tid];
            L.qrg[tid] = range_form(q0 + tid, p);
        }
    }
    __syncthreads();  // per-query state is written by other waves than its owner's

    const int64_t total = GATHER ? *a.sel_count : a.n;
    int64_t per = (total + nchunks - 1) / nchunks;
    per = (per + BR - 1) / BR * BR;
    int64_t c0 = (int64_t)chunk * per;
    int64_t c1 = min(total, c0 + per);
    pass_range(a, c0, c1, BR, total, nchunks);
    const int ntile = c1 > c0 ? (int)((c1 - c0 + BR - 1) / BR) : 0;
    const int EB = STORE == VRS_BF16 ? 2 : 1;
    const char *X = (const char *)a.rows;
    const int64_t row_bytes = (int64_t)dp * EB;

    // query fragments of this wave: blocks qb0, qb0 + 1 (16 queries each)
    const int qb0 = (q0 + wave * QW) >> 4;
    const int nqb = (a.B + 15) >> 4;
    const uint4 *QF = (const uint4 *)a.qhl;
    // (a block past the batch reads the last one: its results are never used)
    auto loadA = [&](int ks, uint4 (&A)[2][2]) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int hl = 0; hl < 2; ++hl)
                A[b][hl] = QF[((int64_t)(min(qb0 + b, nqb - 1) * nks + ks) * 2 + hl) * 64 + lane];
    };

    // per-row record of tile t: thread r < BR writes row r's id, validity
    // and scale; with per-query predicates every thread also evaluates half
    // of the workgroup's queries on row tid % BR (one bit per pair)
    auto rowinfo = [&](int t) {
        const int slot = t % SLOTS;
        const int r = tid & (BR - 1);
        const int64_t pos = c0 + (int64_t)t * BR + r;
        bool ok = pos < c1;
        const int64_t row = ok ? (GATHER ? (int64_t)a.sel_ids[pos] : pos) : 0;
        if (tid < BR) {
            bool okp = ok;
            if (okp && !GATHER && !BATCHED) okp = pred_eval(a.pred, a.attr, a.an, row);
            L.rid[slot * BR + r] = (int)row;
            L.rok[slot * BR + r] = okp;
            L.rsc[slot * BR + r] = (STORE == VRS_FP8E4M3 && okp) ? a.scale[row] : 1.0f;
        }
        if (BATCHED) {
            const int h = tid / BR;  // queries [64 h, 64 h + 64)
            const int32_t v0 = (ok && a.n_attr > 0) ? a.attr[row] : 0;
            const int32_t v1 = (ok && a.n_attr > 1) ? a.attr[a.an + row] : 0;
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                uint32_t bits = 0;
                for (int j = 0; j < 32; ++j) {
                    const int q = h * 64 + w * 32 + j;
                    const QRange &g = L.qrg[q];
                    bool in;
                    if (g.kind == 0)
                        in = ((uint32_t)(v0 - g.lo0) <= g.span0) & ((uint32_t)(v1 - g.lo1) <= g.span1);
                    else if (g.kind == 1)
                        in = ok && pred_eval(a.preds[q0 + q], a.attr, a.an, row);
                    else
                        in = false;
                    bits |= (uint32_t)in << j;
                }
                L.pm[(slot * BR + r) * (QM / 32) + h * 2 + w] = ok ? bits : 0u;
            }
        }
    };
    uint4 xr[XLD];
    uint32_t xm[XLD];
    auto issue = [&](int c) {  // global loads of chunk c (tile c / nkc) into registers
        const int t = c / nkc, kc = c - t * nkc, slot = t % SLOTS;
        int rr[XLD];
#pragma unroll
        for (int i = 0; i < XLD; ++i) {
            const int r = (tid + NT * i) / TPR;
            rr[i] = L.rid[slot * BR + r];
            xm[i] = 0u - (uint32_t)(L.rok[slot * BR + r] != 0);
        }
        // every row id is a valid row (rows past the chunk read row 0), so
        // the loads are unconditional; unwanted rows are zeroed at commit
#pragma unroll
        for (int i = 0; i < XLD; ++i) {
            const int cc = (tid + NT * i) % TPR;
            xr[i] = *(const uint4 *)(X + (int64_t)rr[i] * row_bytes + kc * KC * EB + cc * 16);
        }
    };
    auto commit = [&](int buf) {
        uint16_t *xb = L.xs + buf * BR * LDK;
#pragma unroll
        for (int i = 0; i < XLD; ++i) {
            xr[i] = make_uint4(xr[i].x & xm[i], xr[i].y & xm[i], xr[i].z & xm[i], xr[i].w & xm[i]);
            const int idx = tid + NT * i;
            if (STORE == VRS_BF16) {
                *(uint4 *)(xb + (idx / TPR) * LDK + (idx % TPR) * 8) = xr[i];
            } else {
                uint16_t *d = xb + (idx / TPR) * LDK + (idx % TPR) * 16;
                const uint2 p0 = e4m3x4_to_bf16x4(xr[i].x), p1 = e4m3x4_to_bf16x4(xr[i].y);
                const uint2 p2 = e4m3x4_to_bf16x4(xr[i].z), p3 = e4m3x4_to_bf16x4(xr[i].w);
                *(uint4 *)d = make_uint4(p0.x, p0.y, p1.x, p1.y);
                *(uint4 *)(d + 8) = make_uint4(p2.x, p2.y, p3.x, p3.y);
            }
        }
    };

    const int nch = ntile * nkc;
    // Loads are issued in the order they are consumed (they retire in
    // order): this chunk's second k-step of query fragments, the next
    // chunk's rows, then the next chunk's first k-step of query fragments.
    // query fragments alternate between two register sets by k-step parity
    // (KC / 32 is even, so a chunk's k-step 0 always uses set 0); a chunk
    // loads its k-steps 1 and 3 before its rows and its k-step 2 and the next
    // chunk's k-step 0 after them, so no wait on query fragments waits for
    // rows issued in the same chunk except at the chunk's end
    static_assert((KC / 32) % 2 == 0, "k-steps per chunk");
    uint4 Ab[2][2][2];
    if (nch > 0) {
        rowinfo(0);
        __syncthreads();
        issue(0);
        loadA(0, Ab[0]);
    }
    int c = 0;  // running chunk index (tile t, coordinate chunk kc)
    for (int t = 0; t < ntile; ++t) {
        f4v acc[2][2][NB];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int hl = 0; hl < 2; ++hl)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[b][hl][nb] = (f4v){0.f, 0.f, 0.f, 0.f};
        for (int kc = 0; kc < nkc; ++kc, ++c) {
            const int buf = c & 1;
            commit(buf);
            if (kc == nkc - 1 && t + 1 < ntile) rowinfo(t + 1);
            __syncthreads();
            const int ks0 = kc * (KC / 32);
            const uint16_t *xb = L.xs + buf * BR * LDK + (lane & 15) * LDK + (lane >> 4) * 8;
#pragma unroll
            for (int s = 0; s < KC / 32; ++s) {
                // the next k-step's query fragments (past the chunk: the next
                // chunk's first, past the tile: k-step 0), and after the
                // second-to-last k-step's fragments, the next chunk's rows
                if (s + 1 < KC / 32) {
                    loadA(ks0 + s + 1, Ab[(s + 1) & 1]);
                } else {
                    loadA(ks0 + s + 1 < nks ? ks0 + s + 1 : 0, Ab[0]);
                }
                __builtin_amdgcn_sched_barrier(0);
                if (s == KC / 32 - 2) {
                    issue(c + 1 < nch ? c + 1 : c);  // (the last chunk reloads itself, unused)
                    __builtin_amdgcn_sched_barrier(0);
                }
                const uint4(&A)[2][2] = Ab[s & 1];
                const bf8v a00 = as_bf8(A[0][0]), a01 = as_bf8(A[0][1]);
                const bf8v a10 = as_bf8(A[1][0]), a11 = as_bf8(A[1][1]);
                bf8v Bc = *(const bf8v *)(xb + s * 32);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    // the next 16-row fragment is read while these four run
                    const bf8v Bn = *(const bf8v *)(xb + ((nb + 1) & (NB - 1)) * 16 * LDK + s * 32);
                    __builtin_amdgcn_sched_barrier(0);
                    acc[0][0][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a00, Bc, acc[0][0][nb], 0, 0, 0);
                    acc[0][1][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a01, Bc, acc[0][1][nb], 0, 0, 0);
                    acc[1][0][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a10, Bc, acc[1][0][nb], 0, 0, 0);
                    acc[1][1][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a11, Bc, acc[1][1][nb], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    Bc = Bn;
                }
            }
        }

        // ---- epilogue of tile t: lane holds, per query block b, queries
        // 32w + 16b + 4(lane/16) + i and rows 16nb + lane%16
        const int slot = t % SLOTS;
        if ((t & 7) == 7 && lane < QW) {
            const int qa = q0 + wave * QW + lane;
            if (qa < Bq) {
                const uint64_t g = __atomic_load_n((const unsigned long long *)(a.gthr + qa), __ATOMIC_RELAXED);
                if (g < L.thr[wave * QW + lane]) L.thr[wave * QW + lane] = g;
            }
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int qb = wave * QW + 16 * b + 4 * (lane >> 4);
            uint64_t th[4];
            float thf[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                th[i] = L.thr[qb + i];
                thf[i] = key_dist(th[i]);
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int r = slot * BR + nb * 16 + (lane & 15);
                if (!L.rok[r]) continue;
                const int row = L.rid[r];
                const float sc = L.rsc[r];
                const uint32_t pmw = BATCHED ? L.pm[r * (QM / 32) + (qb >> 5)] >> (qb & 31) : 0xfu;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int q = qb + i, qa = q0 + q;
                    if (qa >= Bq || !((pmw >> i) & 1u)) continue;
                    const float dot = acc[b][0][nb][i] + acc[b][1][nb][i];
                    const float dist = STORE == VRS_FP8E4M3 ? -(sc * dot) : -dot;
                    if (!(dist <= thf[i])) continue;
                    const uint64_t key = make_key(dist, (uint32_t)row);
                    if (key < th[i]) {
                        const int sl = atomicAdd(&L.cnt[q], 1);
                        a.cbuf[((int64_t)qa * nchunks + chunk) * CBq + sl] = key;
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        {
            const int myc = lane < QW ? L.cnt[wave * QW + lane] : 0;
            uint64_t full = __ballot(lane < QW && myc > CBq - BR);
            while (full) {
                const int j = __ffsll((long long)full) - 1;
                full &= full - 1;
                const int q = wave * QW + j, qa = q0 + q;
                const int64_t base = (int64_t)qa * nchunks + chunk;
                const int nq = L.cnt[q], fq = L.fill[q], Kq = list_len(a, qa, K);
                flush_fit<E>(a.partials + base * K, a.cbuf + base * CBq, nq, Kq, fq, &L.thr[q], a.gthr + qa);
                if (lane == 0) {
                    L.cnt[q] = 0;
                    L.fill[q] = min(Kq, fq + nq);
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    const int myc = lane < QW ? L.cnt[wave * QW + lane] : 0;
    uint64_t pend = __ballot(lane < QW && myc > 0 && q0 + wave * QW + lane < Bq);
    while (pend) {
        const int j = __ffsll((long long)pend) - 1;
        pend &= pend - 1;
        const int q = wave * QW + j, qa = q0 + q;
        const int64_t base = (int64_t)qa * nchunks + chunk;
        const int nq = L.cnt[q], fq = L.fill[q], Kq = list_len(a, qa, K);
        flush_fit<E>(a.partials + base * K, a.cbuf + base * CBq, nq, Kq, fq, &L.thr[q], a.gthr + qa);
        if (lane == 0) L.fill[q] = min(Kq, fq + nq);
    }
    // each list's key count, or (no count array) KEY_INF in the list
    // entries past its keys (the whole list length K)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    if (a.fills) {
        if (lane < QW && q0 + wave * QW + lane < Bq)
            a.fills[(int64_t)(q0 + wave * QW + lane) * nchunks + chunk] = L.fill[wave * QW + lane];
    } else {
        for (int j = 0; j < QW; ++j) {
            const int q = wave * QW + j, qa = q0 + q;
            if (qa < Bq) list_tail_inf(a.partials + ((int64_t)qa * nchunks + chunk) * K, L.fill[q], K);
        }
    }
}

// Work item of workgroup `id` in a one-dimensional grid of nchunks x nq
// items.  Workgroups go to the 8 XCDs round-robin (XCD = id mod 8); when
// nchunks is a multiple of 8, XCD x takes chunks x, x + 8, ... and, for each
// chunk, its nq query tiles one after another, so that the query tiles of a
// chunk run at the same time on one XCD and read the chunk's rows through
// its L2 once.
__device__ __forceinline__ void xcd_item(int id, int nchunks, int nq, int *chunk, int *qt) {
    if ((nchunks & 7) == 0) {
        const int x = id & 7, slot = id >> 3;
        *chunk = x + 8 * (slot / nq);
        *qt = slot - (slot / nq) * nq;
    } else {
        *chunk = id % nchunks;
        *qt = id / nchunks;
    }
}

template <int STORE, bool GATHER, bool BATCHED, int E, int KC>
__global__ __launch_bounds__(NT) void screen_mfma_bf16_kernel(ScreenArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    int chunk, qt;
    xcd_item(blockIdx.x, a.n_chunks, (a.B + QM - 1) / QM, &chunk, &qt);
    bf16_tile<STORE, GATHER, BATCHED, E, KC>(a, chunk, a.n_chunks, qt * QM, a.B, smem);
}

// Persistent form (batched uneven launch): the dense queries are positions
// [0, n_dense) and each has n_c row chunks, both decided on the device.
// Workgroup g serves the queue of XCD g % 8 (workgroups are dispatched to
// the XCDs round-robin), which holds chunks c = x (mod 8) with every query
// tile, chunk-major: the query tiles of one chunk run at the same time on
// one XCD and read its rows through the same L2.  An empty queue sends the
// workgroup to the other XCDs' queues.
template <int STORE, int E, int KC>
__global__ __launch_bounds__(NT) void screen_mfma_bf16_persistent(ScreenArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int item_s;
    const int Bq = a.bctl[BC_NDENSE], nc = a.bctl[BC_NC];
    const int ntiles = (Bq + QM - 1) / QM;
    const int per = nc / 8 * ntiles;  // items per XCD queue
    const int x = blockIdx.x & 7;
    int src = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int it = -1;
            while (src < 8) {
                const int qx = (x + src) & 7;
                const int i = atomicAdd(&a.bctl[BC_QDENSE + qx], 1);
                if (i < per) {
                    it = qx * per + i;
                    break;
                }
                ++src;
            }
            item_s = it;
        }
        __syncthreads();
        const int it = item_s;
        __syncthreads();
        if (it < 0) break;
        const int qx = it / per, i = it - qx * per;
        const int chunk = qx + 8 * (i / ntiles), qt = i - (i / ntiles) * ntiles;
        bf16_tile<STORE, false, true, E, KC>(a, chunk, nc, qt * QM, Bq, smem);
        __syncthreads();
    }
}

template <int STORE, int E, int KC>
hipError_t launch_sek(const ScreenArgs &a, hipStream_t s) {
    dim3 grid(a.n_chunks * ((a.B + QM - 1) / QM)), block(NT);
    const size_t lds = screen_mfma_bf16_lds(KC);
    if (a.preds) {
        auto k = screen_mfma_bf16_kernel<STORE, false, true, E, KC>;
        ensure_dyn_lds((const void *)k, lds);
        k<<<grid, block, lds, s>>>(a);
    } else if (a.gather) {
        auto k = screen_mfma_bf16_kernel<STORE, true, false, E, KC>;
        ensure_dyn_lds((const void *)k, lds);
        k<<<grid, block, lds, s>>>(a);
    } else {
        auto k = screen_mfma_bf16_kernel<STORE, false, false, E, KC>;
        ensure_dyn_lds((const void *)k, lds);
        k<<<grid, block, lds, s>>>(a);
    }
    return hipGetLastError();
}

template <int STORE, int E>
hipError_t launch_se(const ScreenArgs &a, hipStream_t s) {
    return kc_for(a.dp) == 128 ? launch_sek<STORE, E, 128>(a, s) : launch_sek<STORE, E, 64>(a, s);
}

template <int STORE>
hipError_t launch_s(const ScreenArgs &a, hipStream_t s) {
    switch ((a.Kp + a.CB) / 64) {
    case 4: return launch_se<STORE, 4>(a, s);
    case 8: return launch_se<STORE, 8>(a, s);
    case 16: return launch_se<STORE, 16>(a, s);
    default: return launch_se<STORE, 32>(a, s);
    }
}

template <int STORE, int E, int KC>
hipError_t launch_pek(const ScreenArgs &a, int grid, hipStream_t s) {
    const size_t lds = screen_mfma_bf16_lds(KC);
    auto k = screen_mfma_bf16_persistent<STORE, E, KC>;
    ensure_dyn_lds((const void *)k, lds);
    k<<<grid, NT, lds, s>>>(a);
    return hipGetLastError();
}

// (the persistent form keeps 64-coordinate chunks: its per-query predicate
// masks leave no registers for the wider chunk's loads, which spill)
template <int STORE, int E>
hipError_t launch_pe(const ScreenArgs &a, int grid, hipStream_t s) {
    return launch_pek<STORE, E, 64>(a, grid, s);
}

template <int STORE>
hipError_t launch_p(const ScreenArgs &a, int grid, hipStream_t s) {
    switch ((a.Kp + a.CB) / 64) {
    case 4: return launch_pe<STORE, 4>(a, grid, s);
    case 8: return launch_pe<STORE, 8>(a, grid, s);
    case 16: return launch_pe<STORE, 16>(a, grid, s);
    default: return launch_pe<STORE, 32>(a, grid, s);
    }
}

}  // namespace

size_t screen_mfma_bf16_lds(int kc) {
    return (size_t)2 * BR * (kc + 8) * 2 + (size_t)3 * SLOTS * BR * 4 + (size_t)SLOTS * BR * (QM / 32) * 4 +
           QM * 4 * 2 + QM * 8 + QM * sizeof(QRange) + 16;
}

int screen_mfma_bf16_qm() { return QM; }

// Fragment-ordered copy of the queries' bfloat16 hi/lo parts: 16-byte unit
// ((qb * (dp / 32) + ks) * 2 + hl) * 64 + lane holds query 16 qb + lane % 16,
// coordinates 32 ks + 8 (lane / 16) .. + 7 (the A operand of one
// v_mfma_f32_16x16x32_bf16); bytes for queries rounded up to 16.
size_t screen_mfma_bf16_qfrag_bytes(int B, int dp) { return (size_t)((B + 15) / 16) * 16 * dp * 2 * 2; }

bool screen_mfma_bf16_supported(int dp, vrs_dtype store, int metric, int Kp, int CB) {
    const int E = (Kp + CB) / 64;
    return (store == VRS_BF16 || store == VRS_FP8E4M3) && metric == VRS_IP && dp % 64 == 0 &&
           (E == 4 || E == 8 || E == 16 || E == 32) && (Kp + CB) == 64 * E;
}

hipError_t launch_screen_mfma_bf16(const ScreenArgs &a, hipStream_t s) {
    if (a.metric != VRS_IP) return hipErrorInvalidValue;
    return a.store == VRS_BF16 ? launch_s<VRS_BF16>(a, s) : launch_s<VRS_FP8E4M3>(a, s);
}

hipError_t launch_screen_mfma_bf16_persistent(const ScreenArgs &a, int grid, hipStream_t s) {
    if (a.metric != VRS_IP || !a.bctl || !a.preds) return hipErrorInvalidValue;
    return a.store == VRS_BF16 ? launch_p<VRS_BF16>(a, grid, s) : launch_p<VRS_FP8E4M3>(a, grid, s);
}

}  // namespace vrs
