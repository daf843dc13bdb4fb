// k_mfma.hip -- MFMA screening for query batches (the N:N strategy and its
// tensor formulation, Section 3.1: a batch of queries against a batch of
// data vectors as one matrix product Q X^T), float32 tables.
//
// Workgroup = 4 waves = 64 queries (16 per wave) x one chunk of rows; for
// batches of at most 16 queries, the four waves share the 16 queries and
// split each tile's rows instead.
//   - Each wave keeps its 16 queries as MFMA A-operands in registers for the
//     whole row width (v_mfma_f32_16x16x4_f32; the coordinate order inside a
//     lane is permuted identically for queries and rows, which leaves the
//     dot products unchanged).
//   - Rows arrive in tiles of 64: every thread issues its non-temporal 16-byte
//     loads for the tile, then writes them into a padded LDS tile; rows that
//     fail the predicate (mask strategy) are neither loaded nor computed, and
//     a tile without any qualifying row is skipped.
//   - Epilogue per (query, row): distance (L2: |q|^2 + |x|^2 - 2 q.x, IP: -q.x),
//     predicate, threshold test against the query's current K-th key.
//   - The candidates of a query are produced only by the wave that owns the
//     query, so its top-k state is wave-private: an append buffer in global
//     memory (L2-resident workspace) plus the sorted list, merged by the
//     owning wave with a register bitonic sort when the buffer fills.
#include "internal.h"
#include "wave_topk.h"

namespace vrs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));

// Row loads: non-temporal when each row is read once (one query tile), plain
// when the other query tiles of the same row chunk will read it again from L2.
__device__ __forceinline__ float4 load_x(const float4 *p, int shared) {
    if (shared) return *p;
    v4u32 v = __builtin_nontemporal_load((const v4u32 *)p);
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
                       __uint_as_float(v.w));
}

constexpr int BR = 64;  // rows per tile

// MB = 16-query blocks per wave (a workgroup holds QM = 64 * MB queries); a
// B-operand read from LDS feeds MB MFMAs.  G = waves sharing one group of QW
// queries (G > 1 only with MB = 1, for batches of at most 64 / G queries):
// the group's waves split every 64-row tile between them, so that all four
// SIMDs of the CU run MFMAs for a small batch; the group's candidates are
// then merged by its first wave after a workgroup barrier.
// DP = the padded dimension, or 0 for rows wider than 256 coordinates (any
// multiple of 128, taken from the table): those are multiplied in chunks of
// 128 coordinates, each chunk staged in LDS while the next one's loads are in
// flight, with the query fragments of the chunk read from the (L2-resident)
// prepared queries; the accumulators carry over the chunks.
// One work item: queries [q0, q0 + QM) (of Bq) against row chunk `chunk` of
// `nchunks`; its lists are (query, chunk) lists of the partials.
template <int DP, int METRIC, bool GATHER, bool BATCHED, int E, int MB, int G = 1>
__device__ __forceinline__ void f32_tile(const ScreenArgs &a, const int chunk, const int nchunks,
                                         const int q0, const int Bq, unsigned char *smem) {
    static_assert(G == 1 || MB == 1, "query groups shared by several waves hold 16 queries");
    constexpr int QM = 64 * MB / G;
    constexpr int QW = 16 * MB;            // queries per wave group
    constexpr int NBW = 4 / G;             // 16-row blocks of a tile per wave
    constexpr bool CHK = DP == 0;          // rows in chunks of 128 coordinates
    constexpr int CH = CHK ? 128 : DP;     // coordinates staged at a time
    constexpr int NT4 = CH / 16;           // float4 A-fragments per lane per block
    constexpr int LDX = CH + 4;            // padded LDS row stride (floats)
    constexpr int NV4 = CH / 4;            // float4 per staged row
    constexpr int RP = 256 / NV4;          // rows staged per pass
    constexpr int PASSES = BR / RP;
    const int dpr = CHK ? a.dp : DP;       // row stride (floats)
    const int nch = CHK ? a.dp / CH : 1;   // coordinate chunks per row
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int qw0 = (wave / G) * QW;       // the wave's first query in the workgroup
    const int nb0 = (wave % G) * NBW;      // the wave's first 16-row block of a tile
    const bool owner = wave % G == 0;      // merges the group's candidates

    float *xs = (float *)smem;                                   // [BR][LDX]
    int *rid = (int *)(xs + BR * LDX);                           // [BR]
    int *rq = rid + BR;                                          // [BR] qualifies
    float *xn2 = (float *)(rq + BR);                             // [BR]
    float *qn2 = xn2 + BR;                                       // [QM]
    int *cnt = (int *)(qn2 + QM);                                // [QM] keys in the append buffer
    int *fill = cnt + QM;                                        // [QM] keys in the list
    uint64_t *thr = (uint64_t *)(((uintptr_t)(fill + QM) + 7) & ~(uintptr_t)7);  // [QM]
    PredDev *qpred = (PredDev *)(thr + QM);                      // [QM] (batched form)

    const int K = a.K, CBq = a.CB;

    // A fragments: lane (m = lane % 16, kq = lane / 16) of wave w holds, for
    // block mb, query q0 + qw0 + 16*mb + m at coordinates 16t + 4kq + c.
    float4 af[MB][NT4];
    auto load_af = [&](int ch) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int mq = q0 + qw0 + mb * 16 + (lane & 15);
#pragma unroll
            for (int t = 0; t < NT4; ++t)
                af[mb][t] = mq < Bq ? *(const float4 *)(a.qp + (int64_t)mq * dpr + ch * CH + 16 * t + 4 * (lane >> 4))
                                     : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    if (!CHK) load_af(0);
    if (BATCHED && tid < QM) qpred[tid] = q0 + tid < Bq ? a.preds[q0 + tid] : PredDev{-1, {0}, {0}, {0}};
    // per-query state (private to the wave group) and list initialisation
    for (int i = lane; owner && i < QW; i += 64) {
        const int q = qw0 + i;
        cnt[q] = 0;
        fill[q] = 0;
        const int qa = q0 + q;
        // start from the best bound any chunk (or a first pass) has published
        thr[q] = qa < Bq ? __atomic_load_n((const unsigned long long *)(a.gthr + qa), __ATOMIC_RELAXED)
                         : KEY_INF;
        qn2[q] = qa < Bq ? a.qn2[qa] : 0.0f;
    }
    __syncthreads();

    const int64_t total = GATHER ? *a.sel_count : a.n;
    int64_t per = (total + nchunks - 1) / nchunks;
    per = (per + BR - 1) / BR * BR;
    int64_t c0 = (int64_t)chunk * per;
    int64_t c1 = min(total, c0 + per);
    pass_range(a, c0, c1, BR, total, nchunks);
    const float *X = (const float *)a.rows;

    // Tile pipeline: the row ids of the next tile whose rows are loaded
    // (gather: sid) and the per-row record of tile t+1 (thread r < 64 holds
    // row r's id, predicate columns and squared norm: ri_*) are fetched while
    // tile t is multiplied, so the vector loads of a tile never wait on
    // another load.
    const int sr = tid / NV4, sc = tid % NV4;  // staging: row within pass, float4 column
    int sid[PASSES];
    int64_t ri_row = 0;
    bool ri_ok = false;
    int32_t ri_av[4] = {0, 0, 0, 0};
    float ri_n2 = 0.0f;

    auto issue_ids = [&](int64_t t0) {
#pragma unroll
        for (int p = 0; p < PASSES; ++p) {
            const int64_t pos = t0 + p * RP + sr;
            sid[p] = (GATHER && pos < c1) ? a.sel_ids[pos] : 0;
        }
    };
    auto issue_rowinfo = [&](int64_t t0) {
        if (tid < BR) {
            const int64_t pos = t0 + tid;
            ri_ok = pos < c1;
            ri_row = ri_ok ? (GATHER ? (int64_t)a.sel_ids[pos] : pos) : 0;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                ri_av[t] = (!GATHER && !BATCHED && ri_ok && t < a.pred.nterms)
                               ? a.attr[(int64_t)a.pred.col[t] * a.an + ri_row]
                               : 0;
            ri_n2 = (METRIC == VRS_L2SQ && ri_ok) ? a.norm2[ri_row] : 0.0f;
        }
    };
    // In the small-batch form (G > 1) the vector loads of tile t+1 are issued
    // as soon as tile t is in LDS, so they are in flight during tile t's
    // product and epilogue (the registers this costs would cost the wide form
    // a resident workgroup); the wide form loads a tile when it starts it.
    constexpr bool PF = G > 1 && !CHK;
    float4 w[PASSES];
    auto issue_rows = [&](int64_t t0, int ch) {
#pragma unroll
        for (int p = 0; p < PASSES; ++p) {
            const int64_t pos = t0 + p * RP + sr;
            const int64_t row = GATHER ? (int64_t)sid[p] : pos;
            w[p] = pos < c1 ? load_x((const float4 *)(X + row * dpr + ch * CH) + sc, a.shared_rows)
                            : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    if (GATHER) issue_ids(c0);
    issue_rowinfo(c0);
    if (PF) {
        issue_rows(c0, 0);
        if (GATHER && c0 + BR < c1) issue_ids(c0 + BR);
    }

    for (int64_t t0 = c0; t0 < c1; t0 += BR) {
        if (!PF) {
            issue_rows(t0, 0);
            // (chunked rows still need this tile's ids for their later chunks)
            if (GATHER && !CHK && t0 + BR < c1) issue_ids(t0 + BR);
        }
        // ---- tile t0: per-row record and rows -> LDS
        bool mine = false;
        if (tid < BR) {
            bool ok = ri_ok;
            if (!GATHER && !BATCHED) {
                ok = ok && a.pred.nterms >= 0;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (t < a.pred.nterms) ok = ok && ri_av[t] >= a.pred.lo[t] && ri_av[t] <= a.pred.hi[t];
            }
            rid[tid] = (int)ri_row;
            rq[tid] = ok;
            xn2[tid] = ri_n2;
            mine = ok;
        }
        if (t0 + BR < c1) issue_rowinfo(t0 + BR);
#pragma unroll
        for (int p = 0; p < PASSES; ++p) *(float4 *)(xs + (p * RP + sr) * LDX + 4 * sc) = w[p];
        const int any = __syncthreads_or(mine);
        if (PF && t0 + BR < c1) {
            issue_rows(t0 + BR, 0);
            if (GATHER && t0 + 2 * BR < c1) issue_ids(t0 + 2 * BR);
        }
        if (!any) {
            if (GATHER && CHK && t0 + BR < c1) issue_ids(t0 + BR);
            continue;
        }

        // A wave whose queries all lie past the batch (a partial query
        // tile) skips the product and the epilogue; it still stages rows
        // and meets every barrier.
        const bool act = q0 + qw0 < Bq;
        // ---- Q X^T for the group's QW queries x the wave's NBW * 16 rows
        f4v acc[MB][NBW];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) acc[mb][nb] = (f4v){0.f, 0.f, 0.f, 0.f};
        for (int ch = 0; ch < nch; ++ch) {
            if (CHK && ch > 0) {
                __syncthreads();  // every wave is done with chunk ch - 1
#pragma unroll
                for (int p = 0; p < PASSES; ++p) *(float4 *)(xs + (p * RP + sr) * LDX + 4 * sc) = w[p];
                __syncthreads();
            }
            if (CHK && ch + 1 < nch) issue_rows(t0, ch + 1);  // in flight during this chunk's product
            if (!act) continue;
            if (CHK) load_af(ch);
#pragma unroll
            for (int t = 0; t < NT4; ++t) {
                float4 bv[NBW];
#pragma unroll
                for (int nb = 0; nb < NBW; ++nb)
                    bv[nb] = *(const float4 *)(xs + ((nb0 + nb) * 16 + (lane & 15)) * LDX + 16 * t + 4 * (lane >> 4));
                // independent accumulators back to back: no MFMA waits on the
                // result of the previous one
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                        for (int nb = 0; nb < NBW; ++nb)
                            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mb][t][c], bv[nb][c], acc[mb][nb], 0, 0, 0);
            }
        }
        if (GATHER && CHK && t0 + BR < c1) issue_ids(t0 + BR);
        if (act) {
            // ---- epilogue: lane holds queries qw0 + 16mb + 4(lane/16) + i, rows
            // 16(nb0 + nb) + lane%16
            if (owner && (((t0 - c0) / BR) & 15) == 15) {
                for (int i = lane; i < QW; i += 64) {
                    const int qa = q0 + qw0 + i;
                    if (qa < Bq) {
                        const uint64_t g = __atomic_load_n((const unsigned long long *)(a.gthr + qa), __ATOMIC_RELAXED);
                        if (g < thr[qw0 + i]) thr[qw0 + i] = g;
                    }
                }
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int qb = qw0 + mb * 16 + 4 * (lane >> 4);
                uint64_t th[4];
                float qn[4], thf[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    th[i] = thr[qb + i];
                    thf[i] = key_dist(th[i]);
                    qn[i] = qn2[qb + i];
                }
#pragma unroll
                for (int nb = 0; nb < NBW; ++nb) {
                    const int r = (nb0 + nb) * 16 + (lane & 15);
                    if (!rq[r]) continue;
                    const int row = rid[r];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int q = qb + i;
                        const int qa = q0 + q;
                        if (qa >= Bq) continue;
                        if (BATCHED && !pred_eval(qpred[q], a.attr, a.an, row)) continue;
                        const float dist = METRIC == VRS_L2SQ ? fmaf(-2.0f, acc[mb][nb][i], qn[i] + xn2[r]) : -acc[mb][nb][i];
                        if (!(dist <= thf[i])) continue;
                        const uint64_t key = make_key(dist, (uint32_t)row);
                        if (key < th[i]) {
                            const int slot = atomicAdd(&cnt[q], 1);
                            a.cbuf[((int64_t)qa * nchunks + chunk) * CBq + slot] = key;
                        }
                    }
                }
            }
        }
        // ---- flush the group's queries whose buffer could overflow next tile
        if (G == 1)
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        else
            __syncthreads();  // every wave of the group has appended its candidates
        if (owner) {
            const int myc = lane < QW ? cnt[qw0 + lane] : 0;
            uint64_t full = __ballot(lane < QW && myc > CBq - BR);
            while (full) {
                const int j = __ffsll((long long)full) - 1;
                full &= full - 1;
                const int q = qw0 + j, qa = q0 + q;
                const int64_t base = (int64_t)qa * nchunks + chunk;
                const int nq = cnt[q], fq = fill[q], Kq = list_len(a, qa, K);
                flush_fit<E>(a.partials + base * K, a.cbuf + base * CBq, nq, Kq, fq, &thr[q], a.gthr + qa);
                if (lane == 0) {
                    cnt[q] = 0;
                    fill[q] = min(Kq, fq + nq);
                }
            }
        }
        __syncthreads();  // the LDS tile is reused
    }
    // ---- final flush of every pending buffer (by each group's first wave)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    if (!owner) return;
    const int myc = lane < QW ? cnt[qw0 + lane] : 0;
    uint64_t pend = __ballot(lane < QW && myc > 0 && q0 + qw0 + lane < Bq);
    while (pend) {
        const int j = __ffsll((long long)pend) - 1;
        pend &= pend - 1;
        const int q = qw0 + j, qa = q0 + q;
        const int64_t base = (int64_t)qa * nchunks + chunk;
        const int nq = cnt[q], fq = fill[q], Kq = list_len(a, qa, K);
        flush_fit<E>(a.partials + base * K, a.cbuf + base * CBq, nq, Kq, fq, &thr[q], a.gthr + qa);
        if (lane == 0) fill[q] = min(Kq, fq + nq);
    }
    // each list's key count, or (no count array) KEY_INF in the list
    // entries past its keys (the whole list length K)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    if (a.fills) {
        if (lane < QW && q0 + qw0 + lane < Bq)
            a.fills[(int64_t)(q0 + qw0 + lane) * nchunks + chunk] = fill[qw0 + lane];
    } else {
        for (int j = 0; j < QW; ++j) {
            const int q = qw0 + j, qa = q0 + q;
            if (qa < Bq) list_tail_inf(a.partials + ((int64_t)qa * nchunks + chunk) * K, fill[q], K);
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

template <int DP, int METRIC, bool GATHER, bool BATCHED, int E, int MB, int G>
// (the chunked form at 3 workgroups per CU spills a few registers outside its
// inner loop; with the registers for 2 it measured 10 % slower on 4M x 768)
__global__ __launch_bounds__(256, (E <= 8 && MB == 1 && G == 1) ? 3 : 2) void screen_mfma_f32_kernel(ScreenArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int QM = 64 * MB / G;
    int chunk, qt;
    xcd_item(blockIdx.x, a.n_chunks, (a.B + QM - 1) / QM, &chunk, &qt);
    f32_tile<DP, METRIC, GATHER, BATCHED, E, MB, G>(a, chunk, a.n_chunks, qt * QM, a.B, smem);
}

// Persistent form (batched uneven launch), queue per XCD: see the bfloat16
// kernel's persistent form.
template <int DP, int METRIC, int E, int MB>
__global__ __launch_bounds__(256, (E <= 8 && MB == 1) ? 3 : 2) void screen_mfma_f32_persistent(ScreenArgs a) {
    constexpr int QM = 64 * MB;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int item_s;
    const int Bq = a.bctl[BC_NDENSE], nc = a.bctl[BC_NC];
    const int ntiles = (Bq + QM - 1) / QM;
    const int per = nc / 8 * ntiles;
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
        f32_tile<DP, METRIC, false, true, E, MB>(a, chunk, nc, qt * QM, Bq, smem);
        __syncthreads();
    }
}

template <int DP, int METRIC, int E, int MB>
hipError_t launch_e(const ScreenArgs &a, hipStream_t s) {
    const size_t lds = screen_mfma_lds(DP ? DP : a.dp, 64 * MB);  // (DP = 0: chunked rows of a.dp)
    if (MB == 1 && !a.preds && a.B <= 16) {
        // one group of 16 queries shared by the four waves (each takes 16 of
        // a tile's 64 rows)
        dim3 grid(a.n_chunks * ((a.B + 15) / 16)), block(256);
        auto k = a.gather ? screen_mfma_f32_kernel<DP, METRIC, true, false, E, 1, 4>
                          : screen_mfma_f32_kernel<DP, METRIC, false, false, E, 1, 4>;
        ensure_dyn_lds((const void *)k, lds);
        k<<<grid, block, lds, s>>>(a);
        return hipGetLastError();
    }
    constexpr int QM = 64 * MB;
    dim3 grid(a.n_chunks * ((a.B + QM - 1) / QM)), block(256);
    if (a.preds) {
        auto k = screen_mfma_f32_kernel<DP, METRIC, false, true, E, MB, 1>;
        ensure_dyn_lds((const void *)k, lds);
        k<<<grid, block, lds, s>>>(a);
    } else if (a.gather) {
        auto k = screen_mfma_f32_kernel<DP, METRIC, true, false, E, MB, 1>;
        ensure_dyn_lds((const void *)k, lds);
        k<<<grid, block, lds, s>>>(a);
    } else {
        auto k = screen_mfma_f32_kernel<DP, METRIC, false, false, E, MB, 1>;
        ensure_dyn_lds((const void *)k, lds);
        k<<<grid, block, lds, s>>>(a);
    }
    return hipGetLastError();
}

template <int DP, int METRIC, int MB>
hipError_t launch_dp(const ScreenArgs &a, hipStream_t s) {
    switch ((a.Kp + a.CB) / 64) {
    case 4: return launch_e<DP, METRIC, 4, MB>(a, s);
    case 8: return launch_e<DP, METRIC, 8, MB>(a, s);
    case 16: return launch_e<DP, METRIC, 16, MB>(a, s);
    default: return launch_e<DP, METRIC, 32, MB>(a, s);
    }
}

template <int METRIC, int MB>
hipError_t launch_m(const ScreenArgs &a, hipStream_t s) {
    switch (a.dp) {
    case 32: return launch_dp<32, METRIC, MB>(a, s);
    case 64: return launch_dp<64, METRIC, MB>(a, s);
    case 128: return launch_dp<128, METRIC, MB>(a, s);
    case 256: return launch_dp<256, METRIC, MB>(a, s);
    default:
        if (a.dp > 256 && a.dp % 128 == 0) return launch_dp<0, METRIC, MB>(a, s);  // chunked rows
        return hipErrorInvalidValue;
    }
}

}  // namespace

size_t screen_mfma_lds(int dp, int qm) {
    const int ch = dp > 256 ? 128 : dp;  // coordinates staged at a time
    return (size_t)BR * (ch + 4) * 4 + BR * 12 + qm * 12 + 8 + qm * 8 + qm * sizeof(PredDev) + 16;
}

// Resident workgroups per CU (register budget of the kernel, set by E and the
// queries per workgroup qm: 64 and 128 for the wide forms, 16 for the
// small-batch form).
int screen_mfma_occupancy(int Kp, int CB, int qm) {
    return ((Kp + CB) / 64 <= 8 && qm == 64) ? 3 : 2;
}

bool screen_mfma_supported(int dp, vrs_dtype store, int Kp, int CB) {
    const int E = (Kp + CB) / 64;
    return store == VRS_F32 && (dp == 32 || dp == 64 || dp == 128 || dp == 256 || (dp > 256 && dp % 128 == 0)) &&
           (E == 4 || E == 8 || E == 16 || E == 32) && (Kp + CB) == 64 * E;
}

template <int DP, int METRIC, int E, int MB>
hipError_t launch_pe(const ScreenArgs &a, int grid, hipStream_t s) {
    const size_t lds = screen_mfma_lds(DP, 64 * MB);
    auto k = screen_mfma_f32_persistent<DP, METRIC, E, MB>;
    ensure_dyn_lds((const void *)k, lds);
    k<<<grid, 256, lds, s>>>(a);
    return hipGetLastError();
}

template <int DP, int METRIC, int MB>
hipError_t launch_pdp(const ScreenArgs &a, int grid, hipStream_t s) {
    switch ((a.Kp + a.CB) / 64) {
    case 4: return launch_pe<DP, METRIC, 4, MB>(a, grid, s);
    case 8: return launch_pe<DP, METRIC, 8, MB>(a, grid, s);
    case 16: return launch_pe<DP, METRIC, 16, MB>(a, grid, s);
    default: return launch_pe<DP, METRIC, 32, MB>(a, grid, s);
    }
}

template <int METRIC, int MB>
hipError_t launch_pm(const ScreenArgs &a, int grid, hipStream_t s) {
    switch (a.dp) {
    case 32: return launch_pdp<32, METRIC, MB>(a, grid, s);
    case 64: return launch_pdp<64, METRIC, MB>(a, grid, s);
    case 128: return launch_pdp<128, METRIC, MB>(a, grid, s);
    case 256: return launch_pdp<256, METRIC, MB>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_screen_mfma_persistent(const ScreenArgs &a, int qm, int grid, hipStream_t s) {
    if (!a.bctl || !a.preds) return hipErrorInvalidValue;
    if (qm == 128)
        return a.metric == VRS_L2SQ ? launch_pm<VRS_L2SQ, 2>(a, grid, s) : launch_pm<VRS_IP, 2>(a, grid, s);
    return a.metric == VRS_L2SQ ? launch_pm<VRS_L2SQ, 1>(a, grid, s) : launch_pm<VRS_IP, 1>(a, grid, s);
}

hipError_t launch_screen_mfma(const ScreenArgs &a, int qm, hipStream_t s) {
    if (qm == 128)
        return a.metric == VRS_L2SQ ? launch_m<VRS_L2SQ, 2>(a, s) : launch_m<VRS_IP, 2>(a, s);
    return a.metric == VRS_L2SQ ? launch_m<VRS_L2SQ, 1>(a, s) : launch_m<VRS_IP, 1>(a, s);
}

}  // namespace vrs
