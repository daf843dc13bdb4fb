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
// Workgroup = 4 waves = 64 queries (16 per wave) x one chunk of rows, rows
// in tiles of 128, coordinates in chunks of 64: the row chunk and the
// queries' hi/lo chunk are staged through LDS, and the loads of the next
// chunk (or of the next tile's first chunk) are in flight while the current
// one is multiplied.  Top-k state is wave-private as in the float32 kernel.
#include "internal.h"
#include "wave_topk.h"

namespace vrs {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));

constexpr int QM = 64;    // queries per workgroup
constexpr int BR = 128;   // rows per tile
constexpr int KC = 64;    // coordinates per chunk
constexpr int LDK = 72;   // LDS row stride in bfloat16 elements (144 bytes)

// Row loads: non-temporal when each row is read once (one query tile), plain
// when the other query tiles of the same row chunk will read it again from L2.
__device__ __forceinline__ uint4 load_x(const void *p, int shared) {
    if (shared) return *(const uint4 *)p;
    v4u32 v = __builtin_nontemporal_load((const v4u32 *)p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// 4 e4m3fn codes -> 4 bfloat16 (exact), packed in two 32-bit words.
__device__ __forceinline__ uint2 e4m3x4_to_bf16x4(uint32_t w) {
    uint32_t h[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) h[j] = __float_as_uint(e4m3_to_f32((w >> (8 * j)) & 0xffu)) >> 16;
    return make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
}

// One work item: queries [q0, q0 + QM) (of Bq) against row chunk `chunk` of
// `nchunks`; its lists are (query, chunk) lists of the partials.
template <int STORE, bool GATHER, bool BATCHED, int E>
__device__ __forceinline__ void bf16_tile(const ScreenArgs &a, const int chunk, const int nchunks,
                                          const int q0, const int Bq, unsigned char *smem) {
    constexpr int XLD = STORE == VRS_BF16 ? 4 : 2;  // 16-byte row loads per thread per chunk
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int dp = a.dp;
    const int nkc = dp / KC;

    uint16_t *xs = (uint16_t *)smem;                      // [BR][LDK]
    uint16_t *qs = xs + BR * LDK;                         // [QM][2][LDK]
    // Per-row records in three rotating slots: tile t+1's record is written
    // before tile t's first barrier, while waves that are still in the
    // epilogue of tile t-1 read theirs (with one coordinate chunk per row
    // there is no other barrier in between).
    int *rid = (int *)(qs + QM * 2 * LDK);                // [3][BR]
    int *rq = rid + 3 * BR;                               // [3][BR]
    float *rsc = (float *)(rq + 3 * BR);                  // [3][BR]
    int *cnt = (int *)(rsc + 3 * BR);                     // [QM]
    uint64_t *thr = (uint64_t *)(((uintptr_t)(cnt + QM) + 7) & ~(uintptr_t)7);  // [QM]
    PredDev *qpred = (PredDev *)(thr + QM);               // [QM]

    const int K = a.K, Kp = a.Kp, CBq = a.CB;
    if (tid < QM) {
        cnt[tid] = 0;
        thr[tid] = KEY_INF;
        if (BATCHED) qpred[tid] = q0 + tid < Bq ? a.preds[q0 + tid] : PredDev{-1, {0}, {0}, {0}};
    }
    for (int i = lane; i < 16 * K; i += 64) {
        const int qa = q0 + wave * 16 + i / K;
        if (qa < Bq) a.partials[((int64_t)qa * nchunks + chunk) * K + (i % K)] = KEY_INF;
    }

    const int64_t total = GATHER ? *a.sel_count : a.n;
    int64_t per = (total + nchunks - 1) / nchunks;
    per = (per + BR - 1) / BR * BR;
    const int64_t c0 = (int64_t)chunk * per;
    const int64_t c1 = min(total, c0 + per);
    const int EB = STORE == VRS_BF16 ? 2 : 1;
    const char *X = (const char *)a.rows;
    const int64_t row_bytes = (int64_t)dp * EB;

    // per-row record of a tile, produced by thread r < BR
    auto rowinfo = [&](int64_t t0, int slot) {
        if (tid < BR) {
            const int64_t pos = t0 + tid;
            bool ok = pos < c1;
            int64_t row = ok ? (GATHER ? (int64_t)a.sel_ids[pos] : pos) : 0;
            if (ok && !GATHER && !BATCHED) ok = pred_eval(a.pred, a.attr, a.an, row);
            rid[slot * BR + tid] = (int)row;
            rq[slot * BR + tid] = ok;
            rsc[slot * BR + tid] = (STORE == VRS_FP8E4M3 && ok) ? a.scale[row] : 1.0f;
        }
    };
    uint4 xr[XLD], qr[4];
    auto issue = [&](int slot, int kc) {
#pragma unroll
        for (int i = 0; i < XLD; ++i) {
            const int idx = tid + 256 * i;
            const int r = STORE == VRS_BF16 ? idx >> 3 : idx >> 2;
            const int c = STORE == VRS_BF16 ? idx & 7 : idx & 3;
            xr[i] = rq[slot * BR + r]
                        ? load_x(X + (int64_t)rid[slot * BR + r] * row_bytes + kc * KC * EB + c * 16, a.shared_rows)
                        : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = tid + 256 * i;
            const int q = idx >> 4, hl = (idx >> 3) & 1, c = idx & 7;
            qr[i] = q0 + q < Bq ? *(const uint4 *)(a.qhl + ((int64_t)(q0 + q) * 2 + hl) * dp + kc * KC + c * 8)
                                 : make_uint4(0, 0, 0, 0);
        }
    };
    auto commit = [&]() {
#pragma unroll
        for (int i = 0; i < XLD; ++i) {
            const int idx = tid + 256 * i;
            if (STORE == VRS_BF16) {
                *(uint4 *)(xs + (idx >> 3) * LDK + (idx & 7) * 8) = xr[i];
            } else {
                uint16_t *d = xs + (idx >> 2) * LDK + (idx & 3) * 16;
                const uint2 p0 = e4m3x4_to_bf16x4(xr[i].x), p1 = e4m3x4_to_bf16x4(xr[i].y);
                const uint2 p2 = e4m3x4_to_bf16x4(xr[i].z), p3 = e4m3x4_to_bf16x4(xr[i].w);
                *(uint4 *)d = make_uint4(p0.x, p0.y, p1.x, p1.y);
                *(uint4 *)(d + 8) = make_uint4(p2.x, p2.y, p3.x, p3.y);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = tid + 256 * i;
            *(uint4 *)(qs + ((idx >> 4) * 2 + ((idx >> 3) & 1)) * LDK + (idx & 7) * 8) = qr[i];
        }
    };

    rowinfo(c0, 0);
    __syncthreads();
    if (c0 < c1) issue(0, 0);
    int slot = 0;
    for (int64_t t0 = c0; t0 < c1; t0 += BR, slot = slot == 2 ? 0 : slot + 1) {
        const int nslot = slot == 2 ? 0 : slot + 1;
        const bool last_tile = t0 + BR >= c1;
        f4v ah[8], al[8];
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
            ah[nb] = (f4v){0.f, 0.f, 0.f, 0.f};
            al[nb] = (f4v){0.f, 0.f, 0.f, 0.f};
        }
        for (int kc = 0; kc < nkc; ++kc) {
            commit();
            if (kc == nkc - 1 && !last_tile) rowinfo(t0 + BR, nslot);
            __syncthreads();
            if (kc + 1 < nkc)
                issue(slot, kc + 1);
            else if (!last_tile)
                issue(nslot, 0);
#pragma unroll
            for (int ks = 0; ks < KC / 32; ++ks) {
                const uint16_t *qa_p = qs + ((wave * 16 + (lane & 15)) * 2) * LDK + ks * 32 + (lane >> 4) * 8;
                const bf8v A_hi = *(const bf8v *)qa_p;
                const bf8v A_lo = *(const bf8v *)(qa_p + LDK);
#pragma unroll
                for (int nb = 0; nb < 8; ++nb) {
                    const bf8v Bv = *(const bf8v *)(xs + (nb * 16 + (lane & 15)) * LDK + ks * 32 + (lane >> 4) * 8);
                    ah[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A_hi, Bv, ah[nb], 0, 0, 0);
                    al[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A_lo, Bv, al[nb], 0, 0, 0);
                }
            }
            __syncthreads();
        }

        // ---- epilogue: lane holds queries 16w + 4(lane/16) + i, rows 16nb + lane%16
        if ((((t0 - c0) / BR) & 7) == 7 && lane < 16) {
            const int qa = q0 + wave * 16 + lane;
            if (qa < Bq) {
                const uint64_t g = __atomic_load_n((const unsigned long long *)(a.gthr + qa), __ATOMIC_RELAXED);
                if (g < thr[wave * 16 + lane]) thr[wave * 16 + lane] = g;
            }
        }
        const int qb = wave * 16 + 4 * (lane >> 4);
        uint64_t th[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) th[i] = thr[qb + i];
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
            const int r = slot * BR + nb * 16 + (lane & 15);
            if (!rq[r]) continue;
            const int row = rid[r];
            const float sc = rsc[r];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int q = qb + i, qa = q0 + q;
                if (qa >= Bq) continue;
                if (BATCHED && !pred_eval(qpred[q], a.attr, a.an, row)) continue;
                const float dot = ah[nb][i] + al[nb][i];
                const float dist = STORE == VRS_FP8E4M3 ? -(sc * dot) : -dot;
                const uint64_t key = make_key(dist, (uint32_t)row);
                if (key < th[i]) {
                    const int sl = atomicAdd(&cnt[q], 1);
                    a.cbuf[((int64_t)qa * nchunks + chunk) * CBq + sl] = key;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        {
            const int myc = lane < 16 ? cnt[wave * 16 + lane] : 0;
            uint64_t full = __ballot(lane < 16 && myc > CBq - BR);
            while (full) {
                const int j = __ffsll((long long)full) - 1;
                full &= full - 1;
                const int q = wave * 16 + j, qa = q0 + q;
                const int64_t base = (int64_t)qa * nchunks + chunk;
                flush_query<E>(a.partials + base * K, a.cbuf + base * CBq, cnt[q], K, Kp, &thr[q],
                               a.gthr + qa);
                if (lane == 0) cnt[q] = 0;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    const int myc = lane < 16 ? cnt[wave * 16 + lane] : 0;
    uint64_t pend = __ballot(lane < 16 && myc > 0 && q0 + wave * 16 + lane < Bq);
    while (pend) {
        const int j = __ffsll((long long)pend) - 1;
        pend &= pend - 1;
        const int q = wave * 16 + j, qa = q0 + q;
        const int64_t base = (int64_t)qa * nchunks + chunk;
        flush_query<E>(a.partials + base * K, a.cbuf + base * CBq, cnt[q], K, Kp, &thr[q],
                       a.gthr + qa);
    }
}


template <int STORE, bool GATHER, bool BATCHED, int E>
__global__ __launch_bounds__(256, 2) void screen_mfma_bf16_kernel(ScreenArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    bf16_tile<STORE, GATHER, BATCHED, E>(a, blockIdx.x, a.n_chunks, blockIdx.y * QM, a.B, smem);
}

// Persistent form (batched uneven launch): the dense queries are positions
// [0, n_dense) and each has n_c row chunks, both decided on the device.
// Workgroup g serves the queue of XCD g % 8 (workgroups are dispatched to
// the XCDs round-robin), which holds chunks c = x (mod 8) with every query
// tile, chunk-major: the query tiles of one chunk run at the same time on
// one XCD and read its rows through the same L2.  An empty queue sends the
// workgroup to the other XCDs' queues.
template <int STORE, int E>
__global__ __launch_bounds__(256, 2) void screen_mfma_bf16_persistent(ScreenArgs a) {
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
        bf16_tile<STORE, false, true, E>(a, chunk, nc, qt * QM, Bq, smem);
        __syncthreads();
    }
}

template <int STORE, int E>
hipError_t launch_se(const ScreenArgs &a, hipStream_t s) {
    dim3 grid(a.n_chunks, (a.B + QM - 1) / QM), block(256);
    const size_t lds = screen_mfma_bf16_lds();
    if (a.preds) {
        auto k = screen_mfma_bf16_kernel<STORE, false, true, E>;
        ensure_dyn_lds((const void *)k, lds);
        k<<<grid, block, lds, s>>>(a);
    } else if (a.gather) {
        auto k = screen_mfma_bf16_kernel<STORE, true, false, E>;
        ensure_dyn_lds((const void *)k, lds);
        k<<<grid, block, lds, s>>>(a);
    } else {
        auto k = screen_mfma_bf16_kernel<STORE, false, false, E>;
        ensure_dyn_lds((const void *)k, lds);
        k<<<grid, block, lds, s>>>(a);
    }
    return hipGetLastError();
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

}  // namespace

size_t screen_mfma_bf16_lds() {
    return (size_t)BR * LDK * 2 + (size_t)QM * 2 * LDK * 2 + 3 * BR * 12 + QM * 4 + 8 + QM * 8 +
           QM * sizeof(PredDev) + 16;
}

bool screen_mfma_bf16_supported(int dp, vrs_dtype store, int metric, int Kp, int CB) {
    const int E = (Kp + CB) / 64;
    return (store == VRS_BF16 || store == VRS_FP8E4M3) && metric == VRS_IP && dp % KC == 0 &&
           (E == 4 || E == 8 || E == 16 || E == 32) && (Kp + CB) == 64 * E;
}

template <int STORE, int E>
hipError_t launch_pe(const ScreenArgs &a, int grid, hipStream_t s) {
    const size_t lds = screen_mfma_bf16_lds();
    auto k = screen_mfma_bf16_persistent<STORE, E>;
    ensure_dyn_lds((const void *)k, lds);
    k<<<grid, 256, lds, s>>>(a);
    return hipGetLastError();
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

hipError_t launch_screen_mfma_bf16_persistent(const ScreenArgs &a, int grid, hipStream_t s) {
    if (a.metric != VRS_IP || !a.bctl || !a.preds) return hipErrorInvalidValue;
    return a.store == VRS_BF16 ? launch_p<VRS_BF16>(a, grid, s) : launch_p<VRS_FP8E4M3>(a, grid, s);
}

hipError_t launch_screen_mfma_bf16(const ScreenArgs &a, hipStream_t s) {
    if (a.metric != VRS_IP) return hipErrorInvalidValue;
    return a.store == VRS_BF16 ? launch_s<VRS_BF16>(a, s) : launch_s<VRS_FP8E4M3>(a, s);
}

}  // namespace vrs
