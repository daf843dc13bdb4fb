// wave_topk.h -- wave-private top-k lists of the MFMA screening kernels:
// a query's candidates are produced by one wave only, appended to a buffer
// in global memory (L2-resident workspace) and merged into the query's sorted
// list by that wave with an in-register bitonic sort.
#pragma once

#include "common.h"

namespace vrs {

// Keys a query keeps per list: its own k'+1 in the batched uneven form
// (lists are K = max k'+1 long, the tail stays KEY_INF), else K.  A shorter
// list gives the query its own, tighter admission bound.
__device__ __forceinline__ int list_len(const ScreenArgs &a, int qa, int K) {
    return a.kps ? min(K, a.kps[qa] + 1) : K;
}

// Merge the append buffer of one query into its sorted list (one wave).
template <int E>
__device__ inline void flush_one(uint64_t *list, const uint64_t *buf, int n, int K, int Kp,
                          uint64_t *thr_out, uint64_t *gthr) {
    const int lane = threadIdx.x & 63;
    uint64_t v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = lane * E + e;
        uint64_t x = KEY_INF;
        if (i < Kp) {
            if (i < K) x = list[i];
        } else if (i - Kp < n) {
            x = buf[i - Kp];
        }
        v[e] = x;
    }
    wave_sort_u64<E>(v);
    uint64_t kth = KEY_INF;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = lane * E + e;
        if (i < K) list[i] = v[e];
        if (i == K - 1) kth = v[e];
    }
    // broadcast the K-th key from the lane that holds it, publish it as a
    // bound for every chunk of this query and take the best bound known
    const int src = (K - 1) / E;
    kth = (uint64_t)__shfl((long long)kth, src);
    if (lane == 0) {
        uint64_t best = kth;
        if (kth != KEY_INF) {
            const uint64_t prev = atomicMin((unsigned long long *)gthr, (unsigned long long)kth);
            best = prev < kth ? prev : kth;
        }
        *thr_out = best;
    }
}

template <int E>
__device__ inline void flush_query(uint64_t *list, const uint64_t *buf, int n, int K, int Kp,
                            uint64_t *thr_out, uint64_t *gthr) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    flush_one<E>(list, buf, n, K, Kp, thr_out, gthr);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// E = (Kp + CB) / 64 keys per lane in a flush (compile-time: sets the
// register budget of the whole kernel).
}  // namespace vrs
