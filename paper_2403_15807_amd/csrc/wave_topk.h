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

// Merge the append buffer of one query (n keys) into its sorted list (one
// wave).  Only the list's first `fill` entries can hold keys; the rest is
// KEY_INF or not written yet (lists are not cleared up front), so the
// bitonic sort covers 64 * E >= fill + n keys and list entries from 64 * E
// on are left as they are.
template <int E>
__device__ inline void flush_one(uint64_t *list, const uint64_t *buf, int n, int K, int fill,
                                 uint64_t *thr_out, uint64_t *gthr) {
    const int lane = threadIdx.x & 63;
    uint64_t v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = lane * E + e;
        uint64_t x = KEY_INF;
        if (i < fill)
            x = list[i];
        else if (i - fill < n)
            x = buf[i - fill];
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
    // broadcast the K-th key from the lane that holds it (past the sorted
    // width it is KEY_INF), publish it as a bound for every chunk of this
    // query and take the best bound known
    if (K <= 64 * E) kth = (uint64_t)__shfl((long long)kth, (K - 1) / E);
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
__device__ __noinline__ void flush_query(uint64_t *list, const uint64_t *buf, int n, int K, int fill,
                                   uint64_t *thr_out, uint64_t *gthr) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    flush_one<E>(list, buf, n, K, fill, thr_out, gthr);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// A flush on the narrowest sort (64 to 64 * EMAX keys) that holds the list's
// real keys and the buffer: a list that holds a few keys costs a few sort
// stages, not those of the full list length.  fill + n <= 64 * EMAX.
template <int EMAX>
__device__ __forceinline__ void flush_fit(uint64_t *list, const uint64_t *buf, int n, int K, int fill,
                                 uint64_t *thr_out, uint64_t *gthr) {
    const int need = __builtin_amdgcn_readfirstlane(fill + n);
    if (EMAX > 1 && need <= 64)
        flush_query<1>(list, buf, n, K, fill, thr_out, gthr);
    else if (EMAX > 2 && need <= 128)
        flush_query<2>(list, buf, n, K, fill, thr_out, gthr);
    else if (EMAX > 4 && need <= 256)
        flush_query<4>(list, buf, n, K, fill, thr_out, gthr);
    else if (EMAX > 8 && need <= 512)
        flush_query<8>(list, buf, n, K, fill, thr_out, gthr);
    else if (EMAX > 16 && need <= 1024)
        flush_query<16>(list, buf, n, K, fill, thr_out, gthr);
    else
        flush_query<EMAX>(list, buf, n, K, fill, thr_out, gthr);
}

// List entries [fill, K) of a list whose first `fill` entries are its keys:
// KEY_INF (one wave).
__device__ inline void list_tail_inf(uint64_t *list, int fill, int K) {
    for (int i = fill + (int)(threadIdx.x & 63); i < K; i += 64) list[i] = KEY_INF;
}

// EMAX = (Kp + CB) / 64 keys per lane in the widest flush (compile-time:
// sets the register budget of the whole kernel).
}  // namespace vrs
