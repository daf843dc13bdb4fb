// topk_sized.h -- TopkLds::flush with a sort only as wide as the keys held.
#pragma once

#include "internal.h"

namespace vrs {

// When every list's keys (its first `fill` entries; the rest of a list is
// +inf) and its buffer fit in the list's Kp entries, the buffer is appended
// to the keys and the first S = next_pow2(max fill + cnt) entries of each
// list are sorted (bitonic, lists at stride M), instead of all M entries of
// every list as flush() does; otherwise it is flush().  Same result either
// way.  All NT threads of the workgroup call it; at most 8 lists.
template <typename K, int NT>
__device__ void flush_sized(TopkLds<K> &tk, int tid) {
    __shared__ int fill_s[8];
    const int nq = tk.nq, Kp = tk.Kp, M = tk.M();
    K *keys = tk.keys;
    if (nq > 8) {
        tk.flush(tid, NT);
        return;
    }
    const K inf = KeyOps<K>::inf();
    if (tid < nq) fill_s[tid] = Kp;
    __syncthreads();
    for (int p = tid; p < nq * Kp; p += NT) {
        const int b = p / Kp, i = p - b * Kp;
        const K *l = keys + (size_t)b * M;
        // the first +inf entry (one per list; no real key is +inf)
        if (!KeyOps<K>::less(l[i], inf) && (i == 0 || KeyOps<K>::less(l[i - 1], inf))) fill_s[b] = i;
    }
    __syncthreads();
    int S = 2;
    bool fits = true;
    for (int b = 0; b < nq; ++b) {
        const int need = fill_s[b] + tk.cnt[b];
        fits = fits && need <= Kp;
        while (S < need) S <<= 1;
    }
    if (!fits || S >= M) {  // (uniform)
        tk.flush(tid, NT);
        return;
    }
    for (int p = tid; p < nq * tk.CB; p += NT) {
        const int b = p / tk.CB, i = p - b * tk.CB;
        if (i < tk.cnt[b]) keys[(size_t)b * M + fill_s[b] + i] = keys[(size_t)b * M + Kp + i];
    }
    __syncthreads();
    const int half = S >> 1, lgh = __ffs(half) - 1;
    for (int size = 2; size <= S; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int lgs = __ffs(stride) - 1;
            for (int p = tid; p < nq * half; p += NT) {
                const int seg = p >> lgh, pi = p & (half - 1);
                const int i = ((pi >> lgs) << (lgs + 1)) + (pi & (stride - 1)), j = i + stride;
                K *sg = keys + (size_t)seg * M;
                const K x = sg[i], y = sg[j];
                if ((i & size) == 0 ? KeyOps<K>::less(y, x) : KeyOps<K>::less(x, y)) {
                    sg[i] = y;
                    sg[j] = x;
                }
            }
            __syncthreads();
        }
    }
    for (int p = tid; p < nq * (Kp - tk.Kkeep); p += NT) {
        const int b = p / (Kp - tk.Kkeep), i = p - b * (Kp - tk.Kkeep);
        keys[(size_t)b * M + tk.Kkeep + i] = inf;
    }
    __syncthreads();
    for (int b = tid; b < nq; b += NT) {
        tk.thr[b] = keys[(size_t)b * M + tk.Kkeep - 1];
        tk.cnt[b] = 0;
    }
    __syncthreads();
}

}  // namespace vrs
