// common.h -- device helpers shared by the gfx950 kernels of the filtered
// top-k scan: sortable keys, storage decoders, the relational predicate and
// the LDS top-k lists.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vrs {

constexpr int WAVE = 64;
constexpr uint64_t KEY_INF = ~0ull;

// ---------------------------------------------------------------- keys
// A candidate is the 64-bit key (order-preserving bits of the float32
// screening distance) << 32 | row id, so that unsigned comparison orders by
// (distance, id) -- ties go to the lower row id.  -0.0 is folded into +0.0
// first, otherwise the bit trick would put -0 before +0.
__device__ __forceinline__ uint32_t ord32(float f) {
    f = (f == 0.0f) ? 0.0f : f;
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord32(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(u);
}
__device__ __forceinline__ uint64_t make_key(float d, uint32_t row) {
    return ((uint64_t)ord32(d) << 32) | row;
}
// Distance part of a key as a float bound: key(d, row) < th implies
// d <= key_dist(th), so the float test can reject before the key is built.
__device__ __forceinline__ float key_dist(uint64_t th) {
    const uint32_t hi = (uint32_t)(th >> 32);
    return hi == 0xffffffffu ? __int_as_float(0x7f800000) : unord32(hi);
}
__device__ __forceinline__ uint64_t ord64(double f) {
    f = (f == 0.0) ? 0.0 : f;
    uint64_t u = (uint64_t)__double_as_longlong(f);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double unord64(uint64_t o) {
    uint64_t u = (o & 0x8000000000000000ull) ? (o & 0x7fffffffffffffffull) : ~o;
    return __longlong_as_double((long long)u);
}

// Exact-distance key for the FP64 fallback: (ord64(dist64), row).
struct Key128 {
    uint64_t hi, lo;
};

template <typename K>
struct KeyOps;
template <>
struct KeyOps<uint64_t> {
    __device__ static uint64_t inf() { return KEY_INF; }
    __device__ static bool less(uint64_t a, uint64_t b) { return a < b; }
};
template <>
struct KeyOps<Key128> {
    __device__ static Key128 inf() { return Key128{KEY_INF, KEY_INF}; }
    __device__ static bool less(const Key128 &a, const Key128 &b) {
        return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
    }
};

// ---------------------------------------------------------------- decoders
__device__ __forceinline__ float bf16_to_f32(uint32_t h16) { return __uint_as_float(h16 << 16); }

// OCP e4m3fn -> float32, exact (every e4m3 value is a float32).
__device__ __forceinline__ float e4m3_to_f32(uint32_t c) {
    uint32_t s = (c & 0x80u) << 24, e = (c >> 3) & 15u, m = c & 7u;
    float mag = (e == 0) ? (float)m * 0.001953125f /* 2^-9 */
                         : __uint_as_float(((e + 120u) << 23) | (m << 20));
    return __uint_as_float(__float_as_uint(mag) | s);
}

// ------------------------------------------------------------- predicate
// Conjunction of inclusive int32 ranges (the host folds the ABI's int64
// half-open bounds into these; an empty range is lo > hi; nterms < 0 means
// the predicate selects nothing).
struct PredDev {
    int32_t nterms;
    int32_t col[4];
    int32_t lo[4];
    int32_t hi[4];
};

__device__ __forceinline__ bool pred_eval(const PredDev &p, const int32_t *__restrict__ attr,
                                          int64_t n, int64_t row) {
    bool ok = p.nterms >= 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (t < p.nterms) {
            int32_t a = attr[(int64_t)p.col[t] * n + row];
            ok = ok && (a >= p.lo[t]) && (a <= p.hi[t]);
        }
    }
    return ok;
}

// ------------------------------------------------------- LDS bitonic sort
// Sort nseg independent segments of M keys (M a power of two) stored back
// to back in LDS, ascending.  Every thread of the block must call it.
template <typename K>
__device__ void lds_bitonic_sort(K *a, int nseg, int M, int tid, int nthr) {
    const int half = M >> 1;
    const int lgh = __ffs(half) - 1;
    const int total = nseg * half;
    for (int size = 2; size <= M; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int lgs = __ffs(stride) - 1;
            for (int p = tid; p < total; p += nthr) {
                int seg = p >> lgh, pi = p & (half - 1);
                int i = ((pi >> lgs) << (lgs + 1)) + (pi & (stride - 1));
                int j = i + stride;
                bool up = (i & size) == 0;
                K *s = a + (size_t)seg * M;
                K x = s[i], y = s[j];
                bool sw = up ? KeyOps<K>::less(y, x) : KeyOps<K>::less(x, y);
                if (sw) {
                    s[i] = y;
                    s[j] = x;
                }
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------ LDS top-k lists
// Per query: keys[0, Kp) is the current sorted list (only the first K are
// kept), keys[Kp, Kp+CB) is an append buffer; thr = K-th smallest kept key
// (KEY_INF while fewer than K are known).  A candidate is appended only when
// it is below thr, so after the list fills up insertions become rare.
template <typename K>
struct TopkLds {
    K *keys;      // [nq][Kp + CB]
    int *cnt;     // [nq]
    K *thr;       // [nq]
    int nq, Kkeep, Kp, CB;

    __device__ int M() const { return Kp + CB; }

    __device__ void init(int tid, int nthr) {
        for (int i = tid; i < nq * M(); i += nthr) keys[i] = KeyOps<K>::inf();
        for (int b = tid; b < nq; b += nthr) {
            cnt[b] = 0;
            thr[b] = KeyOps<K>::inf();
        }
        __syncthreads();
    }

    // Called by one thread; the buffer must have room (see need_flush).
    __device__ void push(int b, const K &key) {
        if (KeyOps<K>::less(key, thr[b])) {
            int s = atomicAdd(&cnt[b], 1);
            keys[(size_t)b * M() + Kp + s] = key;
        }
    }

    // Block-uniform: true if some buffer holds more than CB - room keys.
    __device__ bool need_flush(int room) const {
        bool f = false;
        for (int b = 0; b < nq; ++b) f = f || (cnt[b] > CB - room);
        return f;
    }

    // Merge every buffer into its list.  All threads must call it.
    __device__ void flush(int tid, int nthr) {
        for (int p = tid; p < nq * CB; p += nthr) {
            int b = p / CB, i = p - b * CB;
            if (i >= cnt[b]) keys[(size_t)b * M() + Kp + i] = KeyOps<K>::inf();
        }
        __syncthreads();
        lds_bitonic_sort<K>(keys, nq, M(), tid, nthr);
        for (int p = tid; p < nq * (Kp - Kkeep); p += nthr) {
            int b = p / (Kp - Kkeep), i = p - b * (Kp - Kkeep);
            keys[(size_t)b * M() + Kkeep + i] = KeyOps<K>::inf();
        }
        __syncthreads();
        for (int b = tid; b < nq; b += nthr) {
            thr[b] = keys[(size_t)b * M() + Kkeep - 1];
            cnt[b] = 0;
        }
        __syncthreads();
    }
};

// ---------------------------------------- stored row element decoding
// Elements of one 16-byte load of a stored row, widened exactly to float.
template <int STORE>
struct Elem;
template <>
struct Elem<VRS_F32> {
    static constexpr int V = 4;      // elements per 16-byte load
    __device__ static void decode(const uint4 &w, float *x) {
        x[0] = __uint_as_float(w.x);
        x[1] = __uint_as_float(w.y);
        x[2] = __uint_as_float(w.z);
        x[3] = __uint_as_float(w.w);
    }
};
template <>
struct Elem<VRS_BF16> {
    static constexpr int V = 8;
    __device__ static void decode(const uint4 &w, float *x) {
        const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            x[2 * i] = __uint_as_float(v[i] << 16);
            x[2 * i + 1] = __uint_as_float(v[i] & 0xffff0000u);
        }
    }
};
template <>
struct Elem<VRS_FP8E4M3> {
    static constexpr int V = 16;
    __device__ static void decode(const uint4 &w, float *x) {
        const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) x[4 * i + j] = e4m3_to_f32((v[i] >> (8 * j)) & 0xffu);
    }
};

__host__ __device__ inline int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace vrs

namespace vrs {

// The K-th smallest (1 <= K <= H) of H values spread over the T threads of
// a workgroup (value i in thread i % T, slot i / T of v), by an 8-bit radix
// select: each pass counts the values that share the digits fixed so far
// by their next digit and keeps the digit whose bucket holds the K-th.
// Every thread returns the same value.
template <int S, int T>
__device__ uint32_t block_kth_u32(const uint32_t (&v)[S], int H, int K, uint32_t *hist,
                                  uint32_t *sel) {
    const int tid = threadIdx.x;
    uint32_t prefix = 0, mask = 0, kk = (uint32_t)K;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int i = tid; i < 256; i += T) hist[i] = 0;
        __syncthreads();
#pragma unroll
        for (int e = 0; e < S; ++e) {
            // all-ones values (the distance bits of an empty key, often most
            // of the inputs) are counted per wave: one atomic instead of one
            // per lane on the same bin
            const bool act = e * T + tid < H && (v[e] & mask) == prefix;
            const bool ones = act && v[e] == 0xffffffffu;
            const uint64_t bo = __ballot(ones);
            if (act && !ones) atomicAdd(&hist[(v[e] >> shift) & 255u], 1u);
            if ((tid & 63) == 0 && bo != 0ull) atomicAdd(&hist[255], (uint32_t)__popcll(bo));
        }
        __syncthreads();
        if (tid < 64) {
            uint32_t c[4], sum = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                c[e] = hist[tid * 4 + e];
                sum += c[e];
            }
            uint32_t incl = sum;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(incl, o);
                if (tid >= o) incl += t;
            }
            uint32_t run = incl - sum;
            if (run < kk && kk <= incl) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (run < kk && kk <= run + c[e]) {
                        sel[0] = prefix | ((uint32_t)(tid * 4 + e) << shift);
                        sel[1] = kk - run;
                    }
                    run += c[e];
                }
            }
        }
        __syncthreads();
        prefix = sel[0];
        kk = sel[1];
        mask |= 255u << shift;
    }
    return prefix;
}

// ------------------------------------------------- wave-level bitonic sort
// 64*E keys held E per lane (element index lane*E + e), sorted ascending by
// one wave without LDS or barriers: strides below E are swaps inside a lane,
// larger strides exchange with lane ^ (stride / E) through cross-lane moves.
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = __shfl_xor(lo, m);
    hi = __shfl_xor(hi, m);
    return ((uint64_t)hi << 32) | lo;
}

template <int E>
__device__ __forceinline__ void wave_sort_u64(uint64_t (&v)[E]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int size = 2; size <= 64 * E; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride < E) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if ((e & stride) == 0) {
                        const int i = lane * E + e;
                        const bool up = (i & size) == 0;
                        uint64_t x = v[e], y = v[e + stride];
                        const bool sw = up ? (y < x) : (x < y);
                        v[e] = sw ? y : x;
                        v[e + stride] = sw ? x : y;
                    }
                }
            } else {
                const int ls = stride / E;
                const bool lower = (lane & ls) == 0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int i = lane * E + e;
                    const bool up = (i & size) == 0;
                    const uint64_t p = shfl_xor_u64(v[e], ls);
                    const bool take_min = (lower == up);
                    v[e] = take_min ? (p < v[e] ? p : v[e]) : (p > v[e] ? p : v[e]);
                }
            }
        }
    }
}

}  // namespace vrs
