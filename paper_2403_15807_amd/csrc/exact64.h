// exact64.h -- the exact FP64 distance of the definition (Section 3, eq. 3,
// with the distance of the library's header): coordinates in ascending
// order, one fused multiply-add each, accumulator from +0.0; IP applies the
// FP8 row scale to the finished sum; zero is returned as +0.0.
//
// Two forms share the decoders below: exact_dist (one row, one thread) and
// exact64_wave (64 rows, one per lane of a wave, rows staged through the
// wave's own LDS area in 128-byte column chunks so that the loads stay
// coalesced).  Both evaluate the same chain, so any two kernels that score a
// (query, row) pair with them produce the same FP64 value.
#pragma once

#include "internal.h"

namespace vrs {

template <int STORE>
__device__ __forceinline__ void decode16(const uint4 &w, float *x);
template <>
__device__ __forceinline__ void decode16<VRS_F32>(const uint4 &w, float *x) {
    x[0] = __uint_as_float(w.x);
    x[1] = __uint_as_float(w.y);
    x[2] = __uint_as_float(w.z);
    x[3] = __uint_as_float(w.w);
}
template <>
__device__ __forceinline__ void decode16<VRS_BF16>(const uint4 &w, float *x) {
    const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        x[2 * i] = __uint_as_float(v[i] << 16);
        x[2 * i + 1] = __uint_as_float(v[i] & 0xffff0000u);
    }
}
// An e4m3fn code's 7 magnitude bits, placed as the top of an f32 exponent
// and mantissa field (a normal or subnormal f32), times 2^(127-7) give its
// value exactly: normal codes stay normal, subnormal codes m * 2^-9 come
// from subnormal f32 inputs, which these kernels keep (FP32 denormals are
// not flushed).  Four instructions instead of a branch on the exponent.
__device__ __forceinline__ float e4m3_value(uint32_t c) {
    const float mag = __uint_as_float((c & 0x7fu) << 20) * 0x1p120f;
    return __uint_as_float(__float_as_uint(mag) | ((c & 0x80u) << 24));
}
template <>
__device__ __forceinline__ void decode16<VRS_FP8E4M3>(const uint4 &w, float *x) {
    const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) x[4 * i + j] = e4m3_value((v[i] >> (8 * j)) & 0xffu);
}

// One row by one thread.  The row is read in 16-byte blocks up to the padded
// width dp; `qrow` holds the query padded with zeros to dp, and a padded
// coordinate adds an exact zero (+0 + +0 or acc + 0), so the value equals
// the sum over the first d coordinates.
template <int STORE, int METRIC>
__device__ double exact_dist(const void *rows, const float *scale, int64_t row, int dp,
                             const float *qrow /* dp floats, zero padded */) {
    constexpr int V = STORE == VRS_F32 ? 4 : (STORE == VRS_BF16 ? 8 : 16);
    constexpr int EB = 16 / V;
    const uint4 *p = (const uint4 *)((const char *)rows + row * (int64_t)dp * EB);
    const int nb = dp / V;
    const double sc = (STORE == VRS_FP8E4M3) ? (double)scale[row] : 1.0;
    double acc = 0.0;
    for (int c = 0; c < nb; c += 2) {
        uint4 w0 = p[c];
        uint4 w1 = (c + 1 < nb) ? p[c + 1] : make_uint4(0, 0, 0, 0);
        float x[2 * V];
        decode16<STORE>(w0, x);
        decode16<STORE>(w1, x + V);
        const int jn = min(2 * V, dp - c * V);
        for (int j = 0; j < jn; ++j) {
            const double qj = (double)qrow[c * V + j];
            if (METRIC == VRS_L2SQ) {
                double t = qj - sc * (double)x[j];
                acc = fma(t, t, acc);
            } else {
                acc = fma(qj, (double)x[j], acc);
            }
        }
    }
    if (METRIC == VRS_IP) acc = -(sc * acc);
    return acc == 0.0 ? 0.0 : acc;
}

// ---------------------------------------------------- 64 rows, one per lane
constexpr int X64_CHUNK = 128;                   // bytes of a row staged per step
constexpr int X64_STRIDE = X64_CHUNK / 16 + 1;   // 16-byte slots per staged row (one pad slot)
constexpr size_t X64_WAVE_LDS = (size_t)64 * X64_STRIDE * 16;  // staging bytes per wave
typedef unsigned int x64_u32x4 __attribute__((ext_vector_type(4)));

// Exact distance of `row` (this lane's row; a lane with has == false passes
// any valid row, e.g. 0, and ignores the result) to the query `qd` (FP64,
// zero padded to dp, in LDS).  `stage` = this wave's X64_WAVE_LDS bytes of
// LDS, 16-byte aligned.  Whole wave; rows are whole 128-byte blocks (dp
// padded accordingly).  The wave stages its 64 rows one 128-byte column
// chunk at a time (eight lanes per row chunk, two chunks in flight in
// registers); every lane then runs its chain over its row's chunk.  The LDS
// area is the wave's own and a wave's LDS accesses complete in program
// order, so a chunk is written only after every lane has read the one
// before it.
template <int STORE, int METRIC>
__device__ double exact64_wave(const void *rows, const float *scale, int row, bool has,
                               const double *qd, int dp, x64_u32x4 *stage) {
    constexpr int V = STORE == VRS_F32 ? 4 : (STORE == VRS_BF16 ? 8 : 16);  // elements per 16 B
    constexpr int EB = 16 / V;
    constexpr int SLOTS = X64_CHUNK / 16;
    constexpr int CE = X64_CHUNK / EB;  // coordinates per chunk
    const int lane = threadIdx.x & 63;
    const int nch = dp * EB / X64_CHUNK;
    const int64_t row_bytes = (int64_t)dp * EB;
    const double sc = (STORE == VRS_FP8E4M3 && has) ? (double)scale[row] : 1.0;
    // the rows this lane stages: i * 8 + lane / 8, 16-byte slot lane % 8
    const char *src[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int r = __shfl(row, i * 8 + (lane >> 3));
        src[i] = (const char *)rows + (int64_t)r * row_bytes + (lane & 7) * 16;
    }
    x64_u32x4 *dst = stage + (lane >> 3) * X64_STRIDE + (lane & 7);
    const x64_u32x4 *mine = stage + lane * X64_STRIDE;
    x64_u32x4 wa[8], wb[8];
    auto load = [&](x64_u32x4(&w)[8], int c) {
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] = *(const x64_u32x4 *)(src[i] + (int64_t)c * X64_CHUNK);
    };
    auto put = [&](const x64_u32x4(&w)[8]) {
#pragma unroll
        for (int i = 0; i < 8; ++i) dst[i * 8 * X64_STRIDE] = w[i];
    };
    double acc = 0.0;
    auto chain = [&](int c) {
#pragma unroll
        for (int u = 0; u < SLOTS; ++u) {
            const x64_u32x4 w = mine[u];
            float x[V];
            decode16<STORE>(make_uint4(w.x, w.y, w.z, w.w), x);
            const double *qq = qd + c * CE + u * V;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if (METRIC == VRS_L2SQ) {
                    const double tv = qq[v] - sc * (double)x[v];
                    acc = fma(tv, tv, acc);
                } else {
                    acc = fma(qq[v], (double)x[v], acc);
                }
            }
        }
    };
    // wa holds the even chunks, wb the odd ones
    load(wa, 0);
    if (nch > 1) load(wb, 1);
    for (int c = 0; c < nch; c += 2) {
        put(wa);
        if (c + 2 < nch) load(wa, c + 2);
        chain(c);
        if (c + 1 >= nch) break;
        put(wb);
        if (c + 3 < nch) load(wb, c + 3);
        chain(c + 1);
    }
    if (METRIC == VRS_IP) acc = -(sc * acc);
    return acc == 0.0 ? 0.0 : acc;
}

}  // namespace vrs
