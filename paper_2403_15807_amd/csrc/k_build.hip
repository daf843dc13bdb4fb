// k_build.hip -- table build: optional row normalisation (cosine metric,
// Section 3.1), storage encoding (float32 / bfloat16 / FP8 e4m3fn with a
// per-row scale), per-row squared norms for the screening kernels, the
// largest row norm for the certificate's error bound, a finiteness check,
// and per-column attribute histograms for selectivity estimates.
#include "internal.h"

namespace vrs {

// float32 -> bfloat16 bits, round to nearest-even (finite inputs; overflow
// becomes infinity, which the finiteness check then rejects).
__device__ __forceinline__ uint32_t bf16_rne_bits(float f) {
    uint32_t u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// FP64 value -> OCP e4m3fn code, round to nearest-even, saturating at 448;
// the sign bit follows the sign of v.
__device__ __forceinline__ uint32_t e4m3_rne(double v) {
    uint32_t sign = signbit(v) ? 0x80u : 0u;
    double a = fabs(v);
    if (!(a < 448.0)) return sign | 0x7eu;
    if (a < 0.015625) {                 // below 2^-6: spacing 2^-9
        double m = rint(a * 512.0);     // 0..8; 8 is the smallest normal (code 8)
        return sign | (uint32_t)m;
    }
    int e;
    double f = frexp(a, &e);            // a = f * 2^e, f in [0.5, 1)
    double m = rint((2.0 * f - 1.0) * 8.0);
    int ue = e - 1;
    if (m == 8.0) {
        m = 0.0;
        ue += 1;
    }
    return sign | (uint32_t)(((ue + 7) << 3) | (int)m);
}

template <int STORE>
__global__ __launch_bounds__(256) void build_rows_kernel(const float *__restrict__ vec, int64_t n,
                                                         int d, int dp, int normalize,
                                                         void *__restrict__ rows,
                                                         float *__restrict__ scale,
                                                         float *__restrict__ norm2,
                                                         unsigned long long *max_norm_bits,
                                                         int *bad) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *x = vec + i * (int64_t)d;
    double nrm = 0.0;
    if (normalize) {
        double acc = 0.0;
        for (int j = 0; j < d; ++j) acc = fma((double)x[j], (double)x[j], acc);
        nrm = sqrt(acc);
    }
    auto val = [&](int j) -> float {
        return (normalize && nrm != 0.0) ? (float)((double)x[j] / nrm) : x[j];
    };
    bool finite = true;
    float s = 1.0f;
    if (STORE == VRS_FP8E4M3) {
        float m = 0.0f;
        for (int j = 0; j < d; ++j) {
            float v = val(j);
            finite = finite && isfinite(v);
            m = fmaxf(m, fabsf(v));
        }
        s = (m == 0.0f) ? 1.0f : m / 448.0f;
        scale[i] = s;
    }
    double sq = 0.0;
    for (int j = 0; j < dp; ++j) {
        double stored = 0.0;
        if (STORE == VRS_F32) {
            float v = j < d ? val(j) : 0.0f;
            finite = finite && isfinite(v);
            ((float *)rows)[i * dp + j] = v;
            stored = v;
        } else if (STORE == VRS_BF16) {
            uint32_t c = 0;
            if (j < d) {
                float v = val(j);
                finite = finite && isfinite(v);
                c = bf16_rne_bits(v);
            }
            float st = bf16_to_f32(c);
            finite = finite && isfinite(st);
            ((uint16_t *)rows)[i * dp + j] = (uint16_t)c;
            stored = st;
        } else {
            uint32_t c = 0;
            if (j < d) c = e4m3_rne((double)val(j) / (double)s);
            ((uint8_t *)rows)[i * dp + j] = (uint8_t)c;
            stored = (double)s * (double)e4m3_to_f32(c);
        }
        sq = fma(stored, stored, sq);
    }
    norm2[i] = (float)sq;
    double rn = sqrt(sq) * (1.0 + 0x1p-40);  // rounded up: used only as a bound
    if (finite)
        atomicMax(max_norm_bits, (unsigned long long)__double_as_longlong(rn));
    else
        atomicOr(bad, 1);
}

hipError_t launch_build_rows(const float *vec, int64_t n, int32_t d, int32_t dp, vrs_dtype store,
                             int normalize, void *rows, float *scale, float *norm2,
                             unsigned long long *max_norm_bits, int *bad, hipStream_t s) {
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (store) {
    case VRS_F32:
        build_rows_kernel<VRS_F32><<<grid, block, 0, s>>>(vec, n, d, dp, normalize, rows, scale,
                                                          norm2, max_norm_bits, bad);
        break;
    case VRS_BF16:
        build_rows_kernel<VRS_BF16><<<grid, block, 0, s>>>(vec, n, d, dp, normalize, rows, scale,
                                                           norm2, max_norm_bits, bad);
        break;
    default:
        build_rows_kernel<VRS_FP8E4M3><<<grid, block, 0, s>>>(vec, n, d, dp, normalize, rows,
                                                              scale, norm2, max_norm_bits, bad);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ histograms
__global__ __launch_bounds__(256) void attr_minmax_kernel(const int32_t *__restrict__ attr,
                                                          int64_t n, int32_t *amin,
                                                          int32_t *amax) {
    const int c = blockIdx.y;
    const int32_t *col = attr + (int64_t)c * n;
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t a = col[i];
        lo = min(lo, a);
        hi = max(hi, a);
    }
    __shared__ int32_t slo[256], shi[256];
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            slo[threadIdx.x] = min(slo[threadIdx.x], slo[threadIdx.x + w]);
            shi[threadIdx.x] = max(shi[threadIdx.x], shi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMin(&amin[c], slo[0]);
        atomicMax(&amax[c], shi[0]);
    }
}

__global__ __launch_bounds__(256) void attr_hist_kernel(const int32_t *__restrict__ attr, int64_t n,
                                                        const int32_t *amin, const int32_t *amax,
                                                        uint32_t *hist) {
    const int c = blockIdx.y;
    const int32_t *col = attr + (int64_t)c * n;
    __shared__ uint32_t h[HIST_BINS];
    for (int b = threadIdx.x; b < HIST_BINS; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const int64_t lo = amin[c], span = (int64_t)amax[c] - lo + 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t b = ((int64_t)col[i] - lo) * HIST_BINS / span;
        atomicAdd(&h[b], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < HIST_BINS; b += blockDim.x)
        if (h[b]) atomicAdd(&hist[(int64_t)c * HIST_BINS + b], h[b]);
}

__global__ void attr_init_kernel(int32_t *amin, int32_t *amax, uint32_t *hist, int n_attr) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_attr) {
        amin[t] = INT32_MAX;
        amax[t] = INT32_MIN;
    }
    if (t < n_attr * HIST_BINS) hist[t] = 0;
}

hipError_t launch_attr_stats(const int32_t *attr, int64_t n, int32_t n_attr, int32_t *amin,
                             int32_t *amax, uint32_t *hist, hipStream_t s) {
    if (n_attr == 0) return hipSuccess;
    int tot = n_attr * HIST_BINS;
    attr_init_kernel<<<(tot + 255) / 256, 256, 0, s>>>(amin, amax, hist, n_attr);
    int gx = (int)std::min<int64_t>(1024, (n + 255) / 256);
    attr_minmax_kernel<<<dim3(gx, n_attr), 256, 0, s>>>(attr, n, amin, amax);
    attr_hist_kernel<<<dim3(gx, n_attr), 256, 0, s>>>(attr, n, amin, amax, hist);
    return hipGetLastError();
}

// ------------------------------------------------- stored rows as queries
// Rows [i0, i0 + count) of a table as float32 vectors [count][d]: float32
// and bfloat16 values exactly, an FP8 value (row scale times the code's
// value) rounded to the nearest float32 (one float multiply of two exact
// operands).  The queries of a vector join.
__global__ __launch_bounds__(256) void rows_to_f32_kernel(const void *__restrict__ rows,
                                                          const float *__restrict__ scale,
                                                          int store, int d, int dp, int64_t i0,
                                                          int64_t count, float *__restrict__ out) {
    const int64_t total = count * d;
    for (int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t r = e / d, j = e - r * d, row = i0 + r;
        float v;
        if (store == VRS_F32) {
            v = ((const float *)rows)[row * dp + j];
        } else if (store == VRS_BF16) {
            v = __uint_as_float((uint32_t)((const uint16_t *)rows)[row * dp + j] << 16);
        } else {
            const uint32_t c = ((const uint8_t *)rows)[row * dp + j];
            const float mag = __uint_as_float((c & 0x7fu) << 20) * 0x1p120f;  // exact (see the rerank)
            v = scale[row] * __uint_as_float(__float_as_uint(mag) | ((c & 0x80u) << 24));
        }
        out[e] = v;
    }
}

hipError_t launch_rows_to_f32(const vrs_table_s *t, int64_t i0, int64_t count, float *out, hipStream_t s) {
    const int64_t total = count * t->d;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
    rows_to_f32_kernel<<<grid, 256, 0, s>>>(t->rows, t->scale, (int)t->store, t->d, t->dp, i0, count, out);
    return hipGetLastError();
}

}  // namespace vrs
