// k_mlp.hip -- the access-path chooser's network on the GPU: a
// 6 -> 64 -> 64 -> 16 multilayer perceptron with ReLU, FP32, trained with a
// masked mean-squared error on measured log-times and Adam.
//
// Parameter block (floats, in this order): W1[6][64], b1[64], W2[64][64],
// b2[64], W3[64][16], b3[16]; a layer computes h_out[j] = b[j] +
// sum_i h_in[i] * W[i][j] (inputs in ascending i).
//
// Forward: one thread per sample (the whole network is 5.4k multiply-adds).
// Backward: one thread per sample for the error signals, then one thread per
// parameter summing its gradient over the samples in ascending order -- no
// atomics, so gradients are deterministic.
#include "internal.h"

namespace vrs {

namespace {

constexpr int NI = VRS_MLP_IN, NH = VRS_MLP_HIDDEN, NO = VRS_MLP_OUT;
constexpr int OW1 = 0, OB1 = OW1 + NI * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH * NO, NPARAM = OB3 + NO;
static_assert(NPARAM == VRS_MLP_PARAMS, "parameter count");

// act per sample: h1[64] | h2[64] (post-ReLU) ; y [16] separately
__global__ __launch_bounds__(256) void mlp_fwd_kernel(const float *__restrict__ p,
                                                      const float *__restrict__ x, int nb,
                                                      float *__restrict__ y,
                                                      float *__restrict__ act) {
    __shared__ float w[NPARAM];
    for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) w[i] = p[i];
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nb) return;
    float in[NI], h1[NH], h2[NH];
#pragma unroll
    for (int i = 0; i < NI; ++i) in[i] = x[(int64_t)s * NI + i];
    for (int j = 0; j < NH; ++j) {
        float a = w[OB1 + j];
#pragma unroll
        for (int i = 0; i < NI; ++i) a = fmaf(in[i], w[OW1 + i * NH + j], a);
        h1[j] = a > 0.0f ? a : 0.0f;
    }
    for (int j = 0; j < NH; ++j) {
        float a = w[OB2 + j];
        for (int i = 0; i < NH; ++i) a = fmaf(h1[i], w[OW2 + i * NH + j], a);
        h2[j] = a > 0.0f ? a : 0.0f;
    }
    for (int j = 0; j < NO; ++j) {
        float a = w[OB3 + j];
        for (int i = 0; i < NH; ++i) a = fmaf(h2[i], w[OW3 + i * NO + j], a);
        y[(int64_t)s * NO + j] = a;
    }
    if (act) {
        for (int j = 0; j < NH; ++j) act[(int64_t)s * 2 * NH + j] = h1[j];
        for (int j = 0; j < NH; ++j) act[(int64_t)s * 2 * NH + NH + j] = h2[j];
    }
}

// Error signals per sample: dy = 2 mask (y - t) / count, d2 = (dy W3^T) on
// active h2 units, d1 = (d2 W2^T) on active h1 units.  sig: dy[16] | d2[64] | d1[64].
__global__ __launch_bounds__(256) void mlp_sig_kernel(const float *__restrict__ p,
                                                      const float *__restrict__ y,
                                                      const float *__restrict__ act,
                                                      const float *__restrict__ t,
                                                      const uint8_t *__restrict__ mask, int nb,
                                                      float inv_count, float *__restrict__ sig,
                                                      float *__restrict__ sqerr) {
    __shared__ float w[NPARAM];
    for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) w[i] = p[i];
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nb) return;
    float dy[NO], d2[NH];
    float se = 0.0f;
    for (int j = 0; j < NO; ++j) {
        const int64_t o = (int64_t)s * NO + j;
        const float e = mask[o] ? (y[o] - t[o]) : 0.0f;
        se = fmaf(e, e, se);
        dy[j] = 2.0f * e * inv_count;
    }
    sqerr[s] = se;
    const float *h1 = act + (int64_t)s * 2 * NH, *h2 = h1 + NH;
    float *o = sig + (int64_t)s * (NO + 2 * NH);
    for (int j = 0; j < NO; ++j) o[j] = dy[j];
    for (int i = 0; i < NH; ++i) {
        float a = 0.0f;
        for (int j = 0; j < NO; ++j) a = fmaf(dy[j], w[OW3 + i * NO + j], a);
        d2[i] = h2[i] > 0.0f ? a : 0.0f;
        o[NO + i] = d2[i];
    }
    for (int i = 0; i < NH; ++i) {
        float a = 0.0f;
        for (int j = 0; j < NH; ++j) a = fmaf(d2[j], w[OW2 + i * NH + j], a);
        o[NO + NH + i] = h1[i] > 0.0f ? a : 0.0f;
    }
}

// One thread per parameter: its gradient summed over samples 0..nb-1.
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float *__restrict__ x,
                                                       const float *__restrict__ act,
                                                       const float *__restrict__ sig, int nb,
                                                       float *__restrict__ grad) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NPARAM) return;
    const int SG = NO + 2 * NH;
    float g = 0.0f;
    if (k < OB1) {            // W1[i][j] = sum x_i d1_j
        const int i = k / NH, j = k % NH;
        for (int s = 0; s < nb; ++s) g = fmaf(x[(int64_t)s * NI + i], sig[(int64_t)s * SG + NO + NH + j], g);
    } else if (k < OW2) {     // b1[j]
        const int j = k - OB1;
        for (int s = 0; s < nb; ++s) g += sig[(int64_t)s * SG + NO + NH + j];
    } else if (k < OB2) {     // W2[i][j] = sum h1_i d2_j
        const int i = (k - OW2) / NH, j = (k - OW2) % NH;
        for (int s = 0; s < nb; ++s) g = fmaf(act[(int64_t)s * 2 * NH + i], sig[(int64_t)s * SG + NO + j], g);
    } else if (k < OW3) {     // b2[j]
        const int j = k - OB2;
        for (int s = 0; s < nb; ++s) g += sig[(int64_t)s * SG + NO + j];
    } else if (k < OB3) {     // W3[i][j] = sum h2_i dy_j
        const int i = (k - OW3) / NO, j = (k - OW3) % NO;
        for (int s = 0; s < nb; ++s) g = fmaf(act[(int64_t)s * 2 * NH + NH + i], sig[(int64_t)s * SG + j], g);
    } else {                  // b3[j]
        const int j = k - OB3;
        for (int s = 0; s < nb; ++s) g += sig[(int64_t)s * SG + j];
    }
    grad[k] = g;
}

__global__ void mlp_adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                                float *__restrict__ m, float *__restrict__ v, int n, float lr,
                                float b1, float b2, float eps, float c1, float c2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float mh = mk / c1, vh = vk / c2;
    p[k] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void sum_kernel(const float *__restrict__ a, int n, float scale, float *__restrict__ out) {
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += a[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

}  // namespace

hipError_t launch_mlp_forward(const float *p, const float *x, int nb, float *y, float *act,
                              hipStream_t s) {
    mlp_fwd_kernel<<<(nb + 255) / 256, 256, 0, s>>>(p, x, nb, y, act);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float *p, const float *x, const float *y, const float *act,
                               const float *t, const uint8_t *mask, int nb, float inv_count,
                               float *sig, float *sqerr, float *grad, float *loss,
                               hipStream_t s) {
    mlp_sig_kernel<<<(nb + 255) / 256, 256, 0, s>>>(p, y, act, t, mask, nb, inv_count, sig, sqerr);
    mlp_grad_kernel<<<(NPARAM + 255) / 256, 256, 0, s>>>(x, act, sig, nb, grad);
    if (loss) sum_kernel<<<1, 256, 0, s>>>(sqerr, nb, inv_count, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *p, const float *g, float *m, float *v, int step, float lr,
                           float b1, float b2, float eps, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    mlp_adam_kernel<<<(NPARAM + 255) / 256, 256, 0, s>>>(p, g, m, v, NPARAM, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace vrs
